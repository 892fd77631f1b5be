// bf_das.hip -- delay-and-sum beamforming on gfx950 (Eq. 1, Eqs. 2-3,
// Sec. IV-B, Sec. VII-F).
//
// One lane per output point; a wavefront covers a small 3D tile of
// 2^lx x 2^ly x 2^lz points (z fastest across lanes), so the lanes' delays
// for one (transmit, channel) trace are close together and their sample reads
// fall in a few cache lines (the paper's small-tile dispatch, Sec. VII-F).
//
// Delay precision.  The sample position s = (tof - t0) fs reaches ~2000, where
// an FP32 ulp is 1.2e-4 samples; summed over thousands of traces that costs
// ~3e-5 relative image error.  The kernels therefore split
//     s = B(p) + k * (E_tx + E_rx),   B = ((T(p) + z) k - t0 fs),  k = fs / c,
// with T(p) the transmit path down to the point (z for plane waves and the
// separable modes, whose transmit excess goes into E_tx), B evaluated once per
// lane in FP64 and split into an integer part and an FP32 fraction, and the
// small excess paths E = d - z = rho^2 / (d + z) (exact rewriting of d - z
// without cancellation) in FP32.
//
// Apodization skip (Sec. VII-F): a trace is skipped wavefront-uniformly when
// no lane lies inside its receive aperture, tested on rho^2 against
// z^2 / (4 F#^2) (no cosine, no square root).  FORCES tests once per channel
// for all transmits, HERCULES per (row, column) element.
//
// IQ data (ET_CF32): the trace is read as (re, im) pairs with the same
// interpolator and each term is rotated by the carrier phase of its record
// time before it is added (complex accumulation).
#include "bf_common.h"

namespace bf {

// Catmull-Rom cubic Hermite in Horner form around p0, for real or complex taps.
__device__ inline float cr_eval(float t, float pm, float p0, float p1, float p2)
{
    const float c1 = 0.5f * (p1 - pm);
    const float c2 = pm - 2.5f * p0 + 2.0f * p1 - 0.5f * p2;
    const float c3 = 0.5f * (p2 - pm) + 1.5f * (p0 - p1);
    return fmaf(t, fmaf(t, fmaf(t, c3, c2), c1), p0);
}
__device__ inline float2 cr_eval(float t, float2 pm, float2 p0, float2 p1, float2 p2)
{
    return make_float2(cr_eval(t, pm.x, p0.x, p1.x, p2.x), cr_eval(t, pm.y, p0.y, p1.y, p2.y));
}

// Complex read of an IQ trace at nB + s; zero outside [0, S).
template <int IP>
__device__ inline float2 read_trace_cx(const void *tr, int S, int nB, float s)
{
    const float2 z = make_float2(0.f, 0.f);
    if constexpr (IP == IN_NEAREST) {
        const int n = nB + (int)floorf(s + 0.5f);
        return ((unsigned)n < (unsigned)S) ? load_c(tr, n) : z;
    } else {
        const float fl = floorf(s);
        const float t = s - fl;
        const int n = nB + (int)fl;
        if constexpr (IP == IN_LINEAR) {
            const float2 p0 = ((unsigned)n < (unsigned)S) ? load_c(tr, n) : z;
            const float2 p1 = ((unsigned)(n + 1) < (unsigned)S) ? load_c(tr, n + 1) : z;
            return make_float2(fmaf(t, p1.x - p0.x, p0.x), fmaf(t, p1.y - p0.y, p0.y));
        } else {
            float2 pm, p0, p1, p2;
            if (n >= 1 && n + 2 < S) {
                pm = load_c(tr, n - 1);
                p0 = load_c(tr, n);
                p1 = load_c(tr, n + 1);
                p2 = load_c(tr, n + 2);
            } else {
                pm = ((unsigned)(n - 1) < (unsigned)S) ? load_c(tr, n - 1) : z;
                p0 = ((unsigned)n < (unsigned)S) ? load_c(tr, n) : z;
                p1 = ((unsigned)(n + 1) < (unsigned)S) ? load_c(tr, n + 1) : z;
                p2 = ((unsigned)(n + 2) < (unsigned)S) ? load_c(tr, n + 2) : z;
            }
            return cr_eval(t, pm, p0, p1, p2);
        }
    }
}

// Read of trace `tr` at absolute sample position nB + s (s = small FP32
// offset); zero outside [0, S).
template <int ET, int IP>
__device__ inline float read_trace(const void *tr, int S, int nB, float s)
{
    if constexpr (IP == IN_NEAREST) {
        const int n = nB + (int)floorf(s + 0.5f);
        return ((unsigned)n < (unsigned)S) ? load_e<ET>(tr, n) : 0.f;
    } else {
        const float fl = floorf(s);
        const float t = s - fl;
        const int n = nB + (int)fl;
        if constexpr (IP == IN_LINEAR) {
            const float p0 = ((unsigned)n < (unsigned)S) ? load_e<ET>(tr, n) : 0.f;
            const float p1 = ((unsigned)(n + 1) < (unsigned)S) ? load_e<ET>(tr, n + 1) : 0.f;
            return fmaf(t, p1 - p0, p0);
        } else {
            float pm, p0, p1, p2;
            if (n >= 1 && n + 2 < S) {
                pm = load_e<ET>(tr, n - 1);
                p0 = load_e<ET>(tr, n);
                p1 = load_e<ET>(tr, n + 1);
                p2 = load_e<ET>(tr, n + 2);
            } else {
                pm = ((unsigned)(n - 1) < (unsigned)S) ? load_e<ET>(tr, n - 1) : 0.f;
                p0 = ((unsigned)n < (unsigned)S) ? load_e<ET>(tr, n) : 0.f;
                p1 = ((unsigned)(n + 1) < (unsigned)S) ? load_e<ET>(tr, n + 1) : 0.f;
                p2 = ((unsigned)(n + 2) < (unsigned)S) ? load_e<ET>(tr, n + 2) : 0.f;
            }
            return cr_eval(t, pm, p0, p1, p2);
        }
    }
}

// acc += w * read(e_ij at nB + s), rotated for IQ data.
template <int ET, int IP>
__device__ inline void add_term(const DasArgs &a, const Lane &L, const void *tr, float w, float s,
                                float2 &acc)
{
    if constexpr (ET == ET_CF32)
        rotate_acc(read_trace_cx<IP>(tr, a.S, L.nB, s), w, fmaf(a.rot, s, L.ph0), acc);
    else
        acc.x = fmaf(w, read_trace<ET, IP>(tr, a.S, L.nB, s), acc.x);
}

// FORCES, TPW, VLS: the transmit and receive excess paths separate.  The
// wavefront collects up to JG of its active receivers (a receiver is active
// when some lane lies inside its receive aperture), computes each one's
// receive term and apodization once per lane, then sweeps the transmits: the
// transmit excess path (tx_excess) is shared by the JG terms of that
// transmit.  Terms of one point are added in (receiver chunk, transmit,
// receiver) order.
constexpr int JG = 8;

template <int MODE, int ET, int IP>
__device__ inline float2 das_separable_point(const DasArgs &a, const Lane &L, int jb, int je)
{
    const float xr = rx_coord<MODE>(L.x, L.y);
    const float kf = (float)a.k;
    float2 acc = make_float2(0.f, 0.f);
    int j = jb;
    for (;;) {
        int rows[JG];
        int n = 0;
        for (; j < je && n < JG; ++j) {
            const float dxr = xr - a.rx_c[j];
            if (__any(L.active && dxr * dxr < L.thr)) rows[n++] = j;
        }
        if (n == 0) break;
        float Rj[JG], aj[JG];
#pragma unroll
        for (int q = 0; q < JG; ++q) {
            Rj[q] = 0.f;
            aj[q] = 0.f;
            if (q < n) {
                const float dxr = xr - a.rx_c[rows[q]];
                const float r2 = dxr * dxr;
                const bool act = L.active && r2 < L.thr;
                Rj[q] = fmaf(excess(r2, L.z, L.z2), kf, L.fB);
                aj[q] = act ? hann_u2(r2 * L.wsc) : 0.f;
            }
        }
        for (int i = 0; i < a.n_tx; ++i) {
            const float T = kf * tx_excess<MODE>(a, L.x, L.z, L.z2, i);
#pragma unroll
            for (int q = 0; q < JG; ++q) {
                if (q < n && L.active) {
                    const void *tr = trace_ptr<ET>(a.e, (long)i * a.n_ch + rows[q], a.S);
                    add_term<ET, IP>(a, L, tr, aj[q], Rj[q] + T, acc);
                }
            }
        }
    }
    return acc;
}

// HERCULES: receive element (x_i, y_j, 0), transmit path of the point (plane
// or diverging wave, one per point: already inside B), radial apodization.
template <int ET, int IP>
__device__ inline float2 das_hercules_point(const DasArgs &a, const Lane &L, int jb, int je)
{
    const float kf = (float)a.k;
    float2 acc = make_float2(0.f, 0.f);
    for (int j = jb; j < je; ++j) {
        const float dy = L.y - a.rx_c[j];
        const float dy2 = dy * dy;
        if (!__any(L.active && dy2 < L.thr)) continue;
        for (int i = 0; i < a.n_tx; ++i) {
            const float dx = L.x - a.tx_x[i];
            const float rho2 = fmaf(dx, dx, dy2);
            const bool act = L.active && rho2 < L.thr;
            if (!__any(act)) continue;
            if (act) {
                const float s = fmaf(excess(rho2, L.z, L.z2), kf, L.fB);
                const float w = hann_u2(rho2 * L.wsc);
                const void *tr = trace_ptr<ET>(a.e, (long)i * a.n_ch + j, a.S);
                add_term<ET, IP>(a, L, tr, w, s, acc);
            }
        }
    }
    return acc;
}

// grid: ceil(n_waves / 4) blocks of 256 threads.
template <int MODE, int ET, int IP>
__global__ __launch_bounds__(256) void das_kernel(DasArgs a)
{
    const int wave_id = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wave_id >= a.n_waves) return;
    const Lane L = lane_setup(a, wave_id, threadIdx.x & 63);
    int jb, je;
    group_rows(a.n_ch, blockIdx.y, a.groups, &jb, &je);
    float2 acc;
    if constexpr (MODE == MODE_HERCULES)
        acc = das_hercules_point<ET, IP>(a, L, jb, je);
    else
        acc = das_separable_point<MODE, ET, IP>(a, L, jb, je);
    if (L.valid) {
        if (!L.active) acc = make_float2(0.f, 0.f);
        const long npts = (long)a.g.nx * a.g.ny * a.g.nz;
        float *dst = a.groups > 1 ? a.part + (long)blockIdx.y * npts * (ET == ET_CF32 ? 2 : 1)
                                  : das_out(a);
        if constexpr (ET == ET_CF32)
            reinterpret_cast<float2 *>(dst)[L.out_idx] = acc;
        else
            dst[L.out_idx] = acc.x;
    }
}

// Sum of the channel-group partial images in group order (deterministic).
__global__ __launch_bounds__(256) void sum_groups_kernel(const float *part, float *out_direct,
                                                         float *const *out_ref, long n, int G)
{
    float *out = out_ref ? *out_ref : out_direct;
    for (long q = (long)blockIdx.x * 256 + threadIdx.x; q < n; q += (long)gridDim.x * 256) {
        float s = 0.f;
        for (int g = 0; g < G; ++g) s += part[(long)g * n + q];
        out[q] = s;
    }
}

hipError_t launch_sum_groups(const DasArgs &a, hipStream_t s)
{
    const long n = (long)a.g.nx * a.g.ny * a.g.nz * (a.cx ? 2 : 1);
    long blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(sum_groups_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a.part, a.out,
                       a.out_ref, n, a.groups);
    return hipGetLastError();
}

template <int MODE, int ET>
static hipError_t launch_ip(const DasArgs &a, int ip, hipStream_t s)
{
    dim3 grid((a.n_waves + 3) / 4, a.groups);
    switch (ip) {
        case IN_NEAREST: hipLaunchKernelGGL((das_kernel<MODE, ET, IN_NEAREST>), grid, dim3(256), 0, s, a); break;
        case IN_LINEAR: hipLaunchKernelGGL((das_kernel<MODE, ET, IN_LINEAR>), grid, dim3(256), 0, s, a); break;
        case IN_CUBIC: hipLaunchKernelGGL((das_kernel<MODE, ET, IN_CUBIC>), grid, dim3(256), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int MODE>
static hipError_t launch_et(const DasArgs &a, int et, int ip, hipStream_t s)
{
    switch (et) {
        case ET_F32: return launch_ip<MODE, ET_F32>(a, ip, s);
        case ET_BF16: return launch_ip<MODE, ET_BF16>(a, ip, s);
        case ET_I32: return launch_ip<MODE, ET_I32>(a, ip, s);
        case ET_CF32: return launch_ip<MODE, ET_CF32>(a, ip, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_das(const DasArgs &a, int mode, int et, int ip, hipStream_t s)
{
    hipError_t err;
    switch (mode) {
        case MODE_FORCES: err = launch_et<MODE_FORCES>(a, et, ip, s); break;
        case MODE_HERCULES: err = launch_et<MODE_HERCULES>(a, et, ip, s); break;
        case MODE_TPW: err = launch_et<MODE_TPW>(a, et, ip, s); break;
        case MODE_VLS: err = launch_et<MODE_VLS>(a, et, ip, s); break;
        default: return hipErrorInvalidValue;
    }
    if (err != hipSuccess || a.groups <= 1) return err;
    return launch_sum_groups(a, s);
}

}  // namespace bf
