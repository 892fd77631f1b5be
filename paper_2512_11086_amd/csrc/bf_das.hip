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
//     s = B(p) + k * (E_tx + E_rx),   B = (2 z k - t0 fs),  k = fs / c,
// with B evaluated once per lane in FP64 and split into an integer part and
// an FP32 fraction, and the small excess paths E = d - z = rho^2 / (d + z)
// (exact rewriting of d - z without cancellation) in FP32.
//
// Apodization skip (Sec. VII-F): a trace is skipped wavefront-uniformly when
// no lane lies inside its receive aperture, tested on rho^2 against
// z^2 / (4 F#^2) (no cosine, no square root).  FORCES tests once per channel
// for all transmits, HERCULES per (row, column) element.
#include "bf_common.h"

namespace bf {

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
            // Catmull-Rom cubic Hermite in Horner form around p0.
            const float c1 = 0.5f * (p1 - pm);
            const float c2 = pm - 2.5f * p0 + 2.0f * p1 - 0.5f * p2;
            const float c3 = 0.5f * (p2 - pm) + 1.5f * (p0 - p1);
            return fmaf(t, fmaf(t, fmaf(t, c3, c2), c1), p0);
        }
    }
}

// FORCES: the transmit and receive excess paths separate.  The wavefront
// collects up to JG of its active channel rows (a row is active when some
// lane lies inside its receive aperture), computes each row's receive term
// and apodization once per lane, then sweeps the transmits: the transmit
// excess path (one square root and one reciprocal) is shared by the JG terms
// of that transmit.  Terms of one point are added in (row chunk, transmit,
// row) order.
constexpr int JG = 8;

template <int ET, int IP>
__device__ inline float das_forces_point(const DasArgs &a, const Lane &L, int jb, int je)
{
    const float kf = (float)a.k;
    float acc = 0.f;
    int j = jb;
    for (;;) {
        int rows[JG];
        int n = 0;
        for (; j < je && n < JG; ++j) {
            const float dxr = L.x - a.rx_c[j];
            if (__any(L.active && dxr * dxr < L.thr)) rows[n++] = j;
        }
        if (n == 0) break;
        float Rj[JG], aj[JG];
#pragma unroll
        for (int q = 0; q < JG; ++q) {
            Rj[q] = 0.f;
            aj[q] = 0.f;
            if (q < n) {
                const float dxr = L.x - a.rx_c[rows[q]];
                const float r2 = dxr * dxr;
                const bool act = L.active && r2 < L.thr;
                Rj[q] = fmaf(excess(r2, L.z, L.z2), kf, L.fB);
                aj[q] = act ? hann_u2(r2 * L.wsc) : 0.f;
            }
        }
        for (int i = 0; i < a.n_tx; ++i) {
            const float dxt = L.x - a.tx_x[i];
            const float T = kf * excess(dxt * dxt, L.z, L.z2);
#pragma unroll
            for (int q = 0; q < JG; ++q) {
                if (q < n && L.active) {
                    const void *tr = trace_ptr<ET>(a.e, (long)i * a.n_ch + rows[q], a.S);
                    acc = fmaf(aj[q], read_trace<ET, IP>(tr, a.S, L.nB, Rj[q] + T), acc);
                }
            }
        }
    }
    return acc;
}

// HERCULES: receive element (x_i, y_j, 0), plane-wave transmit (tof_tx = z/c,
// already inside B), radial apodization.
template <int ET, int IP>
__device__ inline float das_hercules_point(const DasArgs &a, const Lane &L, int jb, int je)
{
    const float kf = (float)a.k;
    float acc = 0.f;
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
                acc = fmaf(w, read_trace<ET, IP>(tr, a.S, L.nB, s), acc);
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
    float acc;
    if constexpr (MODE == 0)
        acc = das_forces_point<ET, IP>(a, L, jb, je);
    else
        acc = das_hercules_point<ET, IP>(a, L, jb, je);
    if (L.valid) {
        const float v = L.active ? acc : 0.f;
        if (a.groups > 1)
            a.part[(long)blockIdx.y * a.g.nx * a.g.ny * a.g.nz + L.out_idx] = v;
        else
            das_out(a)[L.out_idx] = v;
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
    const long n = (long)a.g.nx * a.g.ny * a.g.nz;
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
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_das(const DasArgs &a, int mode, int et, int ip, hipStream_t s)
{
    hipError_t err = mode == 0 ? launch_et<0>(a, et, ip, s) : launch_et<1>(a, et, ip, s);
    if (err != hipSuccess || a.groups <= 1) return err;
    return launch_sum_groups(a, s);
}

}  // namespace bf
