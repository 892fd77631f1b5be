// bf_adjoint.hip -- adjoint of DAS and the image-sharpness loss.
//
// DAS is linear in the decoded data e for a fixed sound speed c, so its
// adjoint scatters dL/d(out) back along the same delays and interpolation
// weights.  The sound speed enters only through the delay:
//   s = (tof - t0) fs,  tof = path / c   =>   ds/dc = -tof fs / c
// and the apodization does not depend on c, so
//   dL/dc = sum_p G(p) sum_ij a(p,i,j) v'_ij(s) ds/dc.
// The cubic Hermite read has a continuous derivative (Sec. IV-B), which is
// what makes this gradient usable for sound-speed autofocus.
#include "bf_common.h"

namespace bf {

// One (point, trace) term of the adjoint.  ga = G(p) * a(p,i,j).
// Adds ga * w_k(t) to grad_e taps (if GE) and returns a * v'(s) (if GC).
template <int ET, int IP, bool GE, bool GC>
__device__ inline float adjoint_term(const void *tr, float *ge, int S, int nB, float s, float ga,
                                     float a_w)
{
    if constexpr (IP == IN_NEAREST) {
        if constexpr (GE) {
            const int n = nB + (int)floorf(s + 0.5f);
            if ((unsigned)n < (unsigned)S) atomicAdd(ge + n, ga);
        }
        return 0.f;
    } else {
        const float fl = floorf(s);
        const float t = s - fl;
        const int n = nB + (int)fl;
        float d = 0.f;
        if constexpr (IP == IN_LINEAR) {
            if constexpr (GC) {
                const float p0 = ((unsigned)n < (unsigned)S) ? load_e<ET>(tr, n) : 0.f;
                const float p1 = ((unsigned)(n + 1) < (unsigned)S) ? load_e<ET>(tr, n + 1) : 0.f;
                d = a_w * (p1 - p0);
            }
            if constexpr (GE) {
                if ((unsigned)n < (unsigned)S) atomicAdd(ge + n, ga * (1.f - t));
                if ((unsigned)(n + 1) < (unsigned)S) atomicAdd(ge + n + 1, ga * t);
            }
        } else {
            if constexpr (GC) {
                const float pm = ((unsigned)(n - 1) < (unsigned)S) ? load_e<ET>(tr, n - 1) : 0.f;
                const float p0 = ((unsigned)n < (unsigned)S) ? load_e<ET>(tr, n) : 0.f;
                const float p1 = ((unsigned)(n + 1) < (unsigned)S) ? load_e<ET>(tr, n + 1) : 0.f;
                const float p2 = ((unsigned)(n + 2) < (unsigned)S) ? load_e<ET>(tr, n + 2) : 0.f;
                const float c1 = 0.5f * (p1 - pm);
                const float c2 = pm - 2.5f * p0 + 2.0f * p1 - 0.5f * p2;
                const float c3 = 0.5f * (p2 - pm) + 1.5f * (p0 - p1);
                d = a_w * fmaf(t, fmaf(2.f, c2, 3.f * t * c3), c1);
            }
            if constexpr (GE) {
                const float t2 = t * t, t3 = t2 * t;
                const float w[4] = {-0.5f * t + t2 - 0.5f * t3, 1.f - 2.5f * t2 + 1.5f * t3,
                                    0.5f * t + 2.f * t2 - 1.5f * t3, -0.5f * t2 + 0.5f * t3};
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if ((unsigned)(n - 1 + q) < (unsigned)S) atomicAdd(ge + n - 1 + q, ga * w[q]);
            }
        }
        return d;
    }
}

// Per lane: returns sum_ij a v'(s) ds/dc (if GC); scatters into grad_e (if GE).
template <int MODE, int ET, int IP, bool GE, bool GC>
__device__ inline float adjoint_point(const DasArgs &a, const Lane &L, float G)
{
    const float kf = (float)a.k;
    const float kc = (float)(a.k / a.c);     // d/dc of (path * fs / c) = -path * k / c
    const bool live = L.active && (GC || G != 0.f);
    float acc = 0.f;
    const float xr = rx_coord<MODE>(L.x, L.y);
    for (int j = 0; j < a.n_ch; ++j) {
        const float cj = a.rx_c[j];
        if constexpr (MODE != MODE_HERCULES) {
            // separable modes: transmit path z + Et, receive path z + Er
            const float dxr = xr - cj;
            const float r2 = dxr * dxr;
            const bool act = live && r2 < L.thr;
            if (!__any(act)) continue;
            const float Er = excess(r2, L.z, L.z2);
            const float Rj = fmaf(Er, kf, L.fB);
            const float aj = act ? hann_u2(r2 * L.wsc) : 0.f;
            for (int i = 0; i < a.n_tx; ++i) {
                if (act) {
                    const float Et = tx_excess<MODE>(a, L.x, L.z, L.z2, i);
                    const float s = fmaf(Et, kf, Rj);
                    const long trace = (long)i * a.n_ch + j;
                    const float d = adjoint_term<ET, IP, GE, GC>(
                        trace_ptr<ET>(a.e, trace, a.S), a.grad_e + trace * a.S, a.S, L.nB, s,
                        G * aj, aj);
                    if constexpr (GC) acc = fmaf(d, -(2.f * L.z + Er + Et) * kc, acc);
                }
            }
        } else {
            const float dy = L.y - cj;
            const float dy2 = dy * dy;
            if (!__any(live && dy2 < L.thr)) continue;
            for (int i = 0; i < a.n_tx; ++i) {
                const float dx = L.x - a.tx_x[i];
                const float rho2 = fmaf(dx, dx, dy2);
                const bool act = live && rho2 < L.thr;
                if (!__any(act)) continue;
                if (act) {
                    const float E = excess(rho2, L.z, L.z2);
                    const float s = fmaf(E, kf, L.fB);
                    const float w = hann_u2(rho2 * L.wsc);
                    const long trace = (long)i * a.n_ch + j;
                    const float d = adjoint_term<ET, IP, GE, GC>(
                        trace_ptr<ET>(a.e, trace, a.S), a.grad_e + trace * a.S, a.S, L.nB, s,
                        G * w, w);
                    // path = transmit path of the point (plane or diverging) + z + E
                    if constexpr (GC) acc = fmaf(d, -(L.ptx + L.z + E) * kc, acc);
                }
            }
        }
    }
    return acc;
}

// grid: ceil(n_waves / 4) blocks of 256; writes one FP64 partial of
// sum_p G(p) dout(p)/dc per block (deterministic order).
template <int MODE, int ET, int IP, bool GE, bool GC>
__global__ __launch_bounds__(256) void das_adjoint_kernel(DasArgs a)
{
    __shared__ double red[4];
    const int wave_id = blockIdx.x * 4 + (threadIdx.x >> 6);
    double contrib = 0.0;
    if (wave_id < a.n_waves) {
        const Lane L = lane_setup(a, wave_id, threadIdx.x & 63);
        const float G = L.active ? a.grad_out[L.out_idx] : 0.f;
        const float d = adjoint_point<MODE, ET, IP, GE, GC>(a, L, G);
        contrib = (double)G * (double)d;
    }
    if constexpr (GC) {
        for (int off = 32; off > 0; off >>= 1) contrib += __shfl_down(contrib, off, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = contrib;
        __syncthreads();
        if (threadIdx.x == 0) a.partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
    }
}

// Sum of the per-block partials in a fixed order -> grad_c.
// out[b] = sum of partial[b * n .. b * n + n) in a fixed order (one
// workgroup per frame b).
__global__ __launch_bounds__(256) void reduce_partials_kernel(const double *partial, int n,
                                                             float *out)
{
    __shared__ double red[256];
    partial += (long)blockIdx.x * n;
    out += blockIdx.x;
    double s = 0.0;
    for (int q = threadIdx.x; q < n; q += 256) s += partial[q];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = (float)red[0];
}

hipError_t launch_reduce_partials(const double *partial, int n, float *out, hipStream_t s,
                                  int n_frames)
{
    hipLaunchKernelGGL(reduce_partials_kernel, dim3(n_frames), dim3(256), 0, s, partial, n, out);
    return hipGetLastError();
}

__global__ void fill_kernel(float *p, long n, float v)
{
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (long)gridDim.x * blockDim.x)
        p[q] = v;
}

template <int MODE, int ET, int IP>
static hipError_t launch_adj3(const DasArgs &a, bool ge, bool gc, hipStream_t s)
{
    dim3 grid((a.n_waves + 3) / 4);
    if (ge && gc)
        hipLaunchKernelGGL((das_adjoint_kernel<MODE, ET, IP, true, true>), grid, dim3(256), 0, s, a);
    else if (ge)
        hipLaunchKernelGGL((das_adjoint_kernel<MODE, ET, IP, true, false>), grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((das_adjoint_kernel<MODE, ET, IP, false, true>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

template <int MODE, int ET>
static hipError_t launch_adj2(const DasArgs &a, int ip, bool ge, bool gc, hipStream_t s)
{
    switch (ip) {
        case IN_NEAREST: return launch_adj3<MODE, ET, IN_NEAREST>(a, ge, gc, s);
        case IN_LINEAR: return launch_adj3<MODE, ET, IN_LINEAR>(a, ge, gc, s);
        case IN_CUBIC: return launch_adj3<MODE, ET, IN_CUBIC>(a, ge, gc, s);
        default: return hipErrorInvalidValue;
    }
}

template <int MODE>
static hipError_t launch_adj1(const DasArgs &a, int et, int ip, bool ge, bool gc, hipStream_t s)
{
    switch (et) {
        case ET_F32: return launch_adj2<MODE, ET_F32>(a, ip, ge, gc, s);
        case ET_BF16: return launch_adj2<MODE, ET_BF16>(a, ip, ge, gc, s);
        case ET_I32: return launch_adj2<MODE, ET_I32>(a, ip, ge, gc, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fill(float *p, long n, float v, hipStream_t s)
{
    long blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_das_adjoint(const DasArgs &a, int mode, int et, int ip, float *grad_c,
                              hipStream_t s)
{
    const bool ge = a.grad_e != nullptr, gc = grad_c != nullptr;
    if (!ge && !gc) return hipSuccess;
    hipError_t err;
    if (ge) {
        err = launch_fill(a.grad_e, (long)a.n_tx * a.n_ch * a.S, 0.f, s);
        if (err != hipSuccess) return err;
    }
    switch (mode) {
        case MODE_FORCES: err = launch_adj1<MODE_FORCES>(a, et, ip, ge, gc, s); break;
        case MODE_HERCULES: err = launch_adj1<MODE_HERCULES>(a, et, ip, ge, gc, s); break;
        case MODE_TPW: err = launch_adj1<MODE_TPW>(a, et, ip, ge, gc, s); break;
        case MODE_VLS: err = launch_adj1<MODE_VLS>(a, et, ip, ge, gc, s); break;
        default: return hipErrorInvalidValue;
    }
    if (err != hipSuccess || !gc) return err;
    hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(256), 0, s, a.partial,
                       (a.n_waves + 3) / 4, grad_c);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sharpness: L = -sum I^4 / (sum I^2)^2 per image, FP64 sums, one workgroup
// per image (deterministic order), then dL/dI in a second sweep.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void sharpness_kernel(const float *img, long n, float *loss,
                                                         float *grad)
{
    __shared__ double sP[1024], sQ[1024];
    const float *I = img + (long)blockIdx.x * n;
    double P = 0.0, Q = 0.0;
    for (long q = threadIdx.x; q < n; q += 1024) {
        const double x = I[q], x2 = x * x;
        Q += x2;
        P += x2 * x2;
    }
    sP[threadIdx.x] = P;
    sQ[threadIdx.x] = Q;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            sP[threadIdx.x] += sP[threadIdx.x + w];
            sQ[threadIdx.x] += sQ[threadIdx.x + w];
        }
        __syncthreads();
    }
    P = sP[0];
    Q = sQ[0];
    if (threadIdx.x == 0) loss[blockIdx.x] = (Q > 0.0) ? (float)(-P / (Q * Q)) : 0.f;
    if (grad) {
        float *g = grad + (long)blockIdx.x * n;
        const double a = (Q > 0.0) ? -4.0 / (Q * Q) : 0.0;
        const double b = (Q > 0.0) ? 4.0 * P / (Q * Q * Q) : 0.0;
        for (long q = threadIdx.x; q < n; q += 1024) {
            const double x = I[q];
            g[q] = (float)(a * x * x * x + b * x);
        }
    }
}

hipError_t launch_sharpness(const float *img, long n, int n_images, float *loss, float *grad,
                            hipStream_t s)
{
    hipLaunchKernelGGL(sharpness_kernel, dim3(n_images), dim3(1024), 0, s, img, n, loss, grad);
    return hipGetLastError();
}

}  // namespace bf
