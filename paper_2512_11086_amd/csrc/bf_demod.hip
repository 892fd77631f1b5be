// bf_demod.hip -- demodulation, filtering and decimation of int16 RF
// (Eq. 4; Sec. VII-D), the stage before decoding.
//
// Eq. 4 mixes every input sample with exp(-j 2 pi r n) (r = fd / fs, n counted
// from sample 0) and then applies the FIR filter h (the baseband matched filter
// doubles as the low-pass).  The kernel uses the equivalent form
//     y[n] = exp(-j 2 pi r n) * sum_k g[k] x[n - k],   g[k] = h[k] exp(j 2 pi r k),
// (the mix factors as exp(-j 2 pi r n) exp(j 2 pi r k)), so each tap is one
// complex-by-real product (2 FMAs) on the raw samples and the output is rotated
// once.  g and the per-output rotation exp(-j 2 pi r q D) are computed on the
// host in FP64 and rounded to FP32.  Only the kept outputs q D are computed
// (decimation, Sec. VII-C: as early as possible, after the low-pass).
//
// A workgroup owns 256 consecutive outputs of one trace.  It stages the input
// span they read (255 D + N_f samples, converted to FP32 once, zeros before the
// record -- the paper's LDS filter with zero padding) in LDS, split into its D
// polyphase components so that lanes whose outputs are D samples apart read
// consecutive LDS words.  Taps are workgroup-uniform and come through scalar
// loads.
#include <math.h>
#include <string.h>

#include <vector>

#include "bf.h"
#include "bf_common.h"
#include "bf_plan.h"

namespace bf {

constexpr int DEMOD_THREADS = 256;
constexpr int DEMOD_MAX_TAPS = 1024;
constexpr int DEMOD_MAX_D = 16;

struct DemodArgs {
    const int16_t *x;     // [n_traces][S]
    void *y;              // [n_traces][n_out][2], int16 or f32
    const float2 *g;      // [n_taps] folded taps, polyphase order (see bf_demod_create)
    const float2 *rot;    // [n_out] exp(-j 2 pi r q D)
    int n_traces, S, n_out, D, n_taps;
    int chunks;           // workgroups per trace
    int phase_len;        // LDS words per polyphase component
};

__device__ inline int16_t sat_i16(float v)
{
    const float r = __builtin_rintf(v);                       // ties to even
    return (int16_t)(int)fminf(fmaxf(r, -32768.f), 32767.f);
}

template <int OT>
__global__ __launch_bounds__(DEMOD_THREADS) void demod_kernel(DemodArgs a)
{
    extern __shared__ float xs[];                 // [D][phase_len]
    const int blk = blockIdx.x;
    const int trace = blk / a.chunks;
    const int q0 = (blk - trace * a.chunks) * DEMOD_THREADS;
    const int16_t *x = a.x + (long)trace * a.S;
    // span position p holds input sample n0 + p, n0 = q0 D - (N_f - 1);
    // stored at xs[(p % D) * phase_len + p / D]
    const int n0 = q0 * a.D - (a.n_taps - 1);
    const int span = (DEMOD_THREADS - 1) * a.D + a.n_taps;
    for (int p = threadIdx.x; p < span; p += DEMOD_THREADS) {
        const int n = n0 + p;
        const float v = (n >= 0 && n < a.S) ? (float)x[n] : 0.f;
        const int ph = p % a.D;
        xs[ph * a.phase_len + p / a.D] = v;
    }
    __syncthreads();
    const int q = q0 + threadIdx.x;
    // Output q = q0 + t reads span positions t D + off, off = N_f - 1 - k,
    // i.e. word t + off / D of polyphase component off % D.  Loop over the
    // components; inside one, off = ph + D b, so the LDS word advances by one
    // and the taps (host-ordered the same way in g) are contiguous.
    const int top = a.n_taps - 1;
    float ar = 0.f, ai = 0.f;
    const float2 *__restrict__ gp = a.g;
    for (int ph = 0; ph < a.D && ph <= top; ++ph) {
        const int nb = (top - ph) / a.D + 1;
        const float *xp = xs + ph * a.phase_len + threadIdx.x;
        int b = 0;
        for (; b + 4 <= nb; b += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float v = xp[b + u];
                ar = fmaf(gp[b + u].x, v, ar);
                ai = fmaf(gp[b + u].y, v, ai);
            }
        }
        for (; b < nb; ++b) {
            const float v = xp[b];
            ar = fmaf(gp[b].x, v, ar);
            ai = fmaf(gp[b].y, v, ai);
        }
        gp += nb;
    }
    if (q >= a.n_out) return;
    const float2 r = a.rot[q];
    const float yr = fmaf(ar, r.x, -ai * r.y);
    const float yi = fmaf(ar, r.y, ai * r.x);
    const long o = (long)trace * a.n_out + q;
    if constexpr (OT == BF_IQ_I16) {
        const uint32_t lo = (uint16_t)sat_i16(yr), hi = (uint16_t)sat_i16(yi);
        static_cast<uint32_t *>(a.y)[o] = lo | (hi << 16);
    } else {
        static_cast<float2 *>(a.y)[o] = make_float2(yr, yi);
    }
}

}  // namespace bf

using namespace bf;

struct bf_demod_s {
    uint32_t magic = 0xBFDE0D01u;
    bf_demod_params p;
    int n_out = 0;
    float2 *d_g = nullptr;
    float2 *d_rot = nullptr;
    ~bf_demod_s()
    {
        if (d_g) (void)hipFree(d_g);
        if (d_rot) (void)hipFree(d_rot);
    }
};

static int validate_demod(const bf_demod_params *p)
{
    if (!p) return fail(BF_ERR_NULL, "params is NULL");
    if (!p->taps_re) return fail(BF_ERR_NULL, "taps_re is NULL");
    if (p->n_traces < 1) return fail(BF_ERR_SHAPE, "n_traces=%d < 1", p->n_traces);
    if (p->n_samples < 1 || p->n_samples > 65536)
        return fail(BF_ERR_SHAPE, "n_samples=%d not in [1,65536]", p->n_samples);
    if (p->decimation < 1 || p->decimation > DEMOD_MAX_D)
        return fail(BF_ERR_SHAPE, "decimation=%d not in [1,%d]", p->decimation, DEMOD_MAX_D);
    if (p->n_taps < 1 || p->n_taps > DEMOD_MAX_TAPS)
        return fail(BF_ERR_SHAPE, "n_taps=%d not in [1,%d]", p->n_taps, DEMOD_MAX_TAPS);
    if (p->out_type != BF_IQ_I16 && p->out_type != BF_IQ_F32)
        return fail(BF_ERR_UNSUPPORTED, "unknown IQ output type %d", p->out_type);
    if ((int64_t)p->n_traces * p->n_samples >= (int64_t(1) << 31))
        return fail(BF_ERR_TOO_LARGE, "input has more than 2^31 samples");
    if (!isfinite(p->fs) || p->fs <= 0.0) return fail(BF_ERR_GEOMETRY, "fs must be finite and > 0");
    if (!isfinite(p->fd)) return fail(BF_ERR_GEOMETRY, "fd must be finite");
    for (int k = 0; k < p->n_taps; ++k)
        if (!isfinite(p->taps_re[k]) || (p->taps_im && !isfinite(p->taps_im[k])))
            return fail(BF_ERR_GEOMETRY, "tap %d is not finite", k);
    return BF_OK;
}

// exp(j 2 pi f) with f reduced to [0, 1) in FP64 first
static float2 cis_rev(double f)
{
    f -= floor(f);
    return make_float2((float)cos(2.0 * M_PI * f), (float)sin(2.0 * M_PI * f));
}

extern "C" {

int bf_demod_create(const bf_demod_params *params, bf_demod *out)
{
    clear_err();
    if (!out) return fail(BF_ERR_NULL, "out is NULL");
    *out = nullptr;
    int st = validate_demod(params);
    if (st != BF_OK) return st;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1) {
        (void)hipGetLastError();
        return fail(BF_ERR_NO_DEVICE, "no HIP device available");
    }
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return fail(BF_ERR_HIP, "device query failed");
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(BF_ERR_NO_DEVICE, "device %d is %s, libbf is built for gfx950", dev,
                    prop.gcnArchName);
    bf_demod d = new bf_demod_s();
    d->p = *params;
    d->p.taps_re = nullptr;
    d->p.taps_im = nullptr;
    const int D = params->decimation, N = params->n_taps;
    d->n_out = (params->n_samples + D - 1) / D;
    const double r = params->fd / params->fs;
    std::vector<float2> g, rot(d->n_out);
    // g[k] = h[k] exp(j 2 pi r k) in FP64, stored in the kernel's read order:
    // component ph = 0 .. D-1, then k = N-1-ph, N-1-ph-D, ... >= 0
    for (int ph = 0; ph < D && ph < N; ++ph)
        for (int k = N - 1 - ph; k >= 0; k -= D) {
            const double hr = params->taps_re[k], hi = params->taps_im ? params->taps_im[k] : 0.0;
            double f = r * k;
            f -= floor(f);
            const double c = cos(2.0 * M_PI * f), s = sin(2.0 * M_PI * f);
            g.push_back(make_float2((float)(hr * c - hi * s), (float)(hr * s + hi * c)));
        }
    for (int q = 0; q < d->n_out; ++q) rot[q] = cis_rev(-r * (double)q * D);
    hipError_t e;
    if ((e = hipMalloc(&d->d_g, N * sizeof(float2))) != hipSuccess ||
        (e = hipMalloc(&d->d_rot, d->n_out * sizeof(float2))) != hipSuccess ||
        (e = hipMemcpy(d->d_g, g.data(), N * sizeof(float2), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(d->d_rot, rot.data(), d->n_out * sizeof(float2), hipMemcpyHostToDevice)) !=
            hipSuccess) {
        delete d;
        return hip_fail(e, "demodulator tables");
    }
    *out = d;
    return BF_OK;
}

int bf_demod_destroy(bf_demod d)
{
    clear_err();
    if (!d) return BF_OK;
    if (d->magic != 0xBFDE0D01u) return fail(BF_ERR_STATE, "not a live demodulator");
    (void)hipDeviceSynchronize();
    d->magic = 0;
    delete d;
    return BF_OK;
}

int bf_demod_out_samples(bf_demod d, int32_t *n_out)
{
    clear_err();
    if (!d || !n_out) return fail(BF_ERR_NULL, "demodulator and n_out must be non-NULL");
    if (d->magic != 0xBFDE0D01u) return fail(BF_ERR_STATE, "not a live demodulator");
    *n_out = d->n_out;
    return BF_OK;
}

int bf_demodulate(bf_demod d, const int16_t *rf, void *iq, void *stream)
{
    clear_err();
    if (!d) return fail(BF_ERR_NULL, "demodulator is NULL");
    if (d->magic != 0xBFDE0D01u) return fail(BF_ERR_STATE, "not a live demodulator");
    if (!rf || !iq) return fail(BF_ERR_NULL, "rf and iq must be non-NULL");
    DemodArgs a;
    a.x = rf;
    a.y = iq;
    a.g = d->d_g;
    a.rot = d->d_rot;
    a.n_traces = d->p.n_traces;
    a.S = d->p.n_samples;
    a.n_out = d->n_out;
    a.D = d->p.decimation;
    a.n_taps = d->p.n_taps;
    a.chunks = (d->n_out + DEMOD_THREADS - 1) / DEMOD_THREADS;
    const int span = (DEMOD_THREADS - 1) * a.D + a.n_taps;
    a.phase_len = (span + a.D - 1) / a.D;
    const size_t shm = (size_t)a.D * a.phase_len * sizeof(float);
    const long blocks = (long)a.n_traces * a.chunks;
    if (blocks >= (1L << 31)) return fail(BF_ERR_TOO_LARGE, "too many workgroups");
    hipStream_t s = (hipStream_t)stream;
    if (d->p.out_type == BF_IQ_I16)
        hipLaunchKernelGGL(demod_kernel<BF_IQ_I16>, dim3((unsigned)blocks), dim3(DEMOD_THREADS),
                           shm, s, a);
    else
        hipLaunchKernelGGL(demod_kernel<BF_IQ_F32>, dim3((unsigned)blocks), dim3(DEMOD_THREADS),
                           shm, s, a);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? BF_OK : hip_fail(e, "demodulation launch");
}

}  // extern "C"
