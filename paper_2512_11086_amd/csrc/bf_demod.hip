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
// host in FP64 (quarter turns exactly) and rounded to FP32.  Only the kept
// outputs q D are computed (decimation, Sec. VII-C: as early as possible,
// after the low-pass).  With quadrature sampling (fs = 4 fd, Sec. IV-B) and a
// real filter, g[k] = h[k] j^k: every polyphase component of an even
// decimation is purely real or purely imaginary, and the kernel then spends
// one FMA per tap on it instead of two.
//
// A workgroup of T threads owns 4 T consecutive outputs of one trace.  It
// stages the input span they read (converted to FP32 once, zeros before the
// record -- the paper's LDS filter with zero padding) in LDS, split into its D
// polyphase components: within a component, outputs q and q + 1 read
// neighbouring words.  Each thread computes 4 consecutive outputs from a
// sliding 8-word register window refilled by one aligned 16-byte LDS read per
// 4 taps, so every LDS word read feeds 4 outputs (the paper's LDS sharing,
// carried one level further into registers).  Taps are workgroup-uniform and
// come through scalar loads.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "bf.h"
#include "bf_common.h"
#include "bf_plan.h"

namespace bf {

constexpr int DEMOD_M = 4;            // consecutive outputs per thread
constexpr int DEMOD_MAX_TAPS = 1024;
constexpr int DEMOD_MAX_D = 16;

struct DemodArgs {
    const int16_t *x;     // [n_traces][S]
    void *y;              // [n_traces][n_out][2], int16 or f32
    const float2 *g;      // folded taps, polyphase order, each component padded to 4
    const float2 *rot;    // [n_out] exp(-j 2 pi r q D)
    int n_traces, S, n_out, D, n_taps;
    int chunks;           // workgroups per trace
    int phase_len;        // LDS words per polyphase component (multiple of 4)
    int kind[16];         // per component: 0 complex taps, 1 real only, 2 imaginary only
    int lg_d;             // log2(D) when D is a power of two and the trace rows are
                          // 16-byte aligned (vector staging), else -1
};

enum { TAPS_COMPLEX = 0, TAPS_REAL = 1, TAPS_IMAG = 2 };

__device__ inline int16_t sat_i16(float v)
{
    const float r = __builtin_rintf(v);                       // ties to even
    return (int16_t)(int)fminf(fmaxf(r, -32768.f), 32767.f);
}

// Two rounded, saturated values packed as (lo, hi) int16: round half to
// even, clamp in FP32 (exact at the int16 limits), convert, pack.
__device__ inline uint32_t sat_pk_i16(float lo, float hi)
{
    const int a = (int)__builtin_amdgcn_fmed3f(__builtin_rintf(lo), -32768.f, 32767.f);
    const int b = (int)__builtin_amdgcn_fmed3f(__builtin_rintf(hi), -32768.f, 32767.f);
    return __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pk_i16(a, b));
}

// Taps of polyphase component ph (of D) of an N-tap filter, and that count
// rounded up to a multiple of 4 (the host pads with zero taps).
__host__ __device__ inline int phase_taps(int N, int D, int ph)
{
    return ph < N ? (N - 1 - ph) / D + 1 : 0;
}
__host__ __device__ inline int phase_taps4(int N, int D, int ph)
{
    return (phase_taps(N, D, ph) + 3) & ~3;
}

// One polyphase component's taps for the thread's M = 4 outputs: words
// wp[0 ..] of the component (the outputs' inputs shifted by one word each),
// taps gp[0 .. nb4) (nb4 a multiple of 4, zero-padded).  Each 4-tap block
// reads one aligned 16-byte LDS word group and two 16-byte tap pairs through
// the scalar cache; KIND drops the products the component does not have.
template <int KIND>
__device__ inline void fir_phase(const float4 *wp, const float2 *__restrict__ gp, int nb4,
                                 float (&ar)[DEMOD_M], float (&ai)[DEMOD_M])
{
    const float4 *__restrict__ g4 = reinterpret_cast<const float4 *>(gp);
    float4 lo = wp[0];
#pragma unroll 2
    for (int b = 0; b < nb4; b += 4) {
        const float4 hi = wp[b / 4 + 1];
        const float w[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
        const float4 g01 = g4[b / 2], g23 = g4[b / 2 + 1];
        const float gr[4] = {g01.x, g01.z, g23.x, g23.z};
        const float gi[4] = {g01.y, g01.w, g23.y, g23.w};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
            for (int m = 0; m < DEMOD_M; ++m) {
                if constexpr (KIND != TAPS_IMAG) ar[m] = fmaf(gr[u], w[u + m], ar[m]);
                if constexpr (KIND != TAPS_REAL) ai[m] = fmaf(gi[u], w[u + m], ai[m]);
            }
        }
        lo = hi;
    }
}

template <int OT, int T>
__global__ __launch_bounds__(T) void demod_kernel(DemodArgs a)
{
    extern __shared__ float4 xs4[];                // [D][phase_len / 4]
    float *xs = reinterpret_cast<float *>(xs4);
    const int t = threadIdx.x;
    const int blk = blockIdx.x;
    const int trace = blk / a.chunks;
    const int q0 = (blk - trace * a.chunks) * (T * DEMOD_M);
    const int16_t *x = a.x + (long)trace * a.S;
    // Word w of component ph holds input sample n0 + ph + D w, with
    // n0 = q0 D - (N_f - 1); samples outside the record read as 0.
    const int n0 = q0 * a.D - (a.n_taps - 1);
    if (a.lg_d >= 0) {
        // Vector form: thread c converts the 8 samples nb .. nb + 7
        // (nb = n_al + 8 c, n_al = n0 rounded down to a multiple of 8) from one
        // 16-byte load; sample n goes to component (n - n0) & (D - 1), word
        // (n - n0) >> log2 D, if it lies in the staged span [n0, n0 + D len).
        const int span = a.D * a.phase_len;
        const int n_al = n0 & ~7;
        const int nchunks = (n0 + span - n_al + 7) >> 3;
        for (int c = t; c < nchunks; c += T) {
            const int nb = n_al + 8 * c;
            int vals[8];
            if (nb >= 0 && nb + 8 <= a.S) {
                const int4 raw = *reinterpret_cast<const int4 *>(x + nb);
                const int w4[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    vals[2 * i] = (int16_t)(w4[i] & 0xFFFF);          // low half
                    vals[2 * i + 1] = (int16_t)((uint32_t)w4[i] >> 16);  // high half
                }
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    vals[i] = (nb + i >= 0 && nb + i < a.S) ? (int)x[nb + i] : 0;
            }
            // word address of sample rel: (rel mod D) len + rel / D (the 24-bit
            // product runs at full rate)
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int rel = nb + i - n0;
                if ((unsigned)rel < (unsigned)span)
                    xs[__umul24(rel & (a.D - 1), a.phase_len) + (rel >> a.lg_d)] = (float)vals[i];
            }
        }
    } else
    // Loads are unconditional from a clamped index (then zeroed), four per
    // thread in flight before their conversions.
    for (int ph = 0; ph < a.D; ++ph) {
        for (int w0 = 0; w0 < a.phase_len; w0 += 4 * T) {
            int16_t v[4];
            int n[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                n[u] = n0 + ph + a.D * (w0 + u * T + t);
                v[u] = x[min(max(n[u], 0), a.S - 1)];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int w = w0 + u * T + t;
                if (w < a.phase_len)
                    xs[ph * a.phase_len + w] = (n[u] >= 0 && n[u] < a.S) ? (float)v[u] : 0.f;
            }
        }
    }
    __syncthreads();
    // Output o = t M + m (of this workgroup) reads word o + b of component ph
    // for tap k = N_f - 1 - ph - D b.  The thread slides an 8-word window
    // along its words tM + b .. tM + b + 7, refilled by one aligned 16-byte
    // read per 4 taps; each word then feeds all M outputs.
    float ar[DEMOD_M], ai[DEMOD_M];
#pragma unroll
    for (int m = 0; m < DEMOD_M; ++m) ar[m] = ai[m] = 0.f;
    const float2 *__restrict__ gp = a.g;
    for (int ph = 0; ph < a.D; ++ph) {
        const int nb4 = phase_taps4(a.n_taps, a.D, ph);
        const float4 *wp = xs4 + (ph * a.phase_len) / 4 + t;   // words tM .. (M = 4)
        // the tap kind is uniform per component: one straight loop each
        switch (a.kind[ph]) {
            case TAPS_REAL: fir_phase<TAPS_REAL>(wp, gp, nb4, ar, ai); break;
            case TAPS_IMAG: fir_phase<TAPS_IMAG>(wp, gp, nb4, ar, ai); break;
            default: fir_phase<TAPS_COMPLEX>(wp, gp, nb4, ar, ai); break;
        }
        gp += nb4;
    }
    const int q = q0 + t * DEMOD_M;
    if (q >= a.n_out) return;
    const long o = (long)trace * a.n_out + q;
    if (q + DEMOD_M <= a.n_out) {
        const float4 r01 = *reinterpret_cast<const float4 *>(a.rot + q);
        const float4 r23 = *reinterpret_cast<const float4 *>(a.rot + q + 2);
        const float rx[4] = {r01.x, r01.z, r23.x, r23.z}, ry[4] = {r01.y, r01.w, r23.y, r23.w};
        float yr[4], yi[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            yr[m] = fmaf(ar[m], rx[m], -ai[m] * ry[m]);
            yi[m] = fmaf(ar[m], ry[m], ai[m] * rx[m]);
        }
        if constexpr (OT == BF_IQ_I16) {
            uint4 v;
            v.x = sat_pk_i16(yr[0], yi[0]);
            v.y = sat_pk_i16(yr[1], yi[1]);
            v.z = sat_pk_i16(yr[2], yi[2]);
            v.w = sat_pk_i16(yr[3], yi[3]);
            uint32_t *dst = static_cast<uint32_t *>(a.y) + o;
            if ((reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
                *reinterpret_cast<uint4 *>(dst) = v;
            } else {
                dst[0] = v.x; dst[1] = v.y; dst[2] = v.z; dst[3] = v.w;
            }
        } else {
            float2 *dst = static_cast<float2 *>(a.y) + o;
#pragma unroll
            for (int m = 0; m < 4; ++m) dst[m] = make_float2(yr[m], yi[m]);
        }
    } else {
#pragma unroll
        for (int m = 0; m < DEMOD_M; ++m) {
            if (q + m >= a.n_out) break;
            const float2 r = a.rot[q + m];
            const float yr = fmaf(ar[m], r.x, -ai[m] * r.y);
            const float yi = fmaf(ar[m], r.y, ai[m] * r.x);
            if constexpr (OT == BF_IQ_I16)
                static_cast<uint32_t *>(a.y)[o + m] =
                    (uint16_t)sat_i16(yr) | ((uint32_t)(uint16_t)sat_i16(yi) << 16);
            else
                static_cast<float2 *>(a.y)[o + m] = make_float2(yr, yi);
        }
    }
}

}  // namespace bf

using namespace bf;

struct bf_demod_s {
    uint32_t magic = 0xBFDE0D01u;
    bf_demod_params p;
    int n_out = 0;
    int kind[16];
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

// exp(j 2 pi f) in FP64 with f reduced to [0, 1); quarter turns exactly
static void cis_rev(double f, double *c, double *s)
{
    f -= floor(f);
    const double q = 4.0 * f;
    if (q == floor(q)) {
        static const double cq[4] = {1.0, 0.0, -1.0, 0.0}, sq[4] = {0.0, 1.0, 0.0, -1.0};
        *c = cq[(int)q & 3];
        *s = sq[(int)q & 3];
        return;
    }
    *c = cos(2.0 * M_PI * f);
    *s = sin(2.0 * M_PI * f);
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
    for (int ph = 0; ph < 16; ++ph) d->kind[ph] = TAPS_COMPLEX;
    // g[k] = h[k] exp(j 2 pi r k) in FP64, stored in the kernel's read order:
    // component ph = 0 .. D-1, then k = N-1-ph, N-1-ph-D, ... >= 0, each
    // component padded with zero taps to a multiple of 4
    for (int ph = 0; ph < D; ++ph) {
        const size_t start = g.size();
        bool all_re = true, all_im = true;
        for (int k = N - 1 - ph; k >= 0; k -= D) {
            const double hr = params->taps_re[k], hi = params->taps_im ? params->taps_im[k] : 0.0;
            double c, s;
            cis_rev(r * k, &c, &s);
            const double gr = hr * c - hi * s, gi = hr * s + hi * c;
            all_re = all_re && gi == 0.0;
            all_im = all_im && gr == 0.0;
            g.push_back(make_float2((float)gr, (float)gi));
        }
        g.resize(start + phase_taps4(N, D, ph), make_float2(0.f, 0.f));
        d->kind[ph] = all_re ? TAPS_REAL : all_im ? TAPS_IMAG : TAPS_COMPLEX;
    }
    for (int q = 0; q < d->n_out; ++q) {
        double c, s;
        cis_rev(-r * (double)q * D, &c, &s);
        rot[q] = make_float2((float)c, (float)s);
    }
    hipError_t e;
    if ((e = hipMalloc(&d->d_g, g.size() * sizeof(float2))) != hipSuccess ||
        (e = hipMalloc(&d->d_rot, d->n_out * sizeof(float2))) != hipSuccess ||
        (e = hipMemcpy(d->d_g, g.data(), g.size() * sizeof(float2), hipMemcpyHostToDevice)) !=
            hipSuccess ||
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
    // Workgroup of T threads x 4 outputs; each component needs the words of
    // T*4 outputs plus its padded taps plus the window's 4-word prefetch.
    int nb4max = 0;
    for (int ph = 0; ph < a.D; ++ph) nb4max = std::max(nb4max, phase_taps4(a.n_taps, a.D, ph));
    const int T = (a.D * (256 * DEMOD_M + nb4max + 4) * 4 <= 48 * 1024) ? 256 : 64;
    a.chunks = (d->n_out + T * DEMOD_M - 1) / (T * DEMOD_M);
    for (int ph = 0; ph < 16; ++ph) a.kind[ph] = d->kind[ph];
    a.phase_len = T * DEMOD_M + nb4max + 4;
    // vector staging: D a power of two, every trace row 16-byte aligned
    a.lg_d = -1;
    if ((a.D & (a.D - 1)) == 0 && a.S % 8 == 0 && (reinterpret_cast<uintptr_t>(rf) & 15) == 0)
        for (int l = 0; l < 5; ++l)
            if ((1 << l) == a.D) a.lg_d = l;
    const size_t shm = (size_t)a.D * a.phase_len * sizeof(float);
    const long blocks = (long)a.n_traces * a.chunks;
    if (blocks >= (1L << 31)) return fail(BF_ERR_TOO_LARGE, "too many workgroups");
    hipStream_t s = (hipStream_t)stream;
    if (d->p.out_type == BF_IQ_I16) {
        if (T == 256)
            hipLaunchKernelGGL((demod_kernel<BF_IQ_I16, 256>), dim3((unsigned)blocks), dim3(T), shm, s, a);
        else
            hipLaunchKernelGGL((demod_kernel<BF_IQ_I16, 64>), dim3((unsigned)blocks), dim3(T), shm, s, a);
    } else {
        if (T == 256)
            hipLaunchKernelGGL((demod_kernel<BF_IQ_F32, 256>), dim3((unsigned)blocks), dim3(T), shm, s, a);
        else
            hipLaunchKernelGGL((demod_kernel<BF_IQ_F32, 64>), dim3((unsigned)blocks), dim3(T), shm, s, a);
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? BF_OK : hip_fail(e, "demodulation launch");
}

}  // extern "C"
