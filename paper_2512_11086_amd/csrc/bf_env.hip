// bf_env.hip -- envelope detection and display compression of beamformed
// images (the stage after DAS: the paper's Hilbert transform and its log /
// power display scales).
//
// A real (RF) image is [n_cols][N] with depth fastest; the envelope of a
// column is |x_a| with x_a its analytic signal along depth:
//     X = DFT_N(x),  X_a[k] = h[k] X[k]  (h = 1 at DC and Nyquist, 2 for
//     positive, 0 for negative frequencies),  x_a = IDFT_N(X_a).
// Power-of-two N from 64 to 1024: one wavefront per two columns (packed as
// one complex sequence, see env_fft_reg_kernel), FFT held in registers (four-step split N = 64 M: a 64-point FFT across the lanes by
// xor-partner exchanges, a twiddle, an M-point FFT inside each lane, then the
// mirror image for the inverse); no LDS passes and no barriers.  Other
// power-of-two N: one workgroup per column, radix-2 FFT in LDS (forward
// decimation-in-time from a bit-reversed load, spectrum weighting, inverse
// decimation-in-frequency, read back in bit-reversed order).  Twiddles come
// from a host-FP64, stage-major table in global memory (stage len holds
// exp(-j 2 pi pos / len) for pos < len / 2 at offset len / 2 - 1), so the
// lanes of a stage read consecutive entries (cached; no LDS bank conflicts).  Other N: Re x_a = x exactly, and Im x_a is the
// circular convolution of x with q = Im IDFT(h) (host FP64), summed directly.
// IQ images already are analytic: the envelope is |z|.
//
// Compression (ref > 0 is fused into the store; ref <= 0 uses the image
// maximum: every workgroup writes the maximum of its envelope values to a
// partial-max buffer, one workgroup reduces it in a fixed order, and a second
// pass applies the compression -- no atomics, so repeated calls agree):
//     log:   y = max(20 log10(env / ref), -param)
//     power: y = min(env / ref, 1)^param
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "bf.h"
#include "bf_common.h"
#include "bf_plan.h"

namespace bf {

constexpr int ENV_MAX_N = 4096;

struct EnvArgs {
    const float *img;        // [n_cols][N] real, or [n_cols][N][2] complex (iq)
    float *out;              // [n_cols][N]
    const float2 *tw;        // FFT: [N - 1] stage-major twiddles (see above)
    const float2 *tw_lane;   // register FFT: [6][64] W_{2d}^{l mod d}, d = 32, 16, .., 1
    const float2 *tw_mid;    // register FFT: [64][M] W_N^{r bitrev6(l)}
    float2 wm[8];            // register FFT: W_M^j, j < M / 2
    const float *q;          // direct path: [N] Im IDFT(h)
    float *part_max;         // [n_parts] per-workgroup maxima (ref <= 0)
    float *img_max;          // reduced maximum (ref <= 0)
    long n_cols;
    int N, log2n;
    int compress;
    float ref, param;
    float inv_ref;           // 1 / ref (ref > 0)
};

// Compression with the hardware base-2 logarithm and exponential (about 1 ulp
// each): 20 log10(x) = (20 log10 2) log2(x) and x^p = 2^(p log2 x); x = 0
// gives log2 = -inf, i.e. -param dB and 0 (param > 0).  inv_ref = 1 / ref.
__device__ inline float compress_value(float env, int mode, float inv_ref, float param)
{
    const float x = env * inv_ref;
    if (mode == BF_COMPRESS_LOG)
        return fmaxf(6.0205999132796239f * __builtin_amdgcn_logf(x), -param);
    if (mode == BF_COMPRESS_POWER)
        return __builtin_amdgcn_exp2f(param * __builtin_amdgcn_logf(fminf(x, 1.f)));
    return env;
}

// Store one envelope value: compressed now (ref given), or raw with the
// running maximum (compression pass follows).
__device__ inline void store_env(const EnvArgs &a, long idx, float env, float &local_max)
{
    if (a.compress != BF_COMPRESS_NONE && a.ref > 0.f) {
        a.out[idx] = compress_value(env, a.compress, a.inv_ref, a.param);
    } else {
        a.out[idx] = env;
        local_max = fmaxf(local_max, env);
    }
}

// Maximum of the workgroup's envelope values to part_max[blockIdx.x]
// (wavefront shuffles, then LDS across wavefronts; blockDim <= 256).
__device__ inline void publish_max(const EnvArgs &a, float local_max)
{
    if (!(a.compress != BF_COMPRESS_NONE && a.ref <= 0.f)) return;
    __shared__ float s_max[4];
    for (int o = 32; o > 0; o >>= 1) local_max = fmaxf(local_max, __shfl_xor(local_max, o, 64));
    if ((threadIdx.x & 63) == 0) s_max[threadIdx.x >> 6] = local_max;
    __syncthreads();
    if (threadIdx.x == 0) {
        float m = s_max[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmaxf(m, s_max[w]);
        a.part_max[blockIdx.x] = m;
    }
}

__device__ inline float2 cmul(float2 a, float2 b)
{
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}

__device__ inline unsigned bitrev(unsigned v, int bits) { return __brev(v) >> (32 - bits); }

// grid: n_cols workgroups of T threads; LDS: N float2 data
__global__ __launch_bounds__(256) void env_fft_kernel(EnvArgs a)
{
    extern __shared__ float2 sm[];
    float2 *d = sm;
    const float2 *__restrict__ tw = a.tw;
    const int N = a.N, half_n = N >> 1, T = blockDim.x, t = threadIdx.x;
    const long col = blockIdx.x;
    const float *x = a.img + col * N;
    for (int n = t; n < N; n += T) d[bitrev(n, a.log2n)] = make_float2(x[n], 0.f);
    __syncthreads();
    // forward DIT: butterflies (i, i + h) with twiddle exp(-j 2 pi pos / len)
    for (int len = 2; len <= N; len <<= 1) {
        const int h = len >> 1;
        const float2 *twl = tw + (h - 1);
        for (int b = t; b < half_n; b += T) {
            const int pos = b & (h - 1);
            const int i = ((b - pos) << 1) + pos;
            const float2 u = d[i], v = cmul(d[i + h], twl[pos]);
            d[i] = make_float2(u.x + v.x, u.y + v.y);
            d[i + h] = make_float2(u.x - v.x, u.y - v.y);
        }
        __syncthreads();
    }
    // analytic-signal weights: 1 at DC and Nyquist, 2 positive, 0 negative
    for (int k = t; k < N; k += T) {
        const float w = (k == 0 || k == half_n) ? 1.f : (k < half_n ? 2.f : 0.f);
        d[k] = make_float2(d[k].x * w, d[k].y * w);
    }
    __syncthreads();
    // inverse DIF: butterflies (i, i + h), (u + v, (u - v) exp(+j 2 pi pos / len))
    for (int len = N; len >= 2; len >>= 1) {
        const int h = len >> 1;
        const float2 *twl = tw + (h - 1);
        for (int b = t; b < half_n; b += T) {
            const int pos = b & (h - 1);
            const int i = ((b - pos) << 1) + pos;
            const float2 u = d[i], v = d[i + h];
            const float2 w = twl[pos];
            d[i] = make_float2(u.x + v.x, u.y + v.y);
            d[i + h] = cmul(make_float2(u.x - v.x, u.y - v.y), make_float2(w.x, -w.y));
        }
        __syncthreads();
    }
    const float inv_n = 1.f / (float)N;
    float local_max = 0.f;
    for (int n = t; n < N; n += T) {
        const float2 z = d[bitrev(n, a.log2n)];
        store_env(a, col * N + n, sqrtf(z.x * z.x + z.y * z.y) * inv_n, local_max);
    }
    publish_max(a, local_max);
}

// Any N: y = Im x_a = sum_k q[k] x[(n - k) mod N]; env = sqrt(x^2 + y^2).
// LDS holds the column twice (no modulo in the sum) and q.
__global__ __launch_bounds__(256) void env_direct_kernel(EnvArgs a)
{
    extern __shared__ float sf[];
    const int N = a.N, T = blockDim.x, t = threadIdx.x;
    float *x2 = sf;            // [2N]: x2[i] = x[i mod N]
    float *q = sf + 2 * N;     // [N]
    const long col = blockIdx.x;
    const float *x = a.img + col * N;
    for (int i = t; i < N; i += T) {
        const float v = x[i];
        x2[i] = v;
        x2[i + N] = v;
        q[i] = a.q[i];
    }
    __syncthreads();
    float local_max = 0.f;
    for (int n = t; n < N; n += T) {
        // x[(n - k) mod N] = x2[n - k + N] for 0 <= k < N
        float y = 0.f;
        for (int k = 0; k < N; ++k) y = fmaf(q[k], x2[n - k + N], y);
        const float xv = x2[n];
        store_env(a, col * N + n, sqrtf(fmaf(xv, xv, y * y)), local_max);
    }
    publish_max(a, local_max);
}

// ---------------------------------------------------------------------------
// Register FFT (64 <= N = 64 M <= 1024): sample n = M l + r lives in lane l,
// register r.  X[k1 + 64 k2] = sum_r W_M^{r k2} W_N^{r k1} [sum_l x[M l + r] W_64^{l k1}].
// ---------------------------------------------------------------------------
// Value of lane l ^ m (m a power of two, constant after unrolling).  Lane
// distances 1 and 2 move through DPP quad permutes and 32 through the gfx950
// half-swap (permlane32_swap: lanes 32-63 of the first operand trade places
// with lanes 0-31 of the second), all in the VALU; 4, 8 and 16 go through the
// LDS crossbar (ds_bpermute), so both pipes share the exchanges.
__device__ inline float xor_lane(float x, int m, int lane)
{
    const int xi = __float_as_int(x);
    if (m == 1) return __int_as_float(__builtin_amdgcn_update_dpp(0, xi, 0xB1, 0xF, 0xF, false));
    if (m == 2) return __int_as_float(__builtin_amdgcn_update_dpp(0, xi, 0x4E, 0xF, 0xF, false));
    if (m == 32) {
        const auto r = __builtin_amdgcn_permlane32_swap(xi, xi, false, false);
        return __int_as_float(lane < 32 ? r[1] : r[0]);
    }
    return __shfl_xor(x, m, 64);
}

__device__ inline float2 shfl_xor2(float2 v, int m, int lane)
{
    return make_float2(xor_lane(v.x, m, lane), xor_lane(v.y, m, lane));
}

// 64-point DIF across lanes for each register (sign -1: forward); lane l ends
// with the bin bitrev6(l).  Pairs (l, l ^ d): lower l gets v + p, upper gets
// (p - v) W_{2d}^{l mod d}, both as (sigma v + p) w with sigma = +-1 and w = 1
// on the lower lane (no selects).  tw_l[s] = W_{2d}^{l mod d} for every lane.
template <int M>
__device__ inline void lane_dif(float2 (&v)[M], const float2 *tw_l, int lane)
{
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        const int d = 32 >> s;
        const bool up = (lane & d) != 0;
        const float sg = up ? -1.f : 1.f;
        const float2 w = up ? tw_l[s] : make_float2(1.f, 0.f);
#pragma unroll
        for (int r = 0; r < M; ++r) {
            const float2 p = shfl_xor2(v[r], d, lane);
            v[r] = cmul(make_float2(fmaf(sg, v[r].x, p.x), fmaf(sg, v[r].y, p.y)), w);
        }
    }
}

// 64-point inverse DIT across lanes from bit-reversed bins back to natural
// order (sign +1): lower l gets v + W p, upper gets p - W v, W = conj(W_{2d}^{l mod d}).
// The upper lane multiplies its own value by W before the exchange, so both
// results are sigma u + p with u the lane's (weighted) value, sigma = +-1.
template <int M>
__device__ inline void lane_dit_inv(float2 (&v)[M], const float2 *tw_l, int lane)
{
#pragma unroll
    for (int s = 5; s >= 0; --s) {
        const int d = 32 >> s;
        const bool up = (lane & d) != 0;
        const float sg = up ? -1.f : 1.f;
        const float2 w = up ? make_float2(tw_l[s].x, -tw_l[s].y) : make_float2(1.f, 0.f);
#pragma unroll
        for (int r = 0; r < M; ++r) {
            const float2 u = cmul(v[r], w);
            const float2 p = shfl_xor2(u, d, lane);
            v[r] = make_float2(fmaf(sg, u.x, p.x), fmaf(sg, u.y, p.y));
        }
    }
}

// In-register M-point DFT, natural order in and out; sign -1 forward, +1 inverse.
template <int M>
__device__ inline void reg_fft(float2 (&v)[M], const float2 *wm, float sign)
{
    if constexpr (M > 1) {
        // bit-reverse permutation, then iterative DIT
        constexpr int L = M == 2 ? 1 : M == 4 ? 2 : M == 8 ? 3 : 4;
#pragma unroll
        for (int i = 0; i < M; ++i) {
            int j = 0;
#pragma unroll
            for (int b = 0; b < L; ++b) j |= ((i >> b) & 1) << (L - 1 - b);
            if (j > i) {
                const float2 t = v[i];
                v[i] = v[j];
                v[j] = t;
            }
        }
#pragma unroll
        for (int h = 1; h < M; h <<= 1) {
#pragma unroll
            for (int i0 = 0; i0 < M; i0 += 2 * h) {
#pragma unroll
                for (int j = 0; j < h; ++j) {
                    const float2 w0 = wm[j * (M / (2 * h))];
                    const float2 w = make_float2(w0.x, sign < 0.f ? w0.y : -w0.y);
                    const float2 t = cmul(v[i0 + j + h], w);
                    const float2 u = v[i0 + j];
                    v[i0 + j] = make_float2(u.x + t.x, u.y + t.y);
                    v[i0 + j + h] = make_float2(u.x - t.x, u.y - t.y);
                }
            }
        }
    }
}

// Two real columns per wavefront, 8 per 256-thread workgroup.  The Hilbert
// transform H is linear with a real kernel, so for z = x1 + j x2 the inverse
// DFT of -j sgn(k) DFT(z) (sgn = 0 at DC and Nyquist, +1 for positive and -1
// for negative frequencies) is H{x1} + j H{x2}, and each envelope is
// |x_a| = sqrt(x^2 + H{x}^2): the analytic signal of both columns for one
// complex FFT pair (half the work of one pair per column).
template <int M>
__global__ __launch_bounds__(256) void env_fft_reg_kernel(EnvArgs a)
{
    constexpr int N = 64 * M;
    const int lane = threadIdx.x & 63;
    const long col = ((long)blockIdx.x * 4 + (threadIdx.x >> 6)) * 2;
    float local_max = 0.f;
    if (col < a.n_cols) {
        const bool has2 = col + 1 < a.n_cols;
        const float *x = a.img + col * N + M * lane;
        float x1[M], x2[M];
        float2 v[M];
#pragma unroll
        for (int r = 0; r < M; ++r) {
            x1[r] = x[r];
            x2[r] = has2 ? x[N + r] : 0.f;
            v[r] = make_float2(x1[r], x2[r]);
        }
        float2 twl[6];
#pragma unroll
        for (int s = 0; s < 6; ++s) twl[s] = a.tw_lane[s * 64 + lane];
        lane_dif<M>(v, twl, lane);
        // lane holds bin k1 = bitrev6(lane) of each register's 64-point DFT
        const float2 *tm = a.tw_mid + lane * M;
#pragma unroll
        for (int r = 0; r < M; ++r) v[r] = cmul(v[r], tm[r]);
        reg_fft<M>(v, a.wm, -1.f);
        // -j sgn(k) on Z[k1 + 64 k2] (register k2): -j s (a + j b) = s (b - j a)
        const int k1 = (int)(__brev((unsigned)lane) >> 26);
#pragma unroll
        for (int k2 = 0; k2 < M; ++k2) {
            const int k = k1 + 64 * k2;
            const float sg = (k == 0 || 2 * k == N) ? 0.f : (2 * k < N ? 1.f : -1.f);
            v[k2] = make_float2(sg * v[k2].y, -sg * v[k2].x);
        }
        reg_fft<M>(v, a.wm, 1.f);
#pragma unroll
        for (int r = 0; r < M; ++r) v[r] = cmul(v[r], make_float2(tm[r].x, -tm[r].y));
        lane_dit_inv<M>(v, twl, lane);
        const float inv_n = 1.f / (float)N;
#pragma unroll
        for (int r = 0; r < M; ++r) {
            const float h1 = v[r].x * inv_n, h2 = v[r].y * inv_n;
            store_env(a, col * N + M * lane + r,
                      __builtin_amdgcn_sqrtf(fmaf(x1[r], x1[r], h1 * h1)), local_max);
            if (has2)
                store_env(a, (col + 1) * N + M * lane + r,
                          __builtin_amdgcn_sqrtf(fmaf(x2[r], x2[r], h2 * h2)), local_max);
        }
    }
    publish_max(a, local_max);
}

__global__ __launch_bounds__(256) void env_iq_kernel(EnvArgs a)
{
    const long total = a.n_cols * a.N;
    float local_max = 0.f;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < total; i += (long)gridDim.x * 256) {
        const float2 z = reinterpret_cast<const float2 *>(a.img)[i];
        store_env(a, i, sqrtf(fmaf(z.x, z.x, z.y * z.y)), local_max);
    }
    publish_max(a, local_max);
}

// One workgroup: img_max = max of part_max[0 .. n) (fixed order per thread,
// then a tree over threads).
__global__ __launch_bounds__(256) void env_reduce_kernel(const float *part_max, long n,
                                                         float *img_max)
{
    __shared__ float s[256];
    float m = 0.f;
    for (long i = threadIdx.x; i < n; i += 256) m = fmaxf(m, part_max[i]);
    s[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] = fmaxf(s[threadIdx.x], s[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *img_max = s[0];
}

__global__ __launch_bounds__(256) void env_compress_kernel(EnvArgs a)
{
    const long total = a.n_cols * a.N;
    const float ref = *a.img_max;
    const float inv_ref = ref > 0.f ? 1.f / ref : 0.f;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < total; i += (long)gridDim.x * 256) {
        const float env = a.out[i];
        float y;
        if (ref > 0.f) {
            y = compress_value(env, a.compress, inv_ref, a.param);
        } else {   // all-zero image
            y = a.compress == BF_COMPRESS_LOG ? -a.param : 0.f;
        }
        a.out[i] = y;
    }
}

}  // namespace bf

using namespace bf;

struct bf_env_s {
    uint32_t magic = 0xBFE7E701u;
    long n_cols = 0;
    int N = 0, iq = 0, log2n = -1;
    long n_parts = 0;
    int reg_m = 0;                // register FFT: M = N / 64 (0: not used)
    float2 wm[8] = {};
    float2 *d_tw = nullptr;
    float2 *d_tw_lane = nullptr;  // [6][64]
    float2 *d_tw_mid = nullptr;   // [64][M]
    float *d_q = nullptr;
    float *d_part = nullptr;      // [n_parts] per-workgroup maxima, then the maximum
    ~bf_env_s()
    {
        if (d_tw) (void)hipFree(d_tw);
        if (d_tw_lane) (void)hipFree(d_tw_lane);
        if (d_tw_mid) (void)hipFree(d_tw_mid);
        if (d_q) (void)hipFree(d_q);
        if (d_part) (void)hipFree(d_part);
    }
};

static bool live(bf_env e) { return e && e->magic == 0xBFE7E701u; }

extern "C" {

int bf_env_create(int64_t n_cols, int32_t n, int32_t iq, bf_env *out)
{
    clear_err();
    if (!out) return fail(BF_ERR_NULL, "out is NULL");
    *out = nullptr;
    if (n_cols < 1) return fail(BF_ERR_SHAPE, "n_cols=%lld < 1", (long long)n_cols);
    if (n < 1 || n > ENV_MAX_N) return fail(BF_ERR_SHAPE, "n=%d not in [1,%d]", n, ENV_MAX_N);
    if (iq != 0 && iq != 1) return fail(BF_ERR_UNSUPPORTED, "iq must be 0 or 1");
    if (n_cols >= (int64_t(1) << 31) || n_cols * n * (iq ? 2 : 1) >= (int64_t(1) << 31))
        return fail(BF_ERR_TOO_LARGE, "image exceeds 2^31 elements");
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
    bf_env e = new bf_env_s();
    e->n_cols = n_cols;
    e->N = n;
    e->iq = iq;
    // register FFT for 64 <= N <= 1024 (powers of two)
    if (!iq && (n & (n - 1)) == 0 && n >= 64 && n <= 1024) e->reg_m = n / 64;
    // workgroups of the envelope pass: one per column, four columns per
    // workgroup (register FFT), or the grid-stride launch of the IQ path
    e->n_parts = iq ? std::min<long>((n_cols * n + 255) / 256, 8192)
                    : e->reg_m ? (n_cols + 7) / 8 : n_cols;
    hipError_t err = hipMalloc(&e->d_part, (e->n_parts + 1) * sizeof(float));
    if (err == hipSuccess && !iq) {
        if ((n & (n - 1)) == 0 && n >= 2) {
            int l = 0;
            while ((1 << l) < n) ++l;
            e->log2n = l;
            // stage-major: stage len (h = len / 2) at offset h - 1, pos < h
            std::vector<float2> tw(n - 1);
            for (int h = 1; h < n; h <<= 1)
                for (int pos = 0; pos < h; ++pos) {
                    const double ph = -M_PI * pos / h;      // -2 pi pos / len
                    tw[h - 1 + pos] = make_float2((float)cos(ph), (float)sin(ph));
                }
            err = hipMalloc(&e->d_tw, tw.size() * sizeof(float2));
            if (err == hipSuccess)
                err = hipMemcpy(e->d_tw, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice);
            if (err == hipSuccess && e->reg_m) {
                const int M = e->reg_m;
                // lane stage twiddles W_{2d}^{l mod d}, d = 32 >> s
                std::vector<float2> tl(6 * 64), tm((size_t)64 * M);
                for (int st = 0; st < 6; ++st) {
                    const int d = 32 >> st;
                    for (int l = 0; l < 64; ++l) {
                        const double ph = -M_PI * (l % d) / d;
                        tl[st * 64 + l] = make_float2((float)cos(ph), (float)sin(ph));
                    }
                }
                // W_N^{r bitrev6(l)}
                for (int l = 0; l < 64; ++l) {
                    int br = 0;
                    for (int b = 0; b < 6; ++b) br |= ((l >> b) & 1) << (5 - b);
                    for (int r = 0; r < M; ++r) {
                        const double ph = -2.0 * M_PI * (double)((long)r * br % n) / n;
                        tm[(size_t)l * M + r] = make_float2((float)cos(ph), (float)sin(ph));
                    }
                }
                for (int j = 0; j < M / 2; ++j) {
                    const double ph = -2.0 * M_PI * j / M;
                    e->wm[j] = make_float2((float)cos(ph), (float)sin(ph));
                }
                err = hipMalloc(&e->d_tw_lane, tl.size() * sizeof(float2));
                if (err == hipSuccess) err = hipMalloc(&e->d_tw_mid, tm.size() * sizeof(float2));
                if (err == hipSuccess)
                    err = hipMemcpy(e->d_tw_lane, tl.data(), tl.size() * sizeof(float2),
                                    hipMemcpyHostToDevice);
                if (err == hipSuccess)
                    err = hipMemcpy(e->d_tw_mid, tm.data(), tm.size() * sizeof(float2),
                                    hipMemcpyHostToDevice);
            }
        } else {
            // q[k] = Im IDFT(h)[k] = (1/N) sum_k' h[k'] sin(2 pi k' k / N)
            std::vector<float> q(n);
            for (int k = 0; k < n; ++k) {
                double s = 0.0;
                // weight 2 for 0 < k' < N/2; DC and Nyquist add sin(0) = sin(pi k) = 0
                for (int kk = 1; 2 * kk < n; ++kk)
                    s += 2.0 * sin(2.0 * M_PI * (double)((long)kk * k % n) / n);
                q[k] = (float)(s / n);
            }
            err = hipMalloc(&e->d_q, n * sizeof(float));
            if (err == hipSuccess)
                err = hipMemcpy(e->d_q, q.data(), n * sizeof(float), hipMemcpyHostToDevice);
        }
    }
    if (err != hipSuccess) {
        delete e;
        return hip_fail(err, "envelope tables");
    }
    *out = e;
    return BF_OK;
}

int bf_env_destroy(bf_env e)
{
    clear_err();
    if (!e) return BF_OK;
    if (!live(e)) return fail(BF_ERR_STATE, "not a live envelope plan");
    (void)hipDeviceSynchronize();
    e->magic = 0;
    delete e;
    return BF_OK;
}

int bf_envelope(bf_env e, const float *img, float *out, int32_t compress, double ref,
                double param, void *stream)
{
    clear_err();
    if (!e) return fail(BF_ERR_NULL, "envelope plan is NULL");
    if (!live(e)) return fail(BF_ERR_STATE, "not a live envelope plan");
    if (!img || !out) return fail(BF_ERR_NULL, "img and out must be non-NULL");
    if (compress < BF_COMPRESS_NONE || compress > BF_COMPRESS_POWER)
        return fail(BF_ERR_UNSUPPORTED, "unknown compression %d", compress);
    if (!isfinite(ref)) return fail(BF_ERR_GEOMETRY, "ref must be finite");
    if (compress != BF_COMPRESS_NONE && !(isfinite(param) && param > 0.0))
        return fail(BF_ERR_GEOMETRY, "param must be finite and > 0");
    EnvArgs a;
    a.img = img;
    a.out = out;
    a.tw = e->d_tw;
    a.tw_lane = e->d_tw_lane;
    a.tw_mid = e->d_tw_mid;
    for (int j = 0; j < 8; ++j) a.wm[j] = e->wm[j];
    a.q = e->d_q;
    a.part_max = e->d_part;
    a.img_max = e->d_part + e->n_parts;
    a.n_cols = e->n_cols;
    a.N = e->N;
    a.log2n = e->log2n;
    a.compress = compress;
    a.ref = (float)ref;
    a.param = (float)param;
    // (a ref below 2^-128 keeps a finite reciprocal: env = 0 still maps to 0)
    a.inv_ref = ref > 0.0 ? (float)std::min(1.0 / ref, 3.4028234663852886e38) : 0.f;
    hipStream_t s = (hipStream_t)stream;
    const bool two_pass = compress != BF_COMPRESS_NONE && ref <= 0.0;
    const long total = e->n_cols * e->N;
    const unsigned eblocks = (unsigned)std::min<long>((total + 255) / 256, 8192);
    if (e->iq) {
        hipLaunchKernelGGL(env_iq_kernel, dim3(eblocks), dim3(256), 0, s, a);
    } else if (e->reg_m) {
        const dim3 g((unsigned)((e->n_cols + 7) / 8)), b(256);
        switch (e->reg_m) {
            case 1: hipLaunchKernelGGL(env_fft_reg_kernel<1>, g, b, 0, s, a); break;
            case 2: hipLaunchKernelGGL(env_fft_reg_kernel<2>, g, b, 0, s, a); break;
            case 4: hipLaunchKernelGGL(env_fft_reg_kernel<4>, g, b, 0, s, a); break;
            case 8: hipLaunchKernelGGL(env_fft_reg_kernel<8>, g, b, 0, s, a); break;
            default: hipLaunchKernelGGL(env_fft_reg_kernel<16>, g, b, 0, s, a); break;
        }
    } else if (e->log2n > 0) {
        const int T = std::min(256, std::max(64, e->N / 2));
        hipLaunchKernelGGL(env_fft_kernel, dim3((unsigned)e->n_cols), dim3(T),
                           (size_t)e->N * 8, s, a);
    } else {
        hipLaunchKernelGGL(env_direct_kernel, dim3((unsigned)e->n_cols), dim3(256),
                           (size_t)3 * e->N * sizeof(float), s, a);
    }
    if (two_pass) {
        hipLaunchKernelGGL(env_reduce_kernel, dim3(1), dim3(256), 0, s, e->d_part, e->n_parts,
                           e->d_part + e->n_parts);
        hipLaunchKernelGGL(env_compress_kernel, dim3(eblocks), dim3(256), 0, s, a);
    }
    hipError_t err = hipGetLastError();
    return err == hipSuccess ? BF_OK : hip_fail(err, "envelope launch");
}

}  // extern "C"
