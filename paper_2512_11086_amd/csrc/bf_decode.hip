// bf_decode.hip -- Hadamard aperture decoding on gfx950 (Sec. VII-E).
//
//   e[i][j][t] = sum_k H[k][i] * rf[k][j][t]
//
// For every channel j this is a small dense product E_j = H^T R_j with
// M = K = n_tx (<= 256) and N = samples.  It is HBM bound (2 bytes in, 4 out
// per element) but runs on the int8 matrix cores so that the arithmetic is
// exact and nearly free: each int16 sample x is split into two int8 halves,
//   x = 256 * hi + lo + 128,   hi = x >> 8,   lo = (x & 0xFF) - 128,
// so  E = 256 * (H^T hi) + (H^T lo) + 128 * colsum(H)  with int32
// accumulation (|E| <= 256 * 32768 < 2^24, so FP32 output is exact too).
//
// Wavefront work item: one channel j and 64 consecutive samples.  Lane l
// owns the sample pair t = t0 + 2 (l % 32), t + 1 and the K half l / 32; it
// loads those two samples (one 32-bit load) for 16 transmits per 32-wide K
// block, so every load instruction reads two contiguous 128-byte runs.  The
// byte-sliced registers form the B operand of v_mfma_i32_32x32x32_i8 for the
// even-sample and the odd-sample 32x32 output tiles: the "reorder" of the
// paper (transmits contiguous per sample) happens in registers instead of in
// a separate pass.  The A operand (H^T, shared by every wavefront) is staged
// once per workgroup in LDS in operand order.
//
// Operand K order: the instruction pairs K slot q of lane half g in A with the
// same slot of B.  Both operands are filled with the same slot -> transmit
// mapping (k = 32 kb + 16 g + q), so the product is exact whatever order the
// hardware assigns to the slots.  The output tile is read back with the 32x32
// accumulator layout (row 8 (r/4) + 4 g + r % 4, column l % 32).
#include "bf_common.h"

namespace bf {

__device__ inline uint32_t load_pair(const int16_t *rf, long row, int t, int S, bool even_S)
{
    // Samples t and t+1 of one trace packed as (x[t] | x[t+1] << 16).
    // (global view: the persistent kernel reads rf from a pointer table)
    const gptr<int16_t> p = as_global(rf + row * (long)S + t);
    if (even_S) {
        return (t < S) ? *reinterpret_cast<gptr<uint32_t>>(p) : 0u;
    }
    uint32_t a = (t < S) ? (uint16_t)p[0] : 0u;
    uint32_t b = (t + 1 < S) ? (uint16_t)p[1] : 0u;
    return a | (b << 16);
}

__device__ inline uint32_t pick_bytes(uint32_t d0, uint32_t d1, uint32_t d2, uint32_t d3, int sh)
{
    return ((d0 >> sh) & 0xFFu) | (((d1 >> sh) & 0xFFu) << 8) | (((d2 >> sh) & 0xFFu) << 16) |
           (((d3 >> sh) & 0xFFu) << 24);
}

__device__ inline uint32_t f32_to_bf16_rne(float f)
{
    uint32_t b = __float_as_uint(f);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return b >> 16;
}

template <int OT>
__device__ inline void store_pair(void *e, long idx, int v0, int v1, bool two, bool even_S)
{
    // (with an even sample count the pair is 8-byte aligned: one 8-byte store
    // per lane, so each half-wavefront writes 256 contiguous bytes in one
    // instruction)
    if constexpr (OT == ET_F32 || OT == ET_I32) {
        const uint32_t u0 = OT == ET_F32 ? __float_as_uint((float)v0) : (uint32_t)v0;
        const uint32_t u1 = OT == ET_F32 ? __float_as_uint((float)v1) : (uint32_t)v1;
        const gptr_mut<uint32_t> p = as_global_mut(static_cast<uint32_t *>(e) + idx);
        if (two && even_S) {
            *reinterpret_cast<gptr_mut<unsigned long long>>(p) =
                (unsigned long long)u0 | ((unsigned long long)u1 << 32);
        } else {
            p[0] = u0;
            if (two) p[1] = u1;
        }
    } else {
        const gptr_mut<uint16_t> p = as_global_mut(static_cast<uint16_t *>(e) + idx);
        uint32_t b0 = f32_to_bf16_rne((float)v0), b1 = f32_to_bf16_rne((float)v1);
        if (two && even_S) {
            *reinterpret_cast<gptr_mut<uint32_t>>(p) = b0 | (b1 << 16);
        } else {
            p[0] = (uint16_t)b0;
            if (two) p[1] = (uint16_t)b1;
        }
    }
}

// Decode of one (channel, 64-sample chunk) work item by one wavefront.
// lds_A holds KB*KB operand fragments of 64 lanes x 16 bytes; lds_cs the
// padded column sums.
template <int KB, int OT>
__device__ inline void decode_item(const DecodeArgs &a, const v4i *lds_A, const int *lds_cs,
                                   int j, int chunk, int lane)
{
    const int n = lane & 31, g = lane >> 5;
    const int t = chunk * 64 + 2 * n;
    const bool even_S = (a.S & 1) == 0;

    v4i bhe[KB], bho[KB], ble[KB], blo[KB];
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            uint32_t d[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = kb * 32 + 16 * g + 4 * c + u;
                d[u] = (k < a.n_tx) ? load_pair(a.rf, (long)k * a.n_ch + j, t, a.S, even_S) : 0u;
            }
            bhe[kb][c] = (int)pick_bytes(d[0], d[1], d[2], d[3], 8);
            bho[kb][c] = (int)pick_bytes(d[0], d[1], d[2], d[3], 24);
            ble[kb][c] = (int)(pick_bytes(d[0], d[1], d[2], d[3], 0) ^ 0x80808080u);
            blo[kb][c] = (int)(pick_bytes(d[0], d[1], d[2], d[3], 16) ^ 0x80808080u);
        }
    }

#pragma unroll 1
    for (int mt = 0; mt < KB; ++mt) {
        v16i ce = {0}, co = {0};
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            const v4i A = lds_A[(mt * KB + kb) * 64 + lane];
            ce = __builtin_amdgcn_mfma_i32_32x32x32_i8(A, bhe[kb], ce, 0, 0, 0);
            co = __builtin_amdgcn_mfma_i32_32x32x32_i8(A, bho[kb], co, 0, 0, 0);
        }
        ce = ce << 8;
        co = co << 8;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            const v4i A = lds_A[(mt * KB + kb) * 64 + lane];
            ce = __builtin_amdgcn_mfma_i32_32x32x32_i8(A, ble[kb], ce, 0, 0, 0);
            co = __builtin_amdgcn_mfma_i32_32x32x32_i8(A, blo[kb], co, 0, 0, 0);
        }
        if (t < a.S) {
            const bool two = t + 1 < a.S;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int m = mt * 32 + 8 * (r >> 2) + 4 * g + (r & 3);
                if (m < a.n_tx) {
                    const int corr = 128 * lds_cs[m];
                    store_pair<OT>(a.e, ((long)m * a.n_ch + j) * a.S + t, ce[r] + corr,
                                   co[r] + corr, two, even_S);
                }
            }
        }
    }
}

template <int KB>
__device__ inline void stage_operands(const DecodeArgs &a, v4i *lds_A, int *lds_cs)
{
    constexpr int KP = KB * 32;
    for (int idx = threadIdx.x; idx < KB * KB * 64; idx += blockDim.x) {
        const int frag = idx >> 6, l = idx & 63;
        const int mt = frag / KB, kb = frag % KB;
        lds_A[idx] = *reinterpret_cast<gptr<v4i>>(as_global(a.At) + (long)(mt * 32 + (l & 31)) * KP +
                                                  kb * 32 + 16 * (l >> 5));
    }
    for (int m = threadIdx.x; m < KP; m += blockDim.x) lds_cs[m] = as_global(a.colsum)[m];
    __syncthreads();
}

// grid: (ceil(n_chunks / 4), n_ch); block: 256 = 4 wavefronts, one chunk each.
template <int KB, int OT>
__global__ __launch_bounds__(256) void decode_mfma_kernel(DecodeArgs a, int n_chunks)
{
    __shared__ v4i lds_A[KB * KB * 64];
    __shared__ int lds_cs[KB * 32];
    stage_operands<KB>(a, lds_A, lds_cs);
    const int chunk = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (chunk >= n_chunks) return;
    decode_item<KB, OT>(a, lds_A, lds_cs, blockIdx.y, chunk, threadIdx.x & 63);
}

// Persistent form for a batch of frames of one 32-wide K-block class: the
// workgroups stride over the (frame, channel, 4 chunks) items (items of one
// class cost the same, so a static stride balances them without a queue: no
// atomic and no barrier per item); the operand tables are restaged in LDS
// only when the frame changes (items are grouped by frame, and a
// workgroup's items come in increasing order).
// (register caps: the occupancy of the single-frame kernel of the same K
// blocks; without them the item loop took up to 305 registers, one
// wavefront per SIMD for 128 transmits)
template <int KB> struct DecWaves {
    static constexpr int value = KB == 1 ? 6 : KB == 2 ? 4 : 2;
};
template <int KB, int OT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(DecWaves<KB>::value))) void decode_persistent_kernel(const FrameDec *__restrict__ frames,
                                                                const int2 *__restrict__ items,
                                                                int n_items, int *counter,
                                                                void *const *__restrict__ rf_ptrs)
{
    (void)counter;
    __shared__ v4i lds_A[KB * KB * 64];
    __shared__ int lds_cs[KB * 32];
    int staged = -1;
    for (int item = blockIdx.x; item < n_items; item += gridDim.x) {
        // (a compiler-only memory barrier: the operand fragments are read from
        // LDS per item, as in the single-frame kernel, instead of being held
        // in registers across items, which would cost occupancy)
        asm volatile("" ::: "memory");
        const int fr = __builtin_amdgcn_readfirstlane(items[item].x);
        const int wy = __builtin_amdgcn_readfirstlane(items[item].y);
        DecodeArgs a = frames[fr].a;
        a.rf = static_cast<const int16_t *>(rf_ptrs[fr]);
        if (fr != staged) {
            if (staged >= 0) __syncthreads();     // every wavefront is done with the old tables
            stage_operands<KB>(a, lds_A, lds_cs);
            staged = fr;
        }
        const int n_chunks = (a.S + 63) / 64;
        const int n_cg = (n_chunks + 3) / 4;
        const int j = wy / n_cg;
        const int chunk = (wy % n_cg) * 4 + (threadIdx.x >> 6);
        if (chunk < n_chunks) decode_item<KB, OT>(a, lds_A, lds_cs, j, chunk, threadIdx.x & 63);
    }
}

template <int KB, int OT>
static hipError_t launch_dec_persistent(const DecLaunch &p, hipStream_t s)
{
    hipLaunchKernelGGL((decode_persistent_kernel<KB, OT>), dim3(p.grid), dim3(256), 0, s,
                       p.frames, p.items, p.n_items, p.counter, p.rf_ptrs);
    return hipGetLastError();
}

template <int OT>
static hipError_t launch_dec_persistent_kb(const DecLaunch &p, hipStream_t s)
{
    switch (p.kb) {
        case 1: return launch_dec_persistent<1, OT>(p, s);
        case 2: return launch_dec_persistent<2, OT>(p, s);
        case 3: return launch_dec_persistent<3, OT>(p, s);
        case 4: return launch_dec_persistent<4, OT>(p, s);
        case 5: return launch_dec_persistent<5, OT>(p, s);
        case 6: return launch_dec_persistent<6, OT>(p, s);
        case 7: return launch_dec_persistent<7, OT>(p, s);
        case 8: return launch_dec_persistent<8, OT>(p, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_decode_persistent(const DecLaunch &p, hipStream_t s)
{
    switch (p.ot) {
        case ET_F32: return launch_dec_persistent_kb<ET_F32>(p, s);
        case ET_BF16: return launch_dec_persistent_kb<ET_BF16>(p, s);
        case ET_I32: return launch_dec_persistent_kb<ET_I32>(p, s);
        default: return hipErrorInvalidValue;
    }
}

// FP32 FMA decode (precision-study variant): one lane per (j, t), 32 outputs
// per pass; the +-1 coefficients are wave-uniform scalar loads.
template <int OT>
__global__ __launch_bounds__(256) void decode_fma_kernel(DecodeArgs a, int ip)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    const int j = blockIdx.y;
    const int i0 = blockIdx.z * 32;
    if (t >= a.S) return;
    float acc[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) acc[q] = 0.f;
    for (int k = 0; k < a.n_tx; ++k) {
        const float x = (float)a.rf[((long)k * a.n_ch + j) * a.S + t];
        const float *h = a.Hf + (long)k * ip + i0;
#pragma unroll
        for (int q = 0; q < 32; ++q) acc[q] = fmaf(h[q], x, acc[q]);
    }
    for (int q = 0; q < 32 && i0 + q < a.n_tx; ++q) {
        const long idx = ((long)(i0 + q) * a.n_ch + j) * a.S + t;
        if constexpr (OT == ET_F32) {
            static_cast<float *>(a.e)[idx] = acc[q];
        } else if constexpr (OT == ET_I32) {
            static_cast<int *>(a.e)[idx] = (int)acc[q];
        } else {
            static_cast<uint16_t *>(a.e)[idx] = (uint16_t)f32_to_bf16_rne(acc[q]);
        }
    }
}

template <int KB, int OT>
static hipError_t launch_mfma(const DecodeArgs &a, hipStream_t s)
{
    const int n_chunks = (a.S + 63) / 64;
    dim3 grid((n_chunks + 3) / 4, a.n_ch);
    hipLaunchKernelGGL((decode_mfma_kernel<KB, OT>), grid, dim3(256), 0, s, a, n_chunks);
    return hipGetLastError();
}

template <int OT>
static hipError_t launch_mfma_kb(const DecodeArgs &a, int kb, hipStream_t s)
{
    switch (kb) {
        case 1: return launch_mfma<1, OT>(a, s);
        case 2: return launch_mfma<2, OT>(a, s);
        case 3: return launch_mfma<3, OT>(a, s);
        case 4: return launch_mfma<4, OT>(a, s);
        case 5: return launch_mfma<5, OT>(a, s);
        case 6: return launch_mfma<6, OT>(a, s);
        case 7: return launch_mfma<7, OT>(a, s);
        case 8: return launch_mfma<8, OT>(a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_decode_mfma(const DecodeArgs &a, int kb, int etype, hipStream_t s)
{
    switch (etype) {
        case ET_F32: return launch_mfma_kb<ET_F32>(a, kb, s);
        case ET_BF16: return launch_mfma_kb<ET_BF16>(a, kb, s);
        case ET_I32: return launch_mfma_kb<ET_I32>(a, kb, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_decode_fma(const DecodeArgs &a, int etype, hipStream_t s)
{
    const int ip = 32 * ((a.n_tx + 31) / 32);
    dim3 grid((a.S + 255) / 256, a.n_ch, ip / 32);
    switch (etype) {
        case ET_F32: hipLaunchKernelGGL((decode_fma_kernel<ET_F32>), grid, dim3(256), 0, s, a, ip); break;
        case ET_BF16: hipLaunchKernelGGL((decode_fma_kernel<ET_BF16>), grid, dim3(256), 0, s, a, ip); break;
        case ET_I32: hipLaunchKernelGGL((decode_fma_kernel<ET_I32>), grid, dim3(256), 0, s, a, ip); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace bf
