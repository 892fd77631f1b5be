// bf_common.h -- internal definitions shared by the libbf HIP sources
// (kernel argument blocks, device helpers).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bf {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// Element type of decoded data.  ET_CF32 is complex FP32 (re, im) pairs of IQ
// plans; the DAS kernels then accumulate complex sums.
// ET_RF16: the kernel reads int16 RF channel data and decodes each staged tap
// itself (decode fused into DAS); the rest of the kernel sees FP32 samples.
enum EType { ET_F32 = 0, ET_BF16 = 1, ET_I32 = 2, ET_CF32 = 3, ET_RF16 = 4 };
enum Interp { IN_NEAREST = 0, IN_LINEAR = 1, IN_CUBIC = 2 };

// ---------------------------------------------------------------------------
// Decode
// ---------------------------------------------------------------------------
struct DecodeArgs {
    const int16_t *rf;     // [n_tx][n_ch][S]
    void *e;               // [n_tx][n_ch][S], type per template
    const int8_t *At;      // [KP][KP] with KP = 32*KB: At[m][k] = H[k][m], zero padded
    const int *colsum;     // [KP]: sum_k H[k][m], zero padded
    const float *Hf;       // [n_tx][IP] float copy of H (FMA path), IP = 32*ceil(n_tx/32)
    int n_tx, n_ch, S;
};

// One frame of a batch for the persistent decode kernel (rf comes from the
// per-launch pointer table).
struct FrameDec {
    DecodeArgs a;
};

struct DecLaunch {
    int kb, ot, grid;
    const FrameDec *frames;
    const int2 *items;      // (frame, channel * chunk_groups + chunk_group)
    int n_items;
    int *counter;
    void *const *rf_ptrs;
};

// ---------------------------------------------------------------------------
// DAS
// ---------------------------------------------------------------------------
// Output grid in the array frame, shifted by the lateral reference (cx, cy)
// so that FP32 lateral coordinates stay small.  Point (ix, iy, iz) is
//   org + ix * ax + iy * ay + iz * az.
struct Grid {
    double org[3], ax[3], ay[3], az[3];
    int nx, ny, nz;
};

struct DasArgs {
    const void *e;          // decoded data [n_tx][n_ch][S]
    float *out;             // [ny][nx][nz]
    const float *tx_x;      // [n_tx] x of decoded transmit column (relative to cx)
    const float *rx_c;      // [n_ch] x (FORCES) or y (HERCULES) of channel (relative)
    const float *grad_out;  // adjoint: dL/dout
    float *grad_e;          // adjoint: dL/de (nullable)
    double *partial;        // adjoint: per-block partial sums of grad_c
    int n_tx, n_ch, S;
    Grid g;
    double k;               // fs / c
    double t0fs;            // t0 * fs
    double c;               // sound speed
    float f2;               // F#^2 (0 disables apodization)
    int lx, ly, lz;         // log2 of the wavefront tile along x, y, z (sum 6)
    int tiles_x, tiles_y, tiles_z;
    int n_waves;            // tiles_x * tiles_y * tiles_z
    int groups;             // channel groups (blockIdx.y); > 1 writes partial images
    float *part;            // [groups][ny][nx][nz] partial images when groups > 1
    float *const *out_ref;  // if set, the output pointer is read from here (graph replay)
    const float2 *hann_tab; // [HANN_N + 1] (base, slope) of W over u^2 in [0, 1/4]
    int cx;                 // IQ data: e, out and part hold (re, im) pairs
    float rot;              // IQ: fd / fs, revolutions of carrier phase per sample
    double rot_d;           // the same in FP64 (per-lane phase origin)
    double div_f;           // HERCULES diverging wave: source depth f > 0 (0: plane wave)
    float zf;               // VLS: depth of the virtual line sources
    const float2 *tx_sc;    // TPW: [n_tx] (sin theta, cos theta - 1)
    const float *hf;        // ET_RF16: H[k][i] at hf[k * hf_ld + i] (+-1 as FP32)
    int hf_ld;
};

// Modes: 0 FORCES (2D), 1 HERCULES (3D), 2 TPW and 3 VLS (row-column volumes:
// columns transmit, rows receive).  Modes 0, 2, 3 separate into a transmit
// and a receive excess path; HERCULES has one radial receive path.
constexpr int MODE_FORCES = 0, MODE_HERCULES = 1, MODE_TPW = 2, MODE_VLS = 3;

// Staging of a batch's windows by the LDS kernels: the nb * lmax coefficient
// quads are dealt to the workgroup's threads in rounds.  With real data a
// thread stages two adjacent quads of one window per round (five taps give
// both, and lmax is even); with IQ data one.  stage_rounds is the number of
// rounds the kernels unroll, and the host keeps every batch within it.
__host__ __device__ constexpr bool stage_pairs(bool iq) { return !iq; }
__host__ __device__ constexpr int stage_rounds(int mode, bool iq)
{
    return iq && (mode == MODE_TPW || mode == MODE_VLS) ? 3 : 2;
}

// Hann weight table: W(u) of Eq. 3 sampled at u^2 = k / (4 HANN_N), stored as
// (W_k - k D_k, D_k) with D_k = W_{k+1} - W_k, so that linear interpolation
// in u^2 at table coordinate x = 4 HANN_N u^2 is fma(x, D_k, W_k - k D_k)
// for k = floor(x) (max error 1.2e-7, plus ~6e-8 for the rounded base);
// entry HANN_N is (0, 0), so every u^2 >= 1/4 reads weight 0.
constexpr int HANN_N = 2048;

__device__ inline float *das_out(const DasArgs &a) { return a.out_ref ? *a.out_ref : a.out; }

// Channel rows [j0, j1) of group g of G.
__host__ __device__ inline void group_rows(int n_ch, int g, int G, int *j0, int *j1)
{
    *j0 = (int)(((long)n_ch * g) / G);
    *j1 = (int)(((long)n_ch * (g + 1)) / G);
}

// Channel rows per staged batch of the separable modes (FORCES, TPW, VLS):
// a batch holds JC rows x nb / JC transmits (nb a multiple of JC).
constexpr int JC = 4;

// Workgroup configuration of the LDS-staged DAS kernel.
struct LdsCfg {
    int bwx, bwy, bwz;   // wavefront tiles per workgroup along x, y, z
    int nb;              // traces per batch (separable modes: JC rows x nb/JC transmits)
    int lmax;            // coefficient quads per staged window
    int sorted_tx;       // tx_x ascending (enables the per-row transmit range)
    int blocks_x, blocks_y, blocks_z;
    int uniform_tx;      // tx_x[i] = tx_x0 + i * tx_dx exactly (range by arithmetic)
    float tx_x0, tx_inv_dx;
    float inv_lmax;      // 1 / lmax (staging: quad number -> (trace, quad))
    int zp;              // output points per lane along z (1, or 2 for HERCULES real data)
    int z_off;           // box grid shift along z: box bz holds iz from bz * tz - z_off
                         // (VLS: no box straddles the virtual line's depth)
    int guard;           // zeroed sample intervals after the second window buffer
                         // (HERCULES: reads of lanes outside their aperture)
};

// Workgroups of a single-frame LDS launch (box order xcd_slab_box): whole
// groups of 8 depth slabs.
__host__ __device__ inline int xcd_slab_grid(const LdsCfg &c)
{
    return c.blocks_x * c.blocks_y * 8 * ((c.blocks_z + 7) / 8);
}

// One frame of a batch for the persistent DAS kernel (device table entry).
struct FrameDas {
    DasArgs a;      // out is taken from the per-launch pointer table
    LdsCfg c;
};

// Work queues of the persistent DAS kernel: one per XCD, queue q holding
// items[off[q] .. off[q + 1]).
constexpr int N_XCD_QUEUES = 8;
struct QueueSet {
    int off[N_XCD_QUEUES + 1];
};

struct PersistentLaunch {
    int mode, et, ip, zp;
    int grid, threads;
    size_t shm;
    const FrameDas *frames;
    const int4 *items;      // (frame, workgroup box, channel group, -), grouped by queue
    QueueSet queues;
    int *counters;          // one per queue
    void *const *out_ptrs;  // [n_frames] device pointers
};

// Hann window of Eq. 3 as a function of w = u^2 on [0, 1/4): a degree-6
// polynomial fitted at Chebyshev nodes (max error 2e-7 in FP32 Horner form,
// exact 1 at w = 0 and exact 0 at w = 1/4 up to FP32 rounding).  Using u^2
// avoids a square root and a cosine per sample; the caller zeroes w >= 1/4.
__host__ __device__ inline float hann_u2(float w)
{
    float p = 3.264329195e+00f;
    p = p * w + -1.298379993e+01f;
    p = p * w + 3.008381462e+01f;
    p = p * w + -4.272507095e+01f;
    p = p * w + 3.246955872e+01f;
    p = p * w + -9.869602203e+00f;
    p = p * w + 1.0f;
    return p;
}

// Global and constant address-space views of device pointers.  A kernel
// that reads its pointers from a table in memory (the persistent kernels)
// holds generic pointers, and the compiler turns their loads into FLAT
// instructions, which also count against the LDS wait counter: every LDS wait
// of the terms would then wait for the staging loads in flight, and a
// uniform table read would take a vector round trip.  Data loads go through
// the global view (vector loads counted by vmcnt only); uniform reads of the
// read-only geometry tables through the constant view (scalar loads).
template <typename T> using gptr = const __attribute__((address_space(1))) T *;
template <typename T> using gptr_mut = __attribute__((address_space(1))) T *;
template <typename T> using cptr = const __attribute__((address_space(4))) T *;
template <typename T> __device__ inline gptr<T> as_global(const T *p) { return (gptr<T>)p; }
template <typename T> __device__ inline gptr_mut<T> as_global_mut(T *p) { return (gptr_mut<T>)p; }
template <typename T> __device__ inline cptr<T> as_const(const T *p) { return (cptr<T>)p; }
// LDS views: a 32-bit LDS byte address of a shared-memory pointer, and a
// read through such an address (one DS instruction on the address VGPR)
template <typename T> using lptr = const __attribute__((address_space(3))) T *;
__device__ inline unsigned lds_addr(const void *p)
{
    return (unsigned)(size_t)(lptr<char>)static_cast<const char *>(p);
}
__device__ inline float4 lds_read_f4(unsigned addr)
{
    typedef float v4f __attribute__((ext_vector_type(4)));
    const v4f v = *(lptr<v4f>)(size_t)addr;
    return make_float4(v.x, v.y, v.z, v.w);
}

// Vector accesses through those views go element by element (the views do
// not carry the vector types' constructors); the compiler merges them into
// one wide load or store.
__device__ inline float2 load_f2(const float2 *p, long idx)
{
    const gptr<float> q = as_global(reinterpret_cast<const float *>(p + idx));
    return make_float2(q[0], q[1]);
}
__device__ inline void store_f2(float2 *p, long idx, float2 v)
{
    const gptr_mut<float> q = as_global_mut(reinterpret_cast<float *>(p + idx));
    q[0] = v.x;
    q[1] = v.y;
}

template <int ET>
__device__ inline float load_e(const void *base, long idx)
{
    if constexpr (ET == ET_F32) {
        return as_global(static_cast<const float *>(base))[idx];
    } else if constexpr (ET == ET_BF16) {
        uint32_t b = as_global(static_cast<const uint16_t *>(base))[idx];
        return __uint_as_float(b << 16);
    } else {
        return (float)as_global(static_cast<const int *>(base))[idx];
    }
}

// IQ: the carrier phase restored for sample position nB + s is
// fd (tof - t0) = rot (nB + s) revolutions.  rot * nB is large, so its
// fractional part is taken once per lane in FP64; per term only rot * s (s is
// the small FP32 offset) is added.
__device__ inline float phase_origin(const DasArgs &a, int nB)
{
    const double f = a.rot_d * (double)nB;
    return (float)(f - floor(f));
}

// IQ term: acc += w * v * exp(j 2 pi ph) with ph in revolutions.  The hardware
// sine and cosine take revolutions; the argument is reduced to [0, 1) first.
__device__ inline void rotate_acc(float2 v, float w, float ph, float2 &acc)
{
    const float f = __builtin_amdgcn_fractf(ph);
    const float wc = w * __builtin_amdgcn_cosf(f), ws = w * __builtin_amdgcn_sinf(f);
    acc.x = fmaf(v.x, wc, acc.x);
    acc.x = fmaf(-v.y, ws, acc.x);
    acc.y = fmaf(v.x, ws, acc.y);
    acc.y = fmaf(v.y, wc, acc.y);
}

// Per-lane state of one output point of a DAS wavefront tile.
struct Lane {
    bool valid;     // inside the grid
    bool active;    // valid and in front of the array (z > 0)
    long out_idx;
    float x, y, z, z2;
    int nB;         // integer part of B
    float fB;       // fractional part of B
    float thr;      // rho^2 threshold of the receive aperture (inf: no apodization)
    float wsc;      // u^2 = rho^2 * wsc
    float ph0;      // IQ: carrier phase (revolutions, in [0, 1)) of sample position nB
    float ptx;      // transmit path down to the point: z, or |p - v| - f (diverging)
};

// Transmit path of a point (array-frame offsets from the centre) in FP64: the
// plane wave's z, or for a diverging wave from v = (0, 0, -f) the distance to
// v minus f (zero at the array centre).
__device__ inline double tx_path(const DasArgs &a, double px, double py, double pz)
{
    if (a.div_f > 0.0) {
        const double dz = pz + a.div_f;
        return sqrt(px * px + py * py + dz * dz) - a.div_f;
    }
    return pz;
}

__device__ inline Lane lane_setup(const DasArgs &a, int wave_id, int lane)
{
    Lane L;
    const int tz = wave_id % a.tiles_z;
    const int rest = wave_id / a.tiles_z;
    const int tx = rest % a.tiles_x;
    const int ty = rest / a.tiles_x;
    const int lz = lane & ((1 << a.lz) - 1);
    const int lx = (lane >> a.lz) & ((1 << a.lx) - 1);
    const int ly = lane >> (a.lz + a.lx);
    const int ix = (tx << a.lx) + lx, iy = (ty << a.ly) + ly, iz = (tz << a.lz) + lz;
    L.valid = ix < a.g.nx && iy < a.g.ny && iz < a.g.nz;
    L.out_idx = ((long)iy * a.g.nx + ix) * a.g.nz + iz;
    const double px = a.g.org[0] + ix * a.g.ax[0] + iy * a.g.ay[0] + iz * a.g.az[0];
    const double py = a.g.org[1] + ix * a.g.ax[1] + iy * a.g.ay[1] + iz * a.g.az[1];
    const double pz = a.g.org[2] + ix * a.g.ax[2] + iy * a.g.ay[2] + iz * a.g.az[2];
    L.active = L.valid && pz > 0.0;
    const double ptx = tx_path(a, px, py, pz);
    L.ptx = (float)ptx;
    const double B = (ptx + pz) * a.k - a.t0fs;
    const double fl = floor(B);
    L.nB = (int)fl;
    L.fB = (float)(B - fl);
    L.x = (float)px;
    L.y = (float)py;
    L.z = (float)pz;
    L.z2 = L.z * L.z;
    if (a.f2 > 0.f) {
        L.thr = L.z2 * 0.25f / a.f2;
        L.wsc = a.f2 / L.z2;
    } else {
        L.thr = __builtin_inff();
        L.wsc = 0.f;
    }
    L.ph0 = phase_origin(a, L.nB);
    return L;
}

// Excess path d - z of a lateral offset with squared length rho2.
__device__ inline float excess(float rho2, float z, float z2)
{
    const float d = __builtin_amdgcn_sqrtf(rho2 + z2);
    return rho2 * __builtin_amdgcn_rcpf(d + z);
}

// Receive coordinate of a lane for modes 0, 2, 3 (the receivers of FORCES are
// columns at x, those of TPW and VLS rows at y).
template <int MODE>
__device__ inline float rx_coord(float x, float y)
{
    return MODE == MODE_FORCES ? x : y;
}

// Transmit excess path beyond z of transmit i at lane position (x, z), for
// modes 0, 2, 3 (the transmit path is z + this):
//   FORCES: cylindrical wave of column x_i:   |(x - x_i, z)| - z
//   TPW:    tilted plane wave, zero at the centre: x sin(th) + z (cos(th) - 1)
//   VLS:    virtual line source (x_i, z_f):   z_f + sgn(z - z_f) |(x - x_i, z - z_f)| - z
//           = sgn(dz) rho^2 / (|(rho, dz)| + |dz|),  rho = x - x_i, dz = z - z_f
//           (exact rewriting without cancellation; sgn(0) = +1)
// The same from the transmit's table entries: tsc = (sin, cos - 1) for TPW,
// xi = column position for FORCES and VLS.
template <int MODE>
__device__ inline float tx_excess_p(float x, float z, float z2, float2 tsc, float xi, float zf)
{
    if constexpr (MODE == MODE_TPW) {
        return fmaf(x, tsc.x, z * tsc.y);
    } else if constexpr (MODE == MODE_VLS) {
        const float rho = x - xi, dz = z - zf;
        const float r2 = rho * rho;
        const float den = __builtin_amdgcn_sqrtf(fmaf(dz, dz, r2)) + fabsf(dz);
        const float e = den > 0.f ? r2 * __builtin_amdgcn_rcpf(den) : 0.f;   // 0 on the line
        return dz >= 0.f ? e : -e;
    } else {
        const float dxt = x - xi;
        return excess(dxt * dxt, z, z2);
    }
}

template <int MODE>
__device__ inline float tx_excess(const DasArgs &a, float x, float z, float z2, int i)
{
    return tx_excess_p<MODE>(x, z, z2, MODE == MODE_TPW ? a.tx_sc[i] : make_float2(0.f, 0.f),
                             MODE == MODE_TPW ? 0.f : a.tx_x[i], a.zf);
}

template <int ET>
__device__ inline const void *trace_ptr(const void *e, long trace, int S)
{
    if constexpr (ET == ET_BF16)
        return static_cast<const uint16_t *>(e) + trace * S;
    else if constexpr (ET == ET_CF32)
        return static_cast<const float2 *>(e) + trace * S;
    else
        return static_cast<const float *>(e) + trace * S;   // f32 and i32 are 4 bytes
}

__device__ inline float2 load_c(const void *base, long idx)
{
    return load_f2(static_cast<const float2 *>(base), idx);
}

}  // namespace bf
