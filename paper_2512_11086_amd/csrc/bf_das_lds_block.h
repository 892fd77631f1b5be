// bf_das_lds_block.h -- the LDS-staged delay-and-sum workgroup body shared
// by the forward kernels (bf_das_lds.hip) and the adjoint kernels
// (bf_das_adj.hip).  Internal to libbf.
//
// A workgroup owns a box of output points (a grid of 64-lane wavefront
// tiles).  It walks the (transmit, channel) traces in batches; for every
// trace of a batch it stages, once, the window of samples that any point of
// the box can read -- bounded from the box geometry, since the delay grows
// with depth and with lateral distance -- as cubic-Hermite coefficient quads
// (c0, c1, c2, c3) per sample interval, with zeros outside the record.  Each
// term of Eq. 1 then costs one aligned 16-byte LDS read and three FMAs for
// the read (Sec. IV-B) instead of four bounds-checked global loads.  The
// global loads of the next batch are issued before the current batch is
// beamformed (double-buffered LDS, one barrier per batch), and they read
// contiguous runs along fast time.
//
// HERCULES volumes with real data can give each lane two adjacent depth
// points (ZP = 2): both share the lateral offset to the receiver, rho^2 and
// the per-trace scalars of every term, and each wavefront's per-batch work
// (aperture mask, trace metadata) serves twice the points.
//
// Separable modes (FORCES planes, TPW and VLS row-column volumes): the delay
// is a transmit path per (point, transmit) plus a receive path per (point,
// channel row), and the apodization depends on the row only.  A batch holds
// JC rows x nb/JC transmits; each lane computes the receive path and weight
// of a row once, the transmit path of a transmit once per batch (shared by
// the JC rows), and every term adds the two.  The forward kernels on real
// data fold the trace's window start into the two paths (FOLD in das_block),
// so the sum is the position inside the staged window.
//
// Apodization skip (Sec. VII-F): a channel row is staged only if the receive
// aperture of the deepest point of the box reaches it; within a row only the
// transmits whose lateral offset can fall inside that aperture are staged
// (HERCULES); each wavefront additionally skips traces outside the union of
// its own lanes' apertures with a scalar test (HERCULES), or rows no lane of
// it can receive (separable modes).
//
// Delay precision: as in the gather kernel, s = B(p) + k (E_tx + E_rx) with
// B in FP64 split into integer + FP32 fraction and E = rho^2 / (d + z) in FP32.
//
// IQ data (ET_CF32): a sample interval stages as two adjacent quads, the
// coefficients of the real and of the imaginary part (32 bytes per interval),
// and each term is rotated by its carrier phase before the complex
// accumulation.
//
// Decode fused into DAS (ET_RF16, FORCES planes): the kernel reads the int16
// RF channel data and forms each staged tap of decoded trace (i, j) as
// sum_k H[k][i] rf[k][j][n] (Sec. VII-E) while staging; the sums of at most
// 256 products of +-1 and int16 values are exact in FP32, so the windows, and
// the image, are those of decoding first and beamforming the decoded data.
#pragma once

#include "bf_common.h"

namespace bf {

hipError_t launch_sum_groups(const DasArgs &a, hipStream_t s);

constexpr int HANN_TAB_PAD = HANN_N + 2;   // table entries reserved in LDS (float2, keeps 16-byte alignment)

// Trace slot `lane` of a batch, held by that lane of every wavefront: the
// first sample interval w0 of its window, the x of its transmit column, and
// for staging the window start sw and the element offset off = trace * S + w0
// of that sample in the decoded data.  sw is NO_DATA for a slot with nothing
// to stage (an empty slot, a padding slot, or a window wholly outside the
// record, which stages zeros), so that off stays within the data (no 32-bit
// overflow) whenever it is used.  Staging lanes (and the RF gradient's flush)
// fetch sw and off of their slot with a lane permute; the terms take the
// column from the read-only table and the negated window start from a
// per-batch LDS array (store_w0).  ti: the slot's transmit (the fused decode
// reads H[.][ti]).
constexpr int NO_DATA = -(1 << 29);
struct TraceDesc {
    int w0;
    float xi;
    int sw;
    int off;
    int ti;
};

// Uniform description of one batch (lane_row: per lane, see Iter).
struct BatchDesc {
    int valid;
    int i0, cnt;          // transmits i0 .. i0+cnt-1
    int j;                // HERCULES: channel row
    int rows[JC];         // separable modes: channel rows (row_slot encoding)
    int lane_row;         // separable modes: rows[lane % JC], the row of trace slot `lane`
};

// Row slots of the separable modes.  A chunk of JC slots holds the next
// active channel rows; when fewer remain, the last one is repeated in the
// free slots as a padding slot, encoded -(row + 2): it has that row's
// geometry (so the terms read inside a staged window) but no staged data
// (its window holds zeros) and weight 0.  Every slot is then a real row and
// the terms of a transmit need no per-row branch.
__device__ inline int slot_row(int v) { return v >= 0 ? v : -v - 2; }
__device__ inline bool slot_pad(int v) { return v < 0; }

struct BoxGeom {
    float xmin, xmax, ymin, ymax, zmin, zmax;
    float kf, t0f;    // fs / c and t0 * fs in FP32 (window bounds only)
    float txlo;       // lower bound of the transmit path over the box (HERCULES)
};

__device__ inline float wave_min(float v)
{
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline float wave_max(float v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ inline int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline float uniform_f(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Lane state.  A point outside the grid or at z <= 0 keeps the lane's real
// lateral position (a lane's points share it) and benign depth values: it
// is never inside the aperture mask, its arithmetic stays finite, and its
// sum is discarded (outside the grid) or replaced by 0 (z <= 0, where the
// apodization vanishes) when the outputs are stored.
struct LaneL {
    bool valid;
    float x, y, z, z2, thr, wsc, fB;
    float zk, zk2;  // z / k and its square (k = fs / c): the HERCULES delay
    float wtab;     // u^2 * 4 HANN_N = rho^2 * wtab (table coordinate)
    int nB;
    float ph0;      // IQ: carrier phase of sample position nB (revolutions)
};

// Grid indices of point p (0 .. zp-1) of a lane: the lane's z tile index
// times zp plus p, so a lane's points are adjacent along z.
__device__ inline void lane_point(const DasArgs &a, const LdsCfg &c, int bx, int by, int bz,
                                  int wave, int lane, int p, int *ix, int *iy, int *iz)
{
    const int wz = wave % c.bwz, wx = (wave / c.bwz) % c.bwx, wy = wave / (c.bwz * c.bwx);
    const int lz = lane & ((1 << a.lz) - 1);
    const int lx = (lane >> a.lz) & ((1 << a.lx) - 1);
    const int ly = lane >> (a.lz + a.lx);
    *ix = ((bx * c.bwx + wx) << a.lx) + lx;
    *iy = ((by * c.bwy + wy) << a.ly) + ly;
    *iz = (((bz * c.bwz + wz) << a.lz) + lz) * c.zp + p - c.z_off;
}

// nref (folded HERCULES reads): fB then holds B - nref in one FP32 rounding.
template <int MODE>
__device__ inline LaneL lane_setup_l(const DasArgs &a, const LdsCfg &c, int bx, int by, int bz,
                                     int wave, int lane, int p, const int *nref = nullptr)
{
    LaneL L;
    int ix, iy, iz;
    lane_point(a, c, bx, by, bz, wave, lane, p, &ix, &iy, &iz);
    L.valid = ix < a.g.nx && iy < a.g.ny && iz >= 0 && iz < a.g.nz;
    // The terms read their windows without clamping the index, so every lane
    // takes the geometry of the nearest grid point of its box: its delay then
    // lies within the box's bounds (see hercules_term and the separable terms
    // of das_block)
    ix = min(ix, a.g.nx - 1);
    iy = min(iy, a.g.ny - 1);
    iz = min(max(iz, 0), a.g.nz - 1);
    const double px = a.g.org[0] + ix * a.g.ax[0] + iy * a.g.ay[0] + iz * a.g.az[0];
    const double py = a.g.org[1] + ix * a.g.ax[1] + iy * a.g.ay[1] + iz * a.g.az[1];
    const double pz = a.g.org[2] + ix * a.g.ax[2] + iy * a.g.ay[2] + iz * a.g.az[2];
    L.x = (float)px;
    L.y = (float)py;
    // a point on or behind the array plane (its output is 0) is evaluated
    // just in front of it, inside the box; it and any lane outside the grid
    // stay out of every aperture test (thr < 0: weight 0, no wavefront mask)
    const double pze = fmax(pz, 1e-7);
    const double B = (tx_path(a, px, py, pze) + pze) * a.k - a.t0fs;
    const double fl = floor(B);
    L.nB = (int)fl;
    L.fB = (float)(B - (nref ? (double)*nref : fl));
    L.z = (float)pze;
    L.z2 = L.z * L.z;
    L.zk = (float)(pze / a.k);
    L.zk2 = L.zk * L.zk;
    L.thr = (L.valid && pz > 0.0) ? (a.f2 > 0.f ? L.z2 * 0.25f / a.f2 : __builtin_inff()) : -1.f;
    L.wsc = a.f2 > 0.f ? a.f2 / L.z2 : 0.f;
    L.wtab = L.wsc * (4.f * HANN_N);
    L.ph0 = phase_origin(a, L.nB);
    return L;
}

// Array-frame bounding box of the workgroup's points (clamped to the grid).
__device__ inline BoxGeom block_box(const DasArgs &a, const LdsCfg &c, int bx, int by, int bz)
{
    const int tx = c.bwx << a.lx, ty = c.bwy << a.ly, tz = (c.bwz << a.lz) * c.zp;
    const int i0[3] = {bx * tx, by * ty, max(bz * tz - c.z_off, 0)};
    const int i1[3] = {min(bx * tx + tx - 1, a.g.nx - 1), min(by * ty + ty - 1, a.g.ny - 1),
                       min(bz * tz + tz - 1 - c.z_off, a.g.nz - 1)};
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int q = 0; q < 8; ++q) {
        const int ix = (q & 1) ? i1[0] : i0[0];
        const int iy = (q & 2) ? i1[1] : i0[1];
        const int iz = (q & 4) ? i1[2] : i0[2];
        for (int r = 0; r < 3; ++r) {
            const double v = a.g.org[r] + ix * a.g.ax[r] + iy * a.g.ay[r] + iz * a.g.az[r];
            lo[r] = fmin(lo[r], v);
            hi[r] = fmax(hi[r], v);
        }
    }
    BoxGeom b;
    b.xmin = (float)lo[0]; b.xmax = (float)hi[0];
    b.ymin = (float)lo[1]; b.ymax = (float)hi[1];
    b.zmin = (float)lo[2]; b.zmax = (float)hi[2];
    b.kf = (float)a.k;
    b.t0f = (float)a.t0fs;
    // transmit path: z (plane wave), or the distance from the virtual source
    // (0, 0, -f) to the box minus f (diverging wave); both grow with depth
    const float zlo = fmaxf(b.zmin, 0.f);
    b.txlo = zlo;
    if (a.div_f > 0.0) {
        const float f = (float)a.div_f;
        const float dx = fmaxf(0.f, fmaxf(b.xmin, -b.xmax));
        const float dy = fmaxf(0.f, fmaxf(b.ymin, -b.ymax));
        b.txlo = __builtin_amdgcn_sqrtf(fmaf(dx, dx, fmaf(dy, dy, (zlo + f) * (zlo + f)))) - f;
    }
    // workgroup-uniform: keep the box in scalar registers
    b.xmin = uniform_f(b.xmin); b.xmax = uniform_f(b.xmax);
    b.ymin = uniform_f(b.ymin); b.ymax = uniform_f(b.ymax);
    b.zmin = uniform_f(b.zmin); b.zmax = uniform_f(b.zmax);
    b.kf = uniform_f(b.kf); b.t0f = uniform_f(b.t0f); b.txlo = uniform_f(b.txlo);
    return b;
}

__device__ inline float dist_to_range(float v, float lo, float hi)
{
    return fmaxf(0.f, fmaxf(lo - v, v - hi));
}
__device__ inline float far_to_range(float v, float lo, float hi)
{
    return fmaxf(fabsf(v - lo), fabsf(v - hi));
}

// Lower bounds over the box of the transmit path of transmit i (column at
// xi) and of the receive path of the row or column at cj, for the separable
// modes: the receive path of a row (TPW, VLS) or column (FORCES) is at least
// its distance to the nearest box point at the shallowest depth.  A box
// tabulates both once (tx_lo per transmit, rx_lo per channel) and a trace's
// window starts at their sum (window_start).
template <int MODE>
__device__ inline float tx_lo(const DasArgs &a, const BoxGeom &b, int i, float xi)
{
    const float zlo = fmaxf(b.zmin, 0.f);
    if constexpr (MODE == MODE_FORCES) {
        const float rt = dist_to_range(xi, b.xmin, b.xmax);
        return __builtin_amdgcn_sqrtf(fmaf(rt, rt, zlo * zlo));
    } else if constexpr (MODE == MODE_TPW) {
        // x sin(th) + z cos(th): smallest at the box edge along sin(th), cos(th) > 0
        const float2 sc = load_f2(a.tx_sc, i);
        return (sc.x >= 0.f ? b.xmin : b.xmax) * sc.x + zlo * (1.f + sc.y);
    } else {
        // z_f + sgn(z - z_f) |(x - x_i, z - z_f)|: with the whole box below the
        // line the nearest point bounds it; else z_f minus the farthest reach
        const float zf = a.zf;
        if (zf <= zlo) {
            const float rx = dist_to_range(xi, b.xmin, b.xmax);
            return zf + __builtin_amdgcn_sqrtf(fmaf(rx, rx, (zlo - zf) * (zlo - zf)));
        }
        const float rf = far_to_range(xi, b.xmin, b.xmax);
        return zf - __builtin_amdgcn_sqrtf(fmaf(rf, rf, (zf - zlo) * (zf - zlo)));
    }
}

template <int MODE>
__device__ inline float rx_lo(const BoxGeom &b, float cj)
{
    const float zlo = fmaxf(b.zmin, 0.f);
    const float r = MODE == MODE_FORCES ? dist_to_range(cj, b.xmin, b.xmax)
                                        : dist_to_range(cj, b.ymin, b.ymax);
    return __builtin_amdgcn_sqrtf(fmaf(r, r, zlo * zlo));
}

// First sample interval of the staged window of a trace for the box, from a
// lower bound of its path over the box (the bound has a 2-sample margin, so
// the hardware square root suffices): HERCULES from the transmit column at xi
// and the row at cj; the separable modes from the tabulated bounds (path =
// tx_lo + rx_lo).
__device__ inline int window_from_path(const BoxGeom &b, float path)
{
    return (int)floorf(fmaf(path, b.kf, -b.t0f)) - 2;
}

__device__ inline int window_start_hercules(const BoxGeom &b, float xi, float cj)
{
    const float zlo = fmaxf(b.zmin, 0.f);
    const float rx = dist_to_range(xi, b.xmin, b.xmax);
    const float ry = dist_to_range(cj, b.ymin, b.ymax);
    return window_from_path(b, b.txlo + __builtin_amdgcn_sqrtf(fmaf(rx, rx, fmaf(ry, ry, zlo * zlo))));
}

// Is channel row j reachable by the receive aperture of any point of the box?
// For HERCULES also returns the lateral reach R of the aperture along x.
template <int MODE>
__device__ inline bool row_active(const DasArgs &a, const BoxGeom &b, float cj, float *R)
{
    if (b.zmax <= 0.f) return false;
    if (a.f2 <= 0.f) {
        *R = __builtin_inff();
        return true;
    }
    const float thr = b.zmax * b.zmax * 0.25f / a.f2;
    const float d = MODE == 0 ? dist_to_range(cj, b.xmin, b.xmax) : dist_to_range(cj, b.ymin, b.ymax);
    const float r2 = thr - d * d;
    *R = sqrtf(fmaxf(r2, 0.f));
    return r2 > 0.f;
}

// Transmit range [lo, hi) whose column x lies in [xl, xh] (ascending tx_x).
__device__ inline void tx_range(const float *tx, int n, float xl, float xh, int *lo, int *hi)
{
    int a0 = 0, b0 = n;                   // first index with tx >= xl
    while (a0 < b0) {
        const int m = (a0 + b0) >> 1;
        if (tx[m] < xl) a0 = m + 1; else b0 = m;
    }
    int a1 = a0, b1 = n;                  // first index with tx > xh
    while (a1 < b1) {
        const int m = (a1 + b1) >> 1;
        if (tx[m] <= xh) a1 = m + 1; else b1 = m;
    }
    *lo = a0;
    *hi = a1;
}

// Batch iterator (uniform across the workgroup, except lane_row).
struct Iter {
    int jend;    // end of this workgroup's channel rows
    int j;       // current channel row (HERCULES) / next row to scan (separable)
    int i;       // next transmit
    int ihi;     // end of the current row's transmit range (HERCULES)
    int rows[JC];
    int lane_row;  // rows[lane % JC] (the slots of a separable batch are
                   // transmit-major: slot e = transmit e / JC, row e % JC)
};

template <int MODE>
__device__ inline BatchDesc next_batch(const DasArgs &a, const LdsCfg &c, const BoxGeom &b,
                                       const float *s_tx, const float *s_rx, Iter &it)
{
    BatchDesc d;
    d.valid = 0;
    if constexpr (MODE == 1) {
        while (it.i >= it.ihi) {          // advance to the next active row
            ++it.j;
            if (it.j >= it.jend) return d;
            float R;
            if (!row_active<1>(a, b, s_rx[it.j], &R)) continue;
            if (c.uniform_tx && isfinite(R)) {
                // columns on a regular grid: [lo, hi) by arithmetic (one
                // column of margin each side; the wavefront tests are exact)
                const int lo = (int)floorf((b.xmin - R - c.tx_x0) * c.tx_inv_dx) - 1;
                const int hi = (int)floorf((b.xmax + R - c.tx_x0) * c.tx_inv_dx) + 2;
                it.i = max(lo, 0);
                it.ihi = min(hi, a.n_tx);
                if (it.i > it.ihi) it.i = it.ihi;
            } else if (c.sorted_tx && isfinite(R)) {
                tx_range(s_tx, a.n_tx, b.xmin - R, b.xmax + R, &it.i, &it.ihi);
            } else {
                it.i = 0;
                it.ihi = a.n_tx;
            }
        }
        d.valid = 1;
        d.j = it.j;
        d.i0 = it.i;
        d.cnt = min(c.nb, it.ihi - it.i);
        it.i += d.cnt;
        return d;
    } else {
        const int nbi = c.nb / JC;
        if (it.i >= a.n_tx) {             // next chunk of JC active rows
            int n = 0, last = -1;
            while (n < JC && it.j < it.jend) {
                float R;
                if (row_active<MODE>(a, b, s_rx[it.j], &R)) {
                    // (selects instead of a dynamic index keep rows[] in registers)
#pragma unroll
                    for (int q = 0; q < JC; ++q)
                        if (q == n) it.rows[q] = it.j;
                    last = it.j;
                    ++n;
                }
                ++it.j;
            }
            if (n == 0) return d;
#pragma unroll
            for (int q = 0; q < JC; ++q)          // padding slots (slot_row)
                if (q >= n) it.rows[q] = -last - 2;
            // the row of this lane's trace slot, once per chunk
            const int lq = (threadIdx.x & 63) % JC;
            int v = it.rows[0];
#pragma unroll
            for (int q = 1; q < JC; ++q)
                if (lq == q) v = it.rows[q];
            it.lane_row = v;
            it.i = 0;
        }
        d.valid = 1;
        for (int q = 0; q < JC; ++q) d.rows[q] = it.rows[q];
        d.lane_row = it.lane_row;
        d.i0 = it.i;
        d.cnt = min(nbi, a.n_tx - it.i);
        it.i += d.cnt;
        return d;
    }
}

// Transmit i and channel row j of trace slot e = lane of batch d (j = -1: an
// empty slot); *pad: a padding slot of the separable modes (geometry of row
// j, no data).  Separable batches number their slots transmit-major.
template <int MODE>
__device__ inline void slot_trace(const BatchDesc &d, int e, int *i, int *j, bool *pad)
{
    if constexpr (MODE == 1) {
        *i = d.i0 + e;
        *j = e < d.cnt ? d.j : -1;
        *pad = false;
    } else {
        const int ii = e / JC;
        *i = d.i0 + ii;
        *j = ii < d.cnt ? slot_row(d.lane_row) : -1;
        *pad = slot_pad(d.lane_row);
    }
}

// Staging map: the quads of a batch -- with real data the nb * lmax / 2
// pairs of adjacent quads (lmax is even), with IQ data the nb * lmax quads --
// are numbered trace-major and dealt to the workgroup's threads in order
// (round q, wavefront, lane), so no lane idles on a short window and
// consecutive lanes read consecutive samples of one trace.  A pair costs one
// slot's index arithmetic, lane permutes and bounds checks, and five loads
// instead of eight: on the FORCES plane the staging had issued about as many
// VALU instructions as the terms.  Each lane computes the window start of its
// own trace.
template <int QM>
struct Staged {
    float p[QM][8];    // taps n-1 .. n+3 (IQ: n-1 .. n+2, (re, im) of each)
    int dst[QM];       // first quad of the slot in the batch buffer, -1: none
};

// Whether staging round q holds any slot of the batch (uniform: the
// workgroup skips rounds past the last one, e.g. the second of the FORCES
// plane's 16 windows of 128 quads, which its 1024 threads stage in one).
template <bool PR>
__device__ inline bool stage_round_live(const LdsCfg &c, int q, int nwaves)
{
    const int slots = PR ? (c.nb * c.lmax) >> 1 : c.nb * c.lmax;
    return q == 0 || q * nwaves * 64 < slots;
}

// Slot e and first quad m handled by this lane in staging round q; false if
// none.  PR: pairs, m even.  (g + 1/2) / lmax, and (2g + 1) / lmax for
// pairs, are at least 1 / (2 lmax) away from an integer, far more than the
// FP32 rounding of the product for g < 2^16.
template <bool PR>
__device__ inline bool stage_slot(const LdsCfg &c, int q, int wave, int lane, int nwaves, int *e,
                                  int *m)
{
    const int g = (q * nwaves + wave) * 64 + lane;
    const int g2 = PR ? 2 * g : g;
    const int ee = (int)(((float)g2 + (PR ? 1.f : 0.5f)) * c.inv_lmax);
    *e = ee;
    *m = g2 - ee * c.lmax;
    return ee < c.nb;
}

// Descriptor of trace slot `lane` of batch d (see TraceDesc).  s_lo: the
// box's tx_lo table (n_tx entries) and, at lo_rx, its rx_lo table
// (separable modes).
// FOLD (separable forward kernels on real data, cubic or linear reads):
// s_lo holds the box's integer window-start parts A_i (transmits) and B_j
// (rows) instead of the path bounds, and the trace's window starts at
// A_i + B_j.
template <int MODE, bool FOLD = false>
__device__ inline TraceDesc trace_desc(const DasArgs &a, const LdsCfg &c, const BoxGeom &b,
                                       const float *s_tx, const float *s_rx, const float *s_lo,
                                       int lo_rx, const BatchDesc &d, int lane)
{
    TraceDesc t{0, 0.f, NO_DATA, 0};
    if (lane < c.nb) {
        int i, j;
        bool pad;
        slot_trace<MODE>(d, lane, &i, &j, &pad);
        if (j >= 0) {
            t.xi = s_tx[i];
            t.ti = i;
            if constexpr (MODE == MODE_HERCULES)
                t.w0 = window_start_hercules(b, t.xi, s_rx[j]);
            else if constexpr (FOLD)
                t.w0 = (int)(s_lo[i] + s_lo[lo_rx + j]);   // integers: exact
            else
                t.w0 = window_from_path(b, s_lo[i] + s_lo[lo_rx + j]);
            // taps w0 - 1 .. w0 + lmax + 1 of the window; none inside the record:
            // nothing to stage (and a padding slot stages zeros)
            if (!pad && t.w0 + c.lmax + 1 >= 0 && t.w0 - 1 < a.S) {
                t.sw = t.w0;
                // 24-bit products: traces < 2^18, samples <= 2^16 (plan
                // limits), element offsets < 2^31
                const unsigned tr = __umul24((unsigned)i, (unsigned)a.n_ch) + (unsigned)j;
                t.off = (int)__umul24(tr, (unsigned)a.S) + t.w0;
            }
        }
    }
    return t;
}

// Issue the global loads of a batch's windows (taps n-1 .. n+2 of every quad;
// real data: n-1 .. n+3 of every pair of quads n, n+1).
template <int ET, int QM>
__device__ inline void stage_load(const DasArgs &a, const LdsCfg &c, const TraceDesc &td,
                                  Staged<QM> &st, int wave, int lane, int nwaves)
{
    constexpr bool PR = stage_pairs(ET == ET_CF32);
#pragma unroll
    for (int q = 0; q < QM; ++q) {
        if (!stage_round_live<PR>(c, q, nwaves)) break;
        int e, m;
        const bool on = stage_slot<PR>(c, q, wave, lane, nwaves, &e, &m);
        st.dst[q] = on ? e * c.lmax + m : -1;
        // window start and data offset of slot e, from lane e
        const int src = (e & 63) << 2;
        const int w0 = __builtin_amdgcn_ds_bpermute(src, td.sw);
        const int off = __builtin_amdgcn_ds_bpermute(src, td.off);
        // (the fused decode's transmit of slot e; every lane is active here, as
        // a permute must read its source lane while that lane is active)
        const int ti = ET == ET_RF16 ? __builtin_amdgcn_ds_bpermute(src, td.ti) : 0;
        float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f;
        float p4 = 0.f, p5 = 0.f, p6 = 0.f, p7 = 0.f;
        if (on && w0 != NO_DATA) {
            const int n = w0 + m;
            // sample n of the trace: element off + m (32-bit, see TraceDesc)
            const void *tn = trace_ptr<ET>(a.e, off + m, 1);
            const unsigned S = (unsigned)a.S;
            // (the last tap of the window, of its last quad or pair, is w0 + lmax + 1)
            const bool inside = w0 >= 1 && w0 + c.lmax + 1 < a.S;
            if constexpr (ET == ET_RF16) {
                // decode fused into staging: tap n + u (u = -1 .. 2) of decoded
                // trace (ti, j) is sum_k H[k][ti] rf[k][j][n + u]; sample n of
                // transmit k's trace of row j is element base + k n_ch S
                // (base: off + m less ti's traces; all offsets < 2^31)
                const int kstride = a.n_ch * a.S;
                const int base = off + m - ti * kstride;
                const gptr<int16_t> r = as_global(static_cast<const int16_t *>(a.e));
                const gptr<float> hcol = as_global(a.hf) + ti;
                const unsigned S = (unsigned)a.S;
                const bool t0 = inside || (unsigned)(n - 1) < S, t1 = inside || (unsigned)n < S;
                const bool t2 = inside || (unsigned)(n + 1) < S, t3 = inside || (unsigned)(n + 2) < S;
                const bool t4 = inside || (unsigned)(n + 3) < S;
                // (a transmit index outside the plan reads nothing: a wrong
                // image, never an access outside rf)
                const int nk = (unsigned)ti < (unsigned)a.n_tx ? a.n_tx : 0;
                for (int k = 0; k < nk; ++k) {
                    const int idx = base + k * kstride;
                    const float hk = hcol[k * a.hf_ld];
                    p0 = fmaf(hk, t0 ? (float)r[idx - 1] : 0.f, p0);
                    p1 = fmaf(hk, t1 ? (float)r[idx] : 0.f, p1);
                    p2 = fmaf(hk, t2 ? (float)r[idx + 1] : 0.f, p2);
                    p3 = fmaf(hk, t3 ? (float)r[idx + 2] : 0.f, p3);
                    p4 = fmaf(hk, t4 ? (float)r[idx + 3] : 0.f, p4);
                }
            } else if constexpr (ET == ET_CF32) {
                // (re, im) of taps n-1 .. n+2: 32 contiguous bytes
                const float2 z = make_float2(0.f, 0.f);
                float2 t0, t1, t2, t3;
                if (inside) {
                    const gptr<float> u = as_global(reinterpret_cast<const float *>(tn) - 2);
                    t0 = make_float2(u[0], u[1]); t1 = make_float2(u[2], u[3]);
                    t2 = make_float2(u[4], u[5]); t3 = make_float2(u[6], u[7]);
                } else {
                    t0 = ((unsigned)(n - 1) < S) ? load_c(tn, -1) : z;
                    t1 = ((unsigned)n < S) ? load_c(tn, 0) : z;
                    t2 = ((unsigned)(n + 1) < S) ? load_c(tn, 1) : z;
                    t3 = ((unsigned)(n + 2) < S) ? load_c(tn, 2) : z;
                }
                p0 = t0.x; p1 = t1.x; p2 = t2.x; p3 = t3.x;
                p4 = t0.y; p5 = t1.y; p6 = t2.y; p7 = t3.y;
            } else if (inside) {
                // whole window inside the record (the usual case): the five
                // taps from 20 contiguous bytes (4-byte aligned)
                if constexpr (ET == ET_F32) {
                    const gptr<float> v = as_global(static_cast<const float *>(tn) - 1);
                    p0 = v[0]; p1 = v[1]; p2 = v[2]; p3 = v[3]; p4 = v[4];
                } else {
                    p0 = load_e<ET>(tn, -1);
                    p1 = load_e<ET>(tn, 0);
                    p2 = load_e<ET>(tn, 1);
                    p3 = load_e<ET>(tn, 2);
                    p4 = load_e<ET>(tn, 3);
                }
            } else {
                p0 = ((unsigned)(n - 1) < S) ? load_e<ET>(tn, -1) : 0.f;
                p1 = ((unsigned)n < S) ? load_e<ET>(tn, 0) : 0.f;
                p2 = ((unsigned)(n + 1) < S) ? load_e<ET>(tn, 1) : 0.f;
                p3 = ((unsigned)(n + 2) < S) ? load_e<ET>(tn, 2) : 0.f;
                p4 = ((unsigned)(n + 3) < S) ? load_e<ET>(tn, 3) : 0.f;
            }
        }
        st.p[q][0] = p0;
        st.p[q][1] = p1;
        st.p[q][2] = p2;
        st.p[q][3] = p3;
        st.p[q][4] = p4;
        st.p[q][5] = p5;
        st.p[q][6] = p6;
        st.p[q][7] = p7;
    }
}

// Coefficient quad of one sample interval from taps p[n-1] .. p[n+2].
// Derivative quad of one sample interval (the adjoint's dL/dc): v'(t) =
// d1 + d2 t + d3 t^2 = (c1, 2 c2, 3 c3) of the cubic; the slope of the linear
// read; 0 for nearest (piecewise constant).
template <int IP>
__device__ inline float4 coef_dquad(float pm, float p0, float p1, float p2)
{
    if constexpr (IP == IN_CUBIC)
        return make_float4(0.5f * (p1 - pm), 2.f * (pm - 2.5f * p0 + 2.0f * p1 - 0.5f * p2),
                           3.f * (0.5f * (p2 - pm) + 1.5f * (p0 - p1)), 0.f);
    else if constexpr (IP == IN_LINEAR)
        return make_float4(p1 - p0, 0.f, 0.f, 0.f);
    else
        return make_float4(0.f, 0.f, 0.f, 0.f);
}

template <int IP>
__device__ inline float eval_dquad(const float4 q, float t)
{
    if constexpr (IP == IN_CUBIC) return fmaf(t, fmaf(t, q.z, q.y), q.x);
    return q.x;
}

template <int IP>
__device__ inline float4 coef_quad(float pm, float p0, float p1, float p2)
{
    if constexpr (IP == IN_CUBIC)
        return make_float4(p0, 0.5f * (p1 - pm), pm - 2.5f * p0 + 2.0f * p1 - 0.5f * p2,
                           0.5f * (p2 - pm) + 1.5f * (p0 - p1));
    else if constexpr (IP == IN_LINEAR)
        return make_float4(p0, p1 - p0, 0.f, 0.f);
    else
        return make_float4(p0, p1, 0.f, 0.f);
}

// Negated window starts of a batch's slots into LDS (wavefront 0, lane =
// slot; the separable modes' slots are [transmit][row], so two 16-byte loads
// give the JC rows of a transmit).
__device__ inline void store_w0(const LdsCfg &c, const TraceDesc &td, int *w, int wave, int lane)
{
    if (wave != 0 || lane >= c.nb) return;
    w[lane] = -td.w0;
}

// The HERCULES forward reads' per-slot value (hercules_term, HF): the LDS
// byte address of slot `lane`'s window in buffer `quads` less (w0 - nR)
// quads (modulo 2^32: the terms add floor(s) * 16 back, and the sum is the
// address of quad floor(s) + nR - w0 of the window).
__device__ inline void store_w0_addr(const LdsCfg &c, const TraceDesc &td, int *w, const float4 *quads,
                                     int nR, int wave, int lane)
{
    if (wave != 0 || lane >= c.nb) return;
    w[lane] = (int)(lds_addr(quads + lane * c.lmax) + ((unsigned)(nR - td.w0) << 4));
}

// Convert the loaded taps to coefficient quads and write them to one LDS
// buffer.  QS = quads per sample interval (2 for IQ data: real part, then
// imaginary part).
template <int IP, int QS, int QM, bool DQ>
__device__ inline void stage_store(const LdsCfg &c, const Staged<QM> &st, float4 *quads, int wave,
                                   int lane, int nwaves)
{
    constexpr bool PR = stage_pairs(QS == 2);
#pragma unroll
    for (int q = 0; q < QM; ++q) {
        if (!stage_round_live<PR>(c, q, nwaves)) break;
        if (st.dst[q] >= 0) {
            const float *t = st.p[q];
            float4 *dst = quads + st.dst[q] * QS;
            dst[0] = DQ ? coef_dquad<IP>(t[0], t[1], t[2], t[3]) : coef_quad<IP>(t[0], t[1], t[2], t[3]);
            if constexpr (PR)         // quad m + 1 < lmax (m even, lmax even)
                dst[1] = DQ ? coef_dquad<IP>(t[1], t[2], t[3], t[4]) : coef_quad<IP>(t[1], t[2], t[3], t[4]);
            if constexpr (QS == 2) dst[1] = coef_quad<IP>(t[4], t[5], t[6], t[7]);
        }
    }
}

// clamp to [0, hi] in one instruction (hi wave-uniform)
__device__ inline int clamp0_i32(int x, int hi)
{
    int r;
    asm("v_med3_i32 %0, %1, 0, %2" : "=v"(r) : "v"(x), "s"(hi));
    return r;
}

template <int IP>
__device__ inline float eval_quad(const float4 q, float t)
{
    if constexpr (IP == IN_NEAREST) return t < 0.5f ? q.x : q.y;
    if constexpr (IP == IN_LINEAR) return fmaf(t, q.y, q.x);
    return fmaf(t, fmaf(t, fmaf(t, q.w, q.z), q.y), q.x);
}

// floor to int in one instruction
__device__ inline int cvt_flr(float x)
{
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// a + b + c in one instruction
__device__ inline int add3_vvv(int a, int b, int c)
{
    int r;
    asm("v_add3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// RF gradient accumulation in LDS: 64-bit fixed point with 32 fraction bits
// (LDS integer atomics run at a far higher rate than FP32 ones).  A term
// value u (scaled so that |u| <= 2^18) enters as floor(u) * 2^32 +
// fract(u) * 2^32; at most 2^11 terms of a workgroup reach one entry (one
// per point and trace), so the sum stays below 2^61.
__device__ inline void fx_add(unsigned long long *g, float u)
{
    const int hi = cvt_flr(u);
    const unsigned lo = (unsigned)(__builtin_amdgcn_fractf(u) * 4294967296.f);
    atomicAdd(g, ((unsigned long long)(unsigned)hi << 32) | lo);
}

// Adjoint of one read for the RF gradient: adds ga times the read's tap
// weights to the trace's LDS accumulation window, whose entry r stands for
// sample w0 - 1 + r (k = the read's clamped interval index; the cubic read
// touches taps n-1 .. n+2, the linear read n, n+1).  The weights are the
// coefficients of each tap in the cubic-Hermite (or linear) read, all in
// [-1, 1]; ga carries the workgroup's fixed-point scale.
template <int IP>
__device__ inline void scatter_taps(unsigned long long *gwin, int k, float ga, float t)
{
    if (ga == 0.f) return;
    unsigned long long *g = gwin + k;
    if constexpr (IP == IN_CUBIC) {
        const float t2 = t * t;
        fx_add(g, ga * (t * fmaf(t, fmaf(-0.5f, t, 1.f), -0.5f)));
        fx_add(g + 1, ga * fmaf(t2, fmaf(1.5f, t, -2.5f), 1.f));
        fx_add(g + 2, ga * (t * fmaf(t, fmaf(-1.5f, t, 2.f), 0.5f)));
        fx_add(g + 3, ga * (0.5f * t2 * (t - 1.f)));
    } else {
        fx_add(g + 1, ga - ga * t);
        fx_add(g + 2, ga * t);
    }
}

// Adds a batch's accumulation windows (nb slots of lw entries) to grad_e and
// clears them; unit = the value of one fixed-point step.  Slot e's trace and
// window start come from lane e of td (a lane permute, so the loop keeps
// every lane active); other workgroups add to the same samples, hence
// global atomics.  Entries that stayed zero are skipped.
__device__ inline void flush_grad_e(const DasArgs &a, const LdsCfg &c, unsigned long long *accw,
                                    const TraceDesc &td, int lw, float inv_lw, double unit)
{
    const int total = c.nb * lw;
    for (int base = 0; base < total; base += blockDim.x) {
        const int g = base + threadIdx.x;
        // (g + 1/2) / lw is at least 1 / (2 lw) from an integer
        const int e = min((int)(((float)g + 0.5f) * inv_lw), 63);
        const int w0 = __builtin_amdgcn_ds_bpermute(e << 2, td.sw);
        const int off = __builtin_amdgcn_ds_bpermute(e << 2, td.off);
        if (g < total) {
            const long long v = (long long)accw[g];
            if (v != 0) {
                accw[g] = 0ull;
                const int r = g - e * lw;          // sample w0 - 1 + r, element off - 1 + r
                const int n = w0 - 1 + r;
                if (w0 != NO_DATA && (unsigned)n < (unsigned)a.S)
                    unsafeAtomicAdd(a.grad_e + (off - 1 + r), (float)((double)v * unit));
            }
        }
    }
}

// One HERCULES trace for the lane's ZP points: receiver at lateral offset
// (x - xi, dy) from all of them (same x, y), trace window `win` starting at
// sample interval w0 (passed negated, uniform).  The excess receive path in
// samples, k rho^2 / (d + z), is evaluated as rho^2 / (d/k + z/k) with
// d/k = sqrt(rho^2 / k^2 + (z/k)^2): the scale k is folded into the lane
// constants (ik2 = 1 / k^2).
// HF (real-data forward reads, cubic or linear): the lanes' fB hold
// fB + nB - nR for the box's reference sample nR, and neg_w0 carries the
// LDS byte address of the trace's window less (w0 - nR) quads, so a read's
// address is floor(s) * 16 plus that value: one shift-add per point.
template <int ET, int IP, int ZP, int ADJ, bool HF = false>
__device__ inline void hercules_term(const LaneL (&L)[ZP], const float4 *win, int lmax,
                                     const float2 *hann, float dy2, float ik2, float rot, float xi,
                                     int neg_w0, float2 (&acc)[ZP],   // neg_w0: from LDS
                                     unsigned long long *gwin, const float (&G)[ZP])
{
    static_assert(!HF || (ET != ET_CF32 && ADJ == 0 && IP != IN_NEAREST),
                  "folded reads: real-data forward, cubic or linear");
    const float dx = L[0].x - xi;
    const float rho2 = fmaf(dx, dx, dy2);
#pragma unroll
    for (int p = 0; p < ZP; ++p) {
        const float dk = __builtin_amdgcn_sqrtf(fmaf(rho2, ik2, L[p].zk2));
        const float s = fmaf(rho2, __builtin_amdgcn_rcpf(dk + L[p].zk), L[p].fB);
        const int li = HF ? 0 : add3_vvv(cvt_flr(s), L[p].nB, neg_w0);
        // Hann weight from the LDS table; u^2 >= 1/4 lands on the (0, 0) entry
        const float xw = rho2 * L[p].wtab;
        const float2 h = hann[min((unsigned)cvt_flr(xw), (unsigned)HANN_N)];
        const float w = fmaf(xw, h.y, h.x);
        // no clamp: li lies in [-1, lmax + guard) for every lane (its
        // geometry is inside the box); -1 reads the finite LDS word before the
        // windows, and lanes outside their aperture (weight exactly 0) may
        // read past their window into the next one or the zeroed guard
        const float t = __builtin_amdgcn_fractf(s);
        if constexpr (ET == ET_CF32) {
            const float2 v = make_float2(eval_quad<IP>(win[2 * li], t), eval_quad<IP>(win[2 * li + 1], t));
            rotate_acc(v, w, fmaf(rot, s, L[p].ph0), acc[p]);
        } else if constexpr (ADJ != 0) {
            if constexpr ((ADJ & 1) != 0) {
                // dL/dc: sums of w v'(s) and w v'(s) s (derivative quads)
                const float wv = w * eval_dquad<IP>(win[li], t);
                acc[p].x += wv;
                acc[p].y = fmaf(wv, s, acc[p].y);
            }
            if constexpr ((ADJ & 2) != 0)   // RF gradient (active lanes lie inside the window)
                scatter_taps<IP>(gwin, clamp0_i32(li, lmax - 1), G[p] * w, t);
        } else if constexpr (HF) {
            const unsigned ad = ((unsigned)cvt_flr(s) << 4) + (unsigned)neg_w0;
            const float v = eval_quad<IP>(lds_read_f4(ad), t);
            acc[p].x = fmaf(w, v, acc[p].x);
        } else {
            const float v = eval_quad<IP>(win[li], t);
            acc[p].x = fmaf(w, v, acc[p].x);
        }
    }
}

// Beamforms workgroup box `blk` (channel group `grp`) of one frame.  Every
// thread of the workgroup must call it (it contains barriers).
// ADJ: the adjoint of the image instead of the image, for G = dL/d(image).
// Bit 1, dL/dc: the staged quads hold the read's derivative, each point
// accumulates sum w v'(s) and sum w v'(s) s, and the workgroup writes its
// FP64 partial of dL/dc = -1/c sum_p G(p) sum_terms w v'(s) (s + nB + t0 fs)
// (the delay's derivative: ds/dc = -(s_abs + t0 fs)/c).  Bit 2, dL/de: every
// term adds G(p) w times its read's tap weights to an LDS window per trace
// in 64-bit fixed point, scaled by the box's largest |G| (two sets of
// windows, one per batch buffer); a batch's windows go to grad_e while the
// next batch is beamformed.  Without bit 1 no data are staged.
template <int MODE, int ET, int IP, int ZP, int ADJ = 0>
__device__ inline void das_block(const DasArgs &a, const LdsCfg &c, int blk, int grp,
                                 float4 *smem)
{
    static_assert(ADJ == 0 || ET != ET_CF32, "the adjoint is defined for real data");
    constexpr bool GC = (ADJ & 1) != 0, GE = (ADJ & 2) != 0;
    constexpr bool STAGE = ADJ == 0 || GC;       // data windows needed
    static_assert(ZP == 1 || ((MODE == MODE_HERCULES || MODE == MODE_FORCES) && ET != ET_CF32),
                  "two points per lane: HERCULES and FORCES with real data");
    constexpr int QM = stage_rounds(MODE, ET == ET_CF32);
    const int nthr = blockDim.x;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int nwaves = nthr >> 6;

    // tables: tx_x, rx_c, the box's path bounds tx_lo, rx_lo (separable
    // modes; FOLD: their integer window-start parts), the window starts of the
    // two batch buffers (negated; read by the terms with one LDS load instead
    // of a lane broadcast; zeros under FOLD, whose terms need none), Hann
    // weights (HERCULES; the separable modes weight rows with the polynomial),
    // then two buffers of [nb * lmax] quads (the Hann table, or the zeroed
    // window starts, sit right before them: an index of -1 reads finite data)
    constexpr bool SEP = MODE != MODE_HERCULES;
    // Separable forward kernels on real data fold the window start into the
    // paths.  The start of trace (i, j) is split as A_i + B_j, with
    //   A_i = floor(k tx_lo_i - Zb),  B_j = floor(k rx_lo_j + Zb - t0 fs) - 2,
    // Zb = k times the box's top depth (it keeps both parts, and the sums
    // below, near the window length).  A_i + B_j is at most 2 samples below
    // the box's lowest path (floor(u) + floor(v) <= u + v) and at most one
    // sample below the unsplit start floor(k (tx_lo + rx_lo) - t0 fs) - 2,
    // so the windows grow by one quad.  A term's window position is then
    //   (fB + k E_rx + nB - B_j) + (k E_tx - A_i),
    // the first sum per (point, row) once per row chunk, the second per
    // (point, transmit): its floor is the quad index and no integer add per
    // term is left.  The sums are kept centred, less hc = lmax / 4 quads (the
    // window base pointer is moved by hc instead): active positions fill about
    // the lower two thirds of a window, and FP32 rounds them at a quarter of
    // the window's magnitude.  Nearest reads keep the unsplit position: their
    // sample choice is an integer decision that extra rounding would move at
    // near ties.
    constexpr bool FOLD = SEP && ADJ == 0 && ET != ET_CF32 && IP != IN_NEAREST;
    // HERCULES forward reads on real data fold the lane's integer sample nB,
    // less a box reference nR, into its FP32 position (hercules_term, HF);
    // nearest reads keep the unsplit position, as above
    constexpr bool HF = MODE == MODE_HERCULES && ADJ == 0 && ET != ET_CF32 && IP != IN_NEAREST;
    const int hc = FOLD ? c.lmax >> 2 : 0;
    const int ntx4 = (a.n_tx + 3) & ~3, nch4 = (a.n_ch + 3) & ~3;
    float *s_tx = reinterpret_cast<float *>(smem);
    float *s_rx = s_tx + ntx4;
    float *s_lo = s_rx + nch4;                     // [ntx4] tx_lo, then [nch4] rx_lo
    // (indexed from one base so that the compiler keeps them in LDS)
    int *s_w0 = reinterpret_cast<int *>(s_lo + (SEP ? ntx4 + nch4 : 0));
    const int w0_stride = (c.nb + 3) & ~3;
    float2 *s_hann = reinterpret_cast<float2 *>(s_w0 + 2 * w0_stride);
    float4 *bufbase = reinterpret_cast<float4 *>(s_hann + (MODE == MODE_HERCULES ? HANN_TAB_PAD : 0));
    constexpr int QS = ET == ET_CF32 ? 2 : 1;     // quads per sample interval
    const int buf_quads = STAGE ? c.nb * c.lmax * QS : 0;
    float4 *q0 = bufbase, *q1 = bufbase + buf_quads;
    // RF gradient: two sets of nb accumulation windows of lmax + 3 fixed-point
    // entries, then the wavefronts' maxima of |G|
    const int lw = c.lmax + 3;
    unsigned long long *accw0 =
        reinterpret_cast<unsigned long long *>(q1 + buf_quads + (STAGE ? c.guard * QS : 0));
    unsigned long long *accw1 = accw0 + (GE ? c.nb * lw : 0);
    float *s_gmax = reinterpret_cast<float *>(accw1 + (GE ? c.nb * lw : 0));
    for (int t = tid; t < a.n_tx; t += nthr) s_tx[t] = as_global(a.tx_x)[t];
    for (int t = tid; t < a.n_ch; t += nthr) s_rx[t] = as_global(a.rx_c)[t];
    if constexpr (MODE == 1)
        for (int t = tid; t < HANN_TAB_PAD; t += nthr)
            s_hann[t] = t <= HANN_N ? load_f2(a.hann_tab, t) : make_float2(0.f, 0.f);
    if constexpr (STAGE)   // finite data wherever an unclamped read can land
        for (int t = tid; t < buf_quads + c.guard * QS; t += nthr) q1[t] = make_float4(0.f, 0.f, 0.f, 0.f);
    if constexpr (GE)
        for (int t = tid; t < 2 * c.nb * lw; t += nthr) accw0[t] = 0ull;

    const int bz = blk % c.blocks_z;
    const int bx = (blk / c.blocks_z) % c.blocks_x;
    const int by = blk / (c.blocks_z * c.blocks_x);
    const BoxGeom box = block_box(a, c, bx, by, bz);
    if constexpr (SEP) {   // the box's path bounds (read after the barrier below)
        const float zb = box.kf * fmaxf(box.zmin, 0.f);
        for (int t = tid; t < a.n_tx; t += nthr) {
            const float lo = tx_lo<MODE>(a, box, t, as_global(a.tx_x)[t]);
            s_lo[t] = FOLD ? floorf(fmaf(box.kf, lo, -zb)) : lo;
        }
        for (int t = tid; t < a.n_ch; t += nthr) {
            const float lo = rx_lo<MODE>(box, as_global(a.rx_c)[t]);
            s_lo[ntx4 + t] = FOLD ? floorf(fmaf(box.kf, lo, zb - box.t0f)) - 2.f : lo;
        }
    }
    if constexpr (FOLD)    // the terms keep no window starts; an index of -1 reads these zeros
        for (int t = tid; t < 2 * w0_stride; t += nthr) s_w0[t] = 0;
    // HF: nR = the sample of the two-way path txlo + zmax, near the middle of
    // the box's delays B (the same integer in every thread), so the lanes'
    // folded positions B - nR + excess stay near the excess path's magnitude
    const int nR = HF ? (int)floorf(fmaf(box.txlo + fmaxf(box.zmax, 0.f), box.kf, -box.t0f)) : 0;
    LaneL Lp[ZP];
#pragma unroll
    for (int p = 0; p < ZP; ++p) Lp[p] = lane_setup_l<MODE>(a, c, bx, by, bz, wave, lane, p, HF ? &nR : nullptr);
    const LaneL &L = Lp[0];
    // largest rho^2 bound of the receive aperture over the lane's points
    float thr_l = Lp[0].thr;
#pragma unroll
    for (int p = 1; p < ZP; ++p) thr_l = fmaxf(thr_l, Lp[p].thr);
    const float kf = (float)a.k;
    const float ik2 = uniform_f((float)(1.0 / (a.k * a.k)));
    const float rot = a.rot;
    float2 acc[ZP];
#pragma unroll
    for (int p = 0; p < ZP; ++p) acc[p] = make_float2(0.f, 0.f);
    // G(p) of the lane's points (RF gradient; 0 outside the grid and at z <= 0,
    // where the image is 0)
    float Gv[ZP];
#pragma unroll
    for (int p = 0; p < ZP; ++p) {
        Gv[p] = 0.f;
        if constexpr (GE) {
            int ix, iy, iz;
            lane_point(a, c, bx, by, bz, wave, lane, p, &ix, &iy, &iz);
            if (ix < a.g.nx && iy < a.g.ny && iz >= 0 && iz < a.g.nz) {
                const double pz = a.g.org[2] + ix * a.g.ax[2] + iy * a.g.ay[2] + iz * a.g.az[2];
                if (pz > 0.0) Gv[p] = as_global(a.grad_out)[((long)iy * a.g.nx + ix) * a.g.nz + iz];
            }
        }
    }
    const float inv_lw = 1.f / (float)lw;
    if constexpr (GE) {
        float m = 0.f;
#pragma unroll
        for (int p = 0; p < ZP; ++p) m = fmaxf(m, fabsf(Gv[p]));
        m = wave_max(m);
        if (lane == 0) s_gmax[wave] = m;
    }
    __syncthreads();
    // fixed-point scale of the RF gradient: the box's largest |G| maps to 2^18
    // (G must be finite)
    double gunit = 0.0;
    if constexpr (GE) {
        float m = 0.f;
        for (int w = 0; w < nwaves; ++w) m = fmaxf(m, s_gmax[w]);
        const float scale = m > 0.f ? 262144.f / m : 0.f;
#pragma unroll
        for (int p = 0; p < ZP; ++p) Gv[p] *= scale;
        gunit = (double)m * 0x1p-50;          // one fixed-point step = m 2^-18 2^-32
    }

    int jb, je;
    group_rows(a.n_ch, grp, a.groups, &jb, &je);
    Iter it;
    it.j = MODE == 1 ? jb - 1 : jb;
    it.jend = je;
    it.i = MODE == 1 ? 0 : a.n_tx;
    it.ihi = 0;
    for (int q = 0; q < JC; ++q) it.rows[q] = -1;

    BatchDesc cur = next_batch<MODE>(a, c, box, s_tx, s_rx, it);
    Staged<QM> st;
    TraceDesc td = {0, 0.f, NO_DATA, 0};   // descriptors of the current batch
    if (cur.valid) {
        td = trace_desc<MODE, FOLD>(a, c, box, s_tx, s_rx, s_lo, ntx4, cur, lane);
        if constexpr (STAGE) {
            stage_load<ET, QM>(a, c, td, st, wave, lane, nwaves);
            stage_store<IP, QS, QM, GC>(c, st, q0, wave, lane, nwaves);
        }
        if constexpr (HF)
            store_w0_addr(c, td, s_w0, q0, nR, wave, lane);
        else if constexpr (!FOLD)
            store_w0(c, td, s_w0, wave, lane);
    }
    TraceDesc td_prev = td;            // RF gradient: windows of the previous batch
    __syncthreads();

    // per-row lane state
    int row_j = -1;
    float dy2 = 0.f, wlo = 0.f, whi = 0.f;              // HERCULES
    int rows_cur[JC];
    float Rj[JC][ZP], aj[JC][ZP];
    bool row_on[JC];
    for (int q = 0; q < JC; ++q) {
        rows_cur[q] = -1;
        row_on[q] = false;
        for (int p = 0; p < ZP; ++p) { Rj[q][p] = 0.f; aj[q][p] = 0.f; }
    }

    int bi = 0;
    while (cur.valid) {
        BatchDesc nxt = next_batch<MODE>(a, c, box, s_tx, s_rx, it);
        TraceDesc td_n = {0, 0.f, NO_DATA, 0};
        if (nxt.valid) {
            td_n = trace_desc<MODE, FOLD>(a, c, box, s_tx, s_rx, s_lo, ntx4, nxt, lane);
            if constexpr (STAGE) stage_load<ET, QM>(a, c, td_n, st, wave, lane, nwaves);
        }
        // the previous batch's gradient windows (complete since the last barrier)
        if constexpr (GE)
            if (bi > 0) flush_grad_e(a, c, (bi & 1) ? accw0 : accw1, td_prev, lw, inv_lw, gunit);

        const float4 *quads = (bi & 1) ? q1 : q0;
        unsigned long long *accw = (bi & 1) ? accw1 : accw0;
        const TraceDesc &mine = td;
        if constexpr (MODE == 1) {
            if (cur.j != row_j) {
                row_j = cur.j;
                const float dy = L.y - s_rx[row_j];
                dy2 = dy * dy;
                const float r2 = thr_l - dy2;
                const float r = r2 > 0.f ? sqrtf(r2) : 0.f;
                wlo = uniform_f(wave_min(r2 > 0.f ? L.x - r : __builtin_inff()));
                whi = uniform_f(wave_max(r2 > 0.f ? L.x + r : -__builtin_inff()));
            }
            // traces inside the union of this wavefront's receive apertures
            // (a contiguous run: the columns are sorted within a batch), in
            // pairs whose LDS reads overlap, then an odd last one
            uint64_t mask = __ballot(lane < cur.cnt && mine.xi >= wlo && mine.xi <= whi);
            // per trace: the column position from the read-only table through
            // the scalar cache (uniform index) and the negated window start
            // from LDS -- no lane broadcasts (their SGPR results stall the wave)
            const cptr<float> txcol = as_const(a.tx_x) + cur.i0;
            const int *wst = s_w0 + (bi & 1) * w0_stride;
            if constexpr (ZP == 2) {
                // one trace per step already gives two independent terms
                while (mask) {
                    const int e1 = __builtin_ctzll(mask);
                    mask &= mask - 1;
                    hercules_term<ET, IP, ZP, ADJ, HF>(Lp, quads + e1 * c.lmax * QS, c.lmax, s_hann, dy2,
                                              ik2, rot, txcol[e1], wst[e1], acc, accw + e1 * lw, Gv);
                }
            }
            while (mask & (mask - 1)) {
                const int e1 = __builtin_ctzll(mask);
                mask &= mask - 1;
                const int e2 = __builtin_ctzll(mask);
                mask &= mask - 1;
                hercules_term<ET, IP, ZP, ADJ, HF>(Lp, quads + e1 * c.lmax * QS, c.lmax, s_hann, dy2, ik2,
                                          rot, txcol[e1], wst[e1], acc, accw + e1 * lw, Gv);
                hercules_term<ET, IP, ZP, ADJ, HF>(Lp, quads + e2 * c.lmax * QS, c.lmax, s_hann, dy2, ik2,
                                          rot, txcol[e2], wst[e2], acc, accw + e2 * lw, Gv);
            }
            if (mask) {
                const int e1 = __builtin_ctzll(mask);
                hercules_term<ET, IP, ZP, ADJ, HF>(Lp, quads + e1 * c.lmax * QS, c.lmax, s_hann, dy2, ik2,
                                          rot, txcol[e1], wst[e1], acc, accw + e1 * lw, Gv);
            }
        } else {
            // receive paths and weights of the batch's rows (on a new chunk);
            // the lane's ZP points share the lateral offset to a row
#pragma unroll
            for (int q = 0; q < JC; ++q) {
                if (cur.rows[q] != rows_cur[q]) {
                    rows_cur[q] = cur.rows[q];
                    const int row = slot_row(rows_cur[q]);
                    const float dxr = rx_coord<MODE>(L.x, L.y) - s_rx[row];
                    const float r2 = dxr * dxr;
                    const int bj = FOLD ? (int)s_lo[ntx4 + row] : 0;
                    bool any = false;
#pragma unroll
                    for (int p = 0; p < ZP; ++p) {
                        const bool act = r2 < Lp[p].thr && !slot_pad(rows_cur[q]);
                        Rj[q][p] = fmaf(excess(r2, Lp[p].z, Lp[p].z2), kf, Lp[p].fB);
                        if constexpr (FOLD) Rj[q][p] += (float)(Lp[p].nB - bj - hc);
                        aj[q][p] = act ? hann_u2(r2 * Lp[p].wsc) : 0.f;
                        any = any || act;
                    }
                    row_on[q] = __any(any);
                }
            }
            const int4 *wst4 = reinterpret_cast<const int4 *>(s_w0 + (bi & 1) * w0_stride);
            // the transmits' table entries through the scalar cache (uniform)
            const cptr<float> tscf = as_const(reinterpret_cast<const float *>(a.tx_sc)) + 2 * cur.i0;
            const cptr<float> txc = as_const(a.tx_x) + cur.i0;
            // the next transmit's scalars are fetched one transmit ahead, so
            // their latency overlaps the current transmit's terms
            float2 tsc_n = MODE == MODE_TPW ? make_float2(tscf[0], tscf[1]) : make_float2(0.f, 0.f);
            float xi_n = MODE == MODE_TPW ? 0.f : txc[0];
            static_assert(JC % 4 == 0, "the window starts of a transmit are JC / 4 int4 loads");
            constexpr int NW4 = JC / 4;
            int4 nw4_n[NW4];
            float ai_n = 0.f;                 // FOLD: A_i of the next transmit
            if constexpr (FOLD) {
                ai_n = s_lo[cur.i0];
            } else {
#pragma unroll
                for (int r = 0; r < NW4; ++r) nw4_n[r] = wst4[r];
            }
            for (int ii = 0; ii < cur.cnt; ++ii) {
                const float2 tsc = tsc_n;
                const float xi = xi_n;
                const float ai = ai_n;
                int nw[JC];                   // negated window starts of the JC rows
                if constexpr (!FOLD) {
#pragma unroll
                    for (int r = 0; r < NW4; ++r) {
                        nw[4 * r] = nw4_n[r].x;
                        nw[4 * r + 1] = nw4_n[r].y;
                        nw[4 * r + 2] = nw4_n[r].z;
                        nw[4 * r + 3] = nw4_n[r].w;
                    }
                }
                const int in = min(ii + 1, cur.cnt - 1);
                if constexpr (MODE == MODE_TPW)
                    tsc_n = make_float2(tscf[2 * in], tscf[2 * in + 1]);
                else
                    xi_n = txc[in];
                if constexpr (FOLD) {
                    ai_n = s_lo[cur.i0 + in];
                } else {
#pragma unroll
                    for (int r = 0; r < NW4; ++r) nw4_n[r] = wst4[NW4 * in + r];
                }
                // transmit excess path of each of the lane's points, shared by
                // the batch's rows (FOLD: minus A_i)
                float T[ZP];
#pragma unroll
                for (int p = 0; p < ZP; ++p) {
                    const float ex = tx_excess_p<MODE>(L.x, Lp[p].z, Lp[p].z2, tsc, xi, a.zf);
                    T[p] = FOLD ? fmaf(kf, ex, -ai) : kf * ex;
                }
                // every slot holds a real row (padding slots have weight 0 and
                // a zero window), so the forward and dL/dc terms of the JC rows
                // run without branches and their LDS reads overlap; the RF
                // gradient skips rows no lane of the wavefront receives
#pragma unroll
                for (int q = 0; q < JC; ++q) {
                    if (GE && !row_on[q]) continue;
                    const int e = ii * JC + q;            // slot: transmit-major
#pragma unroll
                    for (int p = 0; p < ZP; ++p) {
                        const float sq = Rj[q][p] + T[p];
                        // no clamp: li lies in [1, lmax + guard) for every lane
                        // (its geometry is inside the box; FOLD: li + hc, and
                        // in [0, ...) with the rounding of the folded sums);
                        // lanes outside the row's aperture (weight 0) may read
                        // into the next window or the zeroed guard
                        int li;
                        if constexpr (FOLD)
                            li = cvt_flr(sq);
                        else
                            li = add3_vvv(cvt_flr(sq), Lp[p].nB, nw[q]);
                        if constexpr (ET == ET_CF32) {
                            const float4 *win = quads + e * c.lmax * QS;
                            const float t = __builtin_amdgcn_fractf(sq);
                            const float2 v = make_float2(eval_quad<IP>(win[2 * li], t),
                                                         eval_quad<IP>(win[2 * li + 1], t));
                            rotate_acc(v, aj[q][p], fmaf(rot, sq, Lp[p].ph0), acc[p]);
                        } else if constexpr (ADJ != 0) {
                            // the RF gradient's scatter stays inside the window;
                            // dL/dc alone reads unclamped, as the forward terms do
                            const int k = GE ? clamp0_i32(li, c.lmax - 1) : li;
                            const float t = __builtin_amdgcn_fractf(sq);
                            if constexpr (GC) {
                                const float wv = aj[q][p] * eval_dquad<IP>(quads[e * c.lmax + k], t);
                                acc[p].x += wv;
                                acc[p].y = fmaf(wv, sq, acc[p].y);
                            }
                            if constexpr (GE)
                                scatter_taps<IP>(accw + e * lw, k, Gv[p] * aj[q][p], t);
                        } else {
                            // (FOLD: li counts from quad hc of the window)
                            const float v = eval_quad<IP>(quads[(e * c.lmax + hc) + li],
                                                          __builtin_amdgcn_fractf(sq));
                            acc[p].x = fmaf(aj[q][p], v, acc[p].x);
                        }
                    }
                }
            }
        }

        if (!nxt.valid) break;
        if constexpr (STAGE) stage_store<IP, QS, QM, GC>(c, st, ((bi + 1) & 1) ? q1 : q0, wave, lane, nwaves);
        if constexpr (HF)
            store_w0_addr(c, td_n, s_w0 + ((bi + 1) & 1) * w0_stride, ((bi + 1) & 1) ? q1 : q0, nR, wave,
                          lane);
        else if constexpr (!FOLD)
            store_w0(c, td_n, s_w0 + ((bi + 1) & 1) * w0_stride, wave, lane);
        __syncthreads();
        cur = nxt;
        td_prev = td;
        td = td_n;
        ++bi;
    }
    if constexpr (GE) {               // the last batch's gradient windows
        __syncthreads();
        flush_grad_e(a, c, (bi & 1) ? accw1 : accw0, td, lw, inv_lw, gunit);
    }
    // the point indices are recomputed here (an opaque copy of the lane
    // number), so they hold no registers during the loop
    int lane_e = lane;
    asm volatile("" : "+v"(lane_e));
    if constexpr (ADJ != 0) {
        if constexpr (!GC) return;
        double contrib = 0.0;
#pragma unroll
        for (int p = 0; p < ZP; ++p) {
            int ix, iy, iz;
            lane_point(a, c, bx, by, bz, wave, lane_e, p, &ix, &iy, &iz);
            if (ix < a.g.nx && iy < a.g.ny && iz >= 0 && iz < a.g.nz) {
                const double pz = a.g.org[2] + ix * a.g.ax[2] + iy * a.g.ay[2] + iz * a.g.az[2];
                if (pz > 0.0) {
                    const double G = a.grad_out[((long)iy * a.g.nx + ix) * a.g.nz + iz];
                    contrib += G * ((double)acc[p].y + ((double)Lp[p].nB + a.t0fs) * (double)acc[p].x);
                }
            }
        }
        // workgroup sum in a fixed order -> one partial per (box, channel group)
        __shared__ double red[16];
        for (int off = 32; off > 0; off >>= 1) contrib += __shfl_down(contrib, off, 64);
        if (lane == 0) red[wave] = contrib;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int w = 0; w < nwaves; ++w) t += red[w];
            a.partial[(long)grp * gridDim.x + blockIdx.x] = -t / a.c;
        }
        return;
    }
    const long npts = (long)a.g.nx * a.g.ny * a.g.nz;
    float *dst = a.groups > 1 ? a.part + (long)grp * npts * QS : das_out(a);
#pragma unroll
    for (int p = 0; p < ZP; ++p) {
        int ix, iy, iz;
        lane_point(a, c, bx, by, bz, wave, lane_e, p, &ix, &iy, &iz);
        if (ix < a.g.nx && iy < a.g.ny && iz >= 0 && iz < a.g.nz) {
            const long idx = ((long)iy * a.g.nx + ix) * a.g.nz + iz;
            const double pz = a.g.org[2] + ix * a.g.ax[2] + iy * a.g.ay[2] + iz * a.g.az[2];
            const float2 v = pz > 0.0 ? acc[p] : make_float2(0.f, 0.f);
            if constexpr (ET == ET_CF32)
                store_f2(reinterpret_cast<float2 *>(dst), idx, v);
            else
                as_global_mut(dst)[idx] = v.x;
        }
    }
}

// Box order of the single-frame kernels (DAS and its adjoints).  Workgroups are dispatched in index
// order, round-robin over the 8 XCDs (index b runs on XCD b % 8), and each
// XCD has its own L2.  XCD x takes the depth slabs x, x + 8, x + 16, ... (a
// slab = every lateral box at one box depth), deepest first: the boxes
// resident on an XCD at a time lie side by side at one depth and stage
// nearly the same trace windows, which then hit in that XCD's L2, and the
// costliest boxes (the widest apertures) start first.  The grid holds
// xcd_slab_grid(c) = nlat * 8 * ceil(blocks_z / 8) workgroups; those past
// the last slab return.
// Any order is correct (each box is visited once); this one measured 5 %
// faster than depth-fastest order on the 128 x 128 x 256 HERCULES volume.
__device__ inline int xcd_slab_box(const LdsCfg &c, int b)
{
    const int nlat = c.blocks_x * c.blocks_y;
    const int slot = b >> 3;
    const int zrank = (slot / nlat) * 8 + (b & 7);     // 0 = deepest slab
    if (zrank >= c.blocks_z) return -1;
    return (c.blocks_z - 1 - zrank) + c.blocks_z * (slot % nlat);
}

// Registers capped for two workgroups per CU: 6 wavefronts per SIMD for
// HERCULES and the row-column modes (12-wavefront workgroups; without the
// cap the IQ volume kernel took 81 VGPRs, one workgroup per CU: 58 ms
// against 42 ms); FORCES planes 8 with one point per lane (16-wavefront
// workgroups; without the cap the plane kernel's registers left room for
// one workgroup per CU: 0.19 ms against 0.15 ms on the 256 x 256 plane of
// 64 x 64 traces) and 4 with two (8-wavefront workgroups).
template <int MODE, int ZP> struct WavesPerEu {
    static constexpr int value = MODE == MODE_FORCES ? (ZP == 2 ? 4 : 8)
                                 : (MODE == MODE_HERCULES || MODE == MODE_TPW || MODE == MODE_VLS) ? 6 : 1;
};

// Dynamic LDS beyond 64 KiB (gfx950 has 160 KiB per CU) is requested per
// kernel before its launch.
static inline hipError_t allow_lds(const void *fn, size_t shm)
{
    if (shm <= 65536) return hipSuccess;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
}

size_t lds_bytes(int n_tx, int n_ch, int nb, int lmax, int qs, int guard, int adj, int mode);

}  // namespace bf
