// bf_api.hip -- host side of libbf: validation, plans, dispatch, errors.
// See include/bf.h for the contract of every entry point.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "bf.h"
#include "bf_common.h"
#include "bf_plan.h"
#include "bf_test.h"

namespace bf {
hipError_t launch_decode_mfma(const DecodeArgs &a, int kb, int etype, hipStream_t s);
hipError_t launch_decode_fma(const DecodeArgs &a, int etype, hipStream_t s);
hipError_t launch_das(const DasArgs &a, int mode, int et, int ip, hipStream_t s);
hipError_t launch_das_adjoint(const DasArgs &a, int mode, int et, int ip, float *grad_c,
                              hipStream_t s);
hipError_t launch_sharpness(const float *img, long n, int n_images, float *loss, float *grad,
                            hipStream_t s);

static thread_local std::string g_err;

void clear_err() { g_err.clear(); }

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(BF_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

static bool is_fin(double v) { return isfinite(v) != 0; }

// ---------------------------------------------------------------------------
// Validation (no HIP calls)
// ---------------------------------------------------------------------------
int validate_params(const bf_params *p)
{
    if (!p) return fail(BF_ERR_NULL, "params is NULL");
    if (p->mode < BF_FORCES_2D || p->mode > BF_VLS_3D)
        return fail(BF_ERR_UNSUPPORTED, "unknown mode %d", p->mode);
    if (p->interp < BF_INTERP_NEAREST || p->interp > BF_INTERP_CUBIC)
        return fail(BF_ERR_UNSUPPORTED, "unknown interpolation %d", p->interp);
    if (p->e_type < BF_E_F32 || p->e_type > BF_E_I32)
        return fail(BF_ERR_UNSUPPORTED, "unknown decoded-data type %d", p->e_type);
    if (p->decode_algo != BF_DECODE_MFMA_I8 && p->decode_algo != BF_DECODE_FMA_F32)
        return fail(BF_ERR_UNSUPPORTED, "unknown decode algorithm %d", p->decode_algo);
    if (p->iq != 0 && p->iq != 1) return fail(BF_ERR_UNSUPPORTED, "iq must be 0 or 1");
    if (p->iq && p->e_type != BF_E_F32)
        return fail(BF_ERR_UNSUPPORTED, "IQ plans decode to BF_E_F32 only");
    if (p->n_tx < 1 || p->n_tx > 256) return fail(BF_ERR_SHAPE, "n_tx=%d not in [1,256]", p->n_tx);
    if (p->n_ch < 1 || p->n_ch > 1024) return fail(BF_ERR_SHAPE, "n_ch=%d not in [1,1024]", p->n_ch);
    if (p->n_samples < 1 || p->n_samples > 65536)
        return fail(BF_ERR_SHAPE, "n_samples=%d not in [1,65536]", p->n_samples);
    if (p->n_elem[0] < 1 || p->n_elem[1] < 1)
        return fail(BF_ERR_SHAPE, "n_elem must be >= 1");
    for (int a = 0; a < 3; ++a)
        if (p->out_dims[a] < 1) return fail(BF_ERR_SHAPE, "out_dims[%d]=%d < 1", a, p->out_dims[a]);
    const int parts = p->iq ? 2 : 1;
    const int64_t ne = (int64_t)p->n_tx * p->n_ch * p->n_samples * parts;
    if (ne >= (int64_t(1) << 31))
        return fail(BF_ERR_TOO_LARGE, "channel data has %lld elements (limit 2^31)", (long long)ne);
    const int64_t nv = (int64_t)p->out_dims[0] * p->out_dims[1] * p->out_dims[2] * parts;
    if (nv >= (int64_t(1) << 31))
        return fail(BF_ERR_TOO_LARGE, "output has %lld points (limit 2^31)", (long long)nv);
    for (int a = 0; a < 2; ++a)
        if (!is_fin(p->pitch[a]) || p->pitch[a] <= 0.0)
            return fail(BF_ERR_GEOMETRY, "pitch[%d] must be finite and > 0", a);
    for (int q = 0; q < 16; ++q)
        if (!is_fin(p->xdc_transform[q])) return fail(BF_ERR_GEOMETRY, "transform not finite");
    if (p->xdc_transform[12] != 0.0 || p->xdc_transform[13] != 0.0 ||
        p->xdc_transform[14] != 0.0 || p->xdc_transform[15] != 1.0)
        return fail(BF_ERR_GEOMETRY, "transform last row must be 0 0 0 1");
    if (!is_fin(p->fs) || p->fs <= 0.0) return fail(BF_ERR_GEOMETRY, "fs must be finite and > 0");
    if (!is_fin(p->c) || p->c <= 0.0) return fail(BF_ERR_GEOMETRY, "c must be finite and > 0");
    if (!is_fin(p->t0)) return fail(BF_ERR_GEOMETRY, "t0 must be finite");
    if (!is_fin(p->fc) || p->fc < 0.0) return fail(BF_ERR_GEOMETRY, "fc must be finite and >= 0");
    if (!is_fin(p->f_number) || p->f_number < 0.0)
        return fail(BF_ERR_GEOMETRY, "f_number must be finite and >= 0");
    for (int a = 0; a < 3; ++a)
        if (!is_fin(p->out_min[a]) || !is_fin(p->out_max[a]))
            return fail(BF_ERR_GEOMETRY, "output region bounds must be finite");
    if (p->mode == BF_HERCULES_3D && !((isinf(p->focal_depth) && p->focal_depth > 0) ||
                                       (is_fin(p->focal_depth) && p->focal_depth < 0)))
        return fail(BF_ERR_UNSUPPORTED, "HERCULES transmits a plane wave (focal_depth = +inf) "
                                        "or a diverging wave (finite focal_depth < 0)");
    if (p->mode == BF_VLS_3D && !is_fin(p->focal_depth))
        return fail(BF_ERR_GEOMETRY, "VLS needs a finite focal_depth (virtual line depth)");
    if (p->mode == BF_TPW_3D) {
        if (!p->tx_angles) return fail(BF_ERR_NULL, "TPW needs tx_angles");
        for (int i = 0; i < p->n_tx; ++i)
            if (!is_fin(p->tx_angles[i]) || fabs(p->tx_angles[i]) >= 0.5 * M_PI)
                return fail(BF_ERR_GEOMETRY, "tx_angles[%d] must be finite, |angle| < pi/2", i);
    }
    if (p->tx_elements)
        for (int i = 0; i < p->n_tx; ++i)
            if (p->tx_elements[i] < 0 || p->tx_elements[i] >= p->n_elem[0])
                return fail(BF_ERR_SHAPE, "tx_elements[%d]=%d outside [0,%d)", i,
                            p->tx_elements[i], p->n_elem[0]);
    const int nrx = p->mode == BF_FORCES_2D ? p->n_elem[0] : p->n_elem[1];
    if (p->channel_map)
        for (int j = 0; j < p->n_ch; ++j)
            if (p->channel_map[j] < 0 || p->channel_map[j] >= nrx)
                return fail(BF_ERR_SHAPE, "channel_map[%d]=%d outside [0,%d)", j,
                            p->channel_map[j], nrx);
    if (!p->hadamard) return BF_OK;        // unencoded acquisition: identity decode
    const int n = p->n_tx;
    const int8_t *H = p->hadamard;
    for (int q = 0; q < n * n; ++q)
        if (H[q] != 1 && H[q] != -1)
            return fail(BF_ERR_NOT_HADAMARD, "hadamard[%d]=%d is not +-1", q, H[q]);
    for (int a = 0; a < n; ++a)
        for (int b = a; b < n; ++b) {
            int dot = 0;
            for (int q = 0; q < n; ++q) dot += H[a * n + q] * H[b * n + q];
            if (dot != (a == b ? n : 0))
                return fail(BF_ERR_NOT_HADAMARD, "rows %d and %d: dot=%d (H H^T != N I)", a, b, dot);
        }
    return BF_OK;
}

// ---------------------------------------------------------------------------
// Device checks and memory
// ---------------------------------------------------------------------------
static int check_device(int *dev)
{
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count < 1) {
        (void)hipGetLastError();
        return fail(BF_ERR_NO_DEVICE, "no HIP device available");
    }
    e = hipGetDevice(dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, *dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(BF_ERR_NO_DEVICE, "device %d is %s, libbf is built for gfx950", *dev,
                    prop.gcnArchName);
    return BF_OK;
}

void *Frame::alloc(size_t bytes)
{
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    allocs.push_back(p);
    total_bytes += (int64_t)bytes;
    return p;
}

Frame::~Frame()
{
    for (void *p : allocs) (void)hipFree(p);
}

// Build host tables and upload them for one frame.
int Frame::init(const bf_params &src)
{
    p = src;
    const int n = p.n_tx;
    if (p.hadamard) {
        H.assign(p.hadamard, p.hadamard + (size_t)n * n);
    } else {   // unencoded: decoding is the identity (exact copy to the e type)
        H.assign((size_t)n * n, 0);
        for (int i = 0; i < n; ++i) H[(size_t)i * n + i] = 1;
    }
    std::vector<float2> tx_sc;
    if (p.mode == BF_TPW_3D)
        for (int i = 0; i < n; ++i) {
            const double th = p.tx_angles[i], sh = sin(0.5 * th);
            tx_sc.push_back(make_float2((float)sin(th), (float)(-2.0 * sh * sh)));   // cos - 1
            tpw_smax = std::max(tpw_smax, fabs(sin(th)));
        }
    p.tx_angles = nullptr;
    tx.resize(n);
    ch.resize(p.n_ch);
    for (int i = 0; i < n; ++i) tx[i] = p.tx_elements ? p.tx_elements[i] : i;
    for (int j = 0; j < p.n_ch; ++j) ch[j] = p.channel_map ? p.channel_map[j] : j;
    p.hadamard = nullptr;
    p.tx_elements = nullptr;
    p.channel_map = nullptr;

    kb = (n + 31) / 32;
    const int KP = 32 * kb;
    std::vector<int8_t> At((size_t)KP * KP, 0);
    std::vector<int> cs(KP, 0);
    std::vector<float> Hf((size_t)n * KP, 0.f);
    for (int k = 0; k < n; ++k)
        for (int m = 0; m < n; ++m) {
            At[(size_t)m * KP + k] = H[(size_t)k * n + m];
            cs[m] += H[(size_t)k * n + m];
            Hf[(size_t)k * KP + m] = (float)H[(size_t)k * n + m];
        }

    // Lateral reference: centre of the element grid (keeps FP32 offsets small).
    const double cx = 0.5 * (p.n_elem[0] - 1) * p.pitch[0];
    const double cy = 0.5 * (p.n_elem[1] - 1) * p.pitch[1];
    std::vector<float> tx_x(n), rx_c(p.n_ch);
    for (int i = 0; i < n; ++i) tx_x[i] = (float)(tx[i] * p.pitch[0] - cx);
    for (int j = 0; j < p.n_ch; ++j)
        rx_c[j] = (float)(p.mode == BF_FORCES_2D ? ch[j] * p.pitch[0] - cx : ch[j] * p.pitch[1] - cy);

    // Grid: point (ix,iy,iz) = M (min + idx * step) - (cx, cy, 0).
    const double *M = p.xdc_transform;
    double step[3];
    for (int a = 0; a < 3; ++a)
        step[a] = p.out_dims[a] > 1 ? (p.out_max[a] - p.out_min[a]) / (p.out_dims[a] - 1) : 0.0;
    for (int r = 0; r < 3; ++r) {
        grid.org[r] = M[4 * r] * p.out_min[0] + M[4 * r + 1] * p.out_min[1] +
                      M[4 * r + 2] * p.out_min[2] + M[4 * r + 3] - (r == 0 ? cx : r == 1 ? cy : 0.0);
        grid.ax[r] = M[4 * r] * step[0];
        grid.ay[r] = M[4 * r + 1] * step[1];
        grid.az[r] = M[4 * r + 2] * step[2];
    }
    grid.nx = p.out_dims[0];
    grid.ny = p.out_dims[1];
    grid.nz = p.out_dims[2];
    // Default DAS workgroups (fastest in measured sweeps on MI355X; the
    // autotuner can replace them): planes = LDS windows on 32x2-point
    // wavefront tiles; HERCULES volumes = LDS windows, flat 8x8x1 lane tiles
    // with two depth points per lane in a 2x2x3 block (12 wavefronts,
    // 16x16x6 points: two such workgroups fill a CU's LDS) with as many traces
    // per staged batch as the LDS cap and the staging rounds allow.
    if (p.mode == BF_FORCES_2D && (grid.ny == 1 || grid.nx == 1)) {
        // a plane: 32 x 2 points per wavefront along its lateral axis and
        // depth, 2 x 8 wavefronts per LDS workgroup (64 x 16 points), batches
        // of JC rows x nb/JC transmits (on the 256 x 256 plane of 64 x 64
        // traces: DAS 151 us, dL/dc 172 us; 16 x 4 tiles in 4 x 4 wavefronts
        // measured slower in the earlier design, 197 / 228 against 193 / 207 us)
        if (grid.ny == 1) {
            set_tile(5, 0, 1);
            bw[0] = 2; bw[1] = 1; bw[2] = 8;
        } else {
            set_tile(0, 5, 1);
            bw[0] = 1; bw[1] = 2; bw[2] = 8;
        }
        nb = 16;
        // (two depth points per lane, BF_DAS_LDS_Z2 over the same box from 2 x 4
        // wavefronts, issues 16 % fewer instructions but hides less latency
        // at half the wavefronts per SIMD: DAS 151 us both, dL/dc 178 against
        // 172 us, the autofocus step and the cross-plane pair 3-6 % slower)
    } else if (p.mode == BF_TPW_3D || p.mode == BF_VLS_3D) {
        // LDS windows, JC rows x nb/JC transmits per batch (separable paths);
        // VLS windows are longer (the path to the line changes along x too)
        if (p.mode == BF_TPW_3D) set_tile(3, 3, 0); else set_tile(2, 3, 1);
        bw[0] = 2; bw[1] = 2; bw[2] = 3;
        nb = 64;                   // trimmed to the LDS cap and staging rounds
        variant = BF_DAS_LDS;
    } else if (p.iq) {
        // IQ (complex accumulators and quads, one point per lane): 12-wavefront
        // workgroups as for real data, batches up to the LDS cap
        set_tile(3, 3, 0);
        bw[0] = 2; bw[1] = 2; bw[2] = 3;
        nb = 48;
    } else {
        set_tile(3, 3, 0);
        bw[0] = 2; bw[1] = 2; bw[2] = 3;
        nb = 40;
        if (p.mode == BF_HERCULES_3D && grid.nz >= 2) {
            variant = BF_DAS_LDS_Z2;
            nb = 48;   // trimmed to the LDS cap and staging rounds by lds_config
        }
    }
    sorted_tx = 1;
    for (int i = 1; i < n; ++i)
        if (tx_x[i] < tx_x[i - 1]) sorted_tx = 0;
    // equally spaced columns (e.g. the full aperture): the kernels find the
    // transmit range of a channel row by arithmetic instead of a search
    uniform_tx = 0;
    if (n >= 2 && sorted_tx && tx[1] > tx[0]) {
        const int step = tx[1] - tx[0];
        uniform_tx = 1;
        for (int i = 1; i < n; ++i)
            if (tx[i] - tx[i - 1] != step) uniform_tx = 0;
        tx_x0 = tx_x[0];
        tx_inv_dx = (float)(1.0 / (step * p.pitch[0]));
    }

    d_At = (int8_t *)alloc(At.size());
    d_colsum = (int *)alloc(cs.size() * sizeof(int));
    d_Hf = (float *)alloc(Hf.size() * sizeof(float));
    d_tx_x = (float *)alloc(tx_x.size() * sizeof(float));
    d_rx_c = (float *)alloc(rx_c.size() * sizeof(float));
    if (!tx_sc.empty()) {
        d_tx_sc = (float2 *)alloc(tx_sc.size() * sizeof(float2));
        if (!d_tx_sc) return fail(BF_ERR_HIP, "device allocation of the TPW angle table failed");
        hipError_t he = hipMemcpy(d_tx_sc, tx_sc.data(), tx_sc.size() * sizeof(float2),
                                  hipMemcpyHostToDevice);
        if (he != hipSuccess) return hip_fail(he, "upload of the TPW angle table");
    }
    // partial-sum buffer of the adjoint, large enough for any tile: one entry
    // per 4-wavefront block (gather kernel) or per (LDS workgroup, channel
    // group); a box holds at least one wavefront, the slab order pads the
    // boxes to whole groups of 8 depth slabs (at most 8x), and the channel
    // split keeps groups x wavefronts below wavefronts + 8192
    long max_waves = 0;
    for (int lx = 0; lx <= 6; ++lx)
        for (int ly = 0; ly + lx <= 6; ++ly) {
            const int lz = 6 - lx - ly;
            const long w = (long)((grid.nx + (1 << lx) - 1) >> lx) *
                           ((grid.ny + (1 << ly) - 1) >> ly) * ((grid.nz + (1 << lz) - 1) >> lz);
            if (w > max_waves) max_waves = w;
        }
    max_blocks = 8 * (max_waves + 8192);
    d_partial = (double *)alloc((size_t)max_blocks * sizeof(double));
    {
        // Eq. 3 in double precision at u^2 = k / (4 HANN_N): entry k holds the
        // slope D_k = W_{k+1} - W_k and the base W_k - k D_k (with D_k as
        // rounded), so that the weight at table coordinate x in [k, k + 1) is
        // one FMA, base + x D_k
        std::vector<float2> tab(HANN_N + 1);
        std::vector<double> W(HANN_N + 1);
        for (int k = 0; k <= HANN_N; ++k) {
            const double u = sqrt(k / (4.0 * HANN_N));
            const double cu = cos(M_PI * u);
            W[k] = (k == HANN_N) ? 0.0 : cu * cu;
        }
        for (int k = 0; k < HANN_N; ++k) {
            const float d = (float)(W[k + 1] - W[k]);
            tab[k] = make_float2((float)(W[k] - k * (double)d), d);
        }
        tab[HANN_N] = make_float2(0.f, 0.f);
        d_hann = (float2 *)alloc(tab.size() * sizeof(float2));
        if (!d_hann) return fail(BF_ERR_HIP, "device allocation of the Hann table failed");
        hipError_t he = hipMemcpy(d_hann, tab.data(), tab.size() * sizeof(float2), hipMemcpyHostToDevice);
        if (he != hipSuccess) return hip_fail(he, "upload of the Hann table");
    }
    // Small grids give too few wavefronts to fill 256 CUs; split the channel
    // sum over `groups` workgroup sets (>= 8192 wavefronts in flight) and add
    // the partial images in a fixed order afterwards.
    {
        const long nvox = (long)grid.nx * grid.ny * grid.nz;
        const long waves = (nvox + 63) / 64;
        long G = (8192 + waves - 1) / waves;
        const long gmax = p.n_ch / 4 > 1 ? p.n_ch / 4 : 1;
        if (G > 16) G = 16;
        if (G > gmax) G = gmax;
        groups = (int)(G < 1 ? 1 : G);
        if (groups > 1) {
            d_part = (float *)alloc((size_t)groups * nvox * (p.iq ? 2 : 1) * sizeof(float));
            if (!d_part) return fail(BF_ERR_HIP, "device allocation of partial images failed");
        }
    }
    if (!d_At || !d_colsum || !d_Hf || !d_tx_x || !d_rx_c || !d_partial)
        return fail(BF_ERR_HIP, "device allocation for plan tables failed");
    hipError_t e;
    if ((e = hipMemcpy(d_At, At.data(), At.size(), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(d_colsum, cs.data(), cs.size() * sizeof(int), hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (e = hipMemcpy(d_Hf, Hf.data(), Hf.size() * sizeof(float), hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (e = hipMemcpy(d_tx_x, tx_x.data(), tx_x.size() * sizeof(float), hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (e = hipMemcpy(d_rx_c, rx_c.data(), rx_c.size() * sizeof(float), hipMemcpyHostToDevice)) !=
            hipSuccess)
        return hip_fail(e, "upload of plan tables");
    return BF_OK;
}

void Frame::set_tile(int lx_, int ly_, int lz_)
{
    lx = lx_;
    ly = ly_;
    lz = lz_;
}

int64_t Frame::e_elems() const { return (int64_t)p.n_tx * p.n_ch * p.n_samples * (p.iq ? 2 : 1); }
int64_t Frame::out_elems() const { return (int64_t)grid.nx * grid.ny * grid.nz * (p.iq ? 2 : 1); }
int Frame::das_et() const { return p.iq ? ET_CF32 : p.e_type; }
size_t Frame::e_bytes() const { return (size_t)e_elems() * (p.e_type == BF_E_BF16 ? 2 : 4); }

DecodeArgs Frame::decode_args(const int16_t *rf, void *e) const
{
    DecodeArgs a;
    a.rf = rf;
    a.e = e;
    a.At = d_At;
    a.colsum = d_colsum;
    a.Hf = d_Hf;
    a.n_tx = p.n_tx;
    a.n_ch = p.n_ch;
    a.S = p.n_samples * (p.iq ? 2 : 1);   // IQ: (re, im) pairs decode as two samples
    return a;
}

DasArgs Frame::das_args(const void *e, float *out, double c) const
{
    DasArgs a;
    memset(&a, 0, sizeof a);
    a.e = e;
    a.out = out;
    a.tx_x = d_tx_x;
    a.rx_c = d_rx_c;
    a.partial = d_partial;
    a.n_tx = p.n_tx;
    a.n_ch = p.n_ch;
    a.S = p.n_samples;
    a.g = grid;
    a.k = p.fs / c;
    a.t0fs = p.t0 * p.fs;
    a.c = c;
    a.f2 = (float)(p.f_number * p.f_number);
    a.lx = lx;
    a.ly = ly;
    a.lz = lz;
    a.tiles_x = (grid.nx + (1 << lx) - 1) >> lx;
    a.tiles_y = (grid.ny + (1 << ly) - 1) >> ly;
    a.tiles_z = (grid.nz + (1 << lz) - 1) >> lz;
    a.n_waves = a.tiles_x * a.tiles_y * a.tiles_z;
    a.groups = groups;
    a.part = d_part;
    a.hann_tab = d_hann;
    a.cx = p.iq;
    a.rot_d = p.iq ? p.fc / p.fs : 0.0;
    a.rot = (float)a.rot_d;
    a.div_f = (p.mode == BF_HERCULES_3D && is_fin(p.focal_depth)) ? -p.focal_depth : 0.0;
    a.zf = p.mode == BF_VLS_3D ? (float)p.focal_depth : 0.f;
    a.tx_sc = d_tx_sc;
    return a;
}

int Frame::decode(const int16_t *rf, void *e, hipStream_t s) const
{
    const DecodeArgs a = decode_args(rf, e);
    hipError_t err = p.decode_algo == BF_DECODE_FMA_F32 ? launch_decode_fma(a, p.e_type, s)
                                                         : launch_decode_mfma(a, kb, p.e_type, s);
    return err == hipSuccess ? BF_OK : hip_fail(err, "decode launch");
}

// Workgroup box, staged-window length and batch size of the LDS kernel for
// this frame at the sound speed of `a`; false if the window would not fit
// (the direct-gather kernel is used then).
// Dynamic LDS of one workgroup: the device's per-block limit, at most 80 KiB
// so that two workgroups share a CU's 160 KiB.
static size_t lds_cap_bytes()
{
    static const size_t cap = [] {
        int dev = 0, v = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
            v <= 0)
            v = 64 * 1024;
        return std::min<size_t>((size_t)v, 80 * 1024);
    }();
    return cap;
}

// adj: the adjoint's LDS layout (1: dL/dc, 2: dL/de, 3: both), 0 for DAS.
// The wavefront tile is a's; bw_adj (if set) replaces the plan's workgroup
// shape.
bool Frame::lds_config(const DasArgs &a, LdsCfg *cfg, int adj, const int *bw_adj) const
{
    const bool sep = p.mode != BF_HERCULES_3D;   // separable: FORCES, TPW, VLS
    const int *bw = bw_adj ? bw_adj : this->bw;
    const int lx = a.lx, ly = a.ly, lz = a.lz;
    // points per lane along z: two for the HERCULES real-data variant
    const int zp = variant == BF_DAS_LDS_Z2 && z2_ok() ? 2 : 1;
    const int tx = bw[0] << lx, ty = bw[1] << ly, tz = (bw[2] << lz) * zp;
    // VLS: the transmit path jumps at the virtual line's depth (converging
    // above it, diverging below), so no box may hold points of both sides:
    // the box grid is shifted along z to start a box where the side changes.
    // The side is decided as in the kernels (FP32 depth minus FP32 line
    // depth); depth must follow the z index alone.
    int z_off = 0;
    if (p.mode == BF_VLS_3D) {
        if (grid.ax[2] != 0.0 || grid.ay[2] != 0.0) return false;
        const float zf = (float)p.focal_depth;
        auto below = [&](int iz) { return (float)(grid.org[2] + iz * grid.az[2]) - zf < 0.f; };
        for (int iz = 1; iz < grid.nz; ++iz)
            if (below(iz) != below(iz - 1)) {
                z_off = (tz - iz % tz) % tz;
                break;
            }
    }
    double E[3];
    for (int r = 0; r < 3; ++r)
        E[r] = fabs(grid.ax[r]) * (tx - 1) + fabs(grid.ay[r]) * (ty - 1) + fabs(grid.az[r]) * (tz - 1);
    // Bound on the spread of the sample position over the box for the points
    // that contribute (apodization > 0): the delay grows with depth (2 dz on
    // the round trip) and with lateral distance.  The receive path
    // sqrt(rho^2 + z^2) changes with the lateral offset at rate
    // rho / d <= 1 / sqrt(1 + 4 F#^2) inside the receive aperture
    // (F# rho / z < 1/2); points outside it have weight 0 and read a clamped
    // index.  Transmit paths are not apodized: rate 1 (FORCES column
    // cylinder, and a VLS path over the box's x-z diagonal), |sin| of the
    // steepest angle along x for TPW, and a diverging wave changes by at most
    // the box diagonal.  Row receivers (TPW, VLS) see y and z only.
    const double lat = sqrt(E[0] * E[0] + E[1] * E[1]);
    const double srx = p.f_number > 0.0 ? 1.0 / sqrt(1.0 + 4.0 * p.f_number * p.f_number) : 1.0;
    double spread;
    switch (p.mode) {
        case BF_FORCES_2D: spread = 2.0 * E[2] + (1.0 + srx) * E[0]; break;
        case BF_TPW_3D: spread = 2.0 * E[2] + srx * E[1] + tpw_smax * E[0]; break;
        case BF_VLS_3D: spread = E[2] + srx * E[1] + sqrt(E[0] * E[0] + E[2] * E[2]); break;
        default:
            spread = a.div_f > 0.0 ? E[2] + srx * lat + sqrt(lat * lat + E[2] * E[2])
                                   : 2.0 * E[2] + srx * lat;
    }
    // Window of an active point: its quad index floor(s) - w0 lies in
    // [1, k spread + 3] (the start w0 is floored 2 samples below the box's
    // lowest path, the quad covers taps n-1 .. n+2); one quad of FP32 slack.
    // The separable forward kernels on real data with cubic or linear reads
    // split the start into a transmit part and a row part, each floored,
    // which puts it up to one sample lower: one more quad, and one more guard
    // entry (plus one for the rounding of the folded sums).
    const int fold = (sep && adj == 0 && !p.iq && p.interp != BF_INTERP_NEAREST) ? 1 : 0;
    // (real data is staged in pairs of quads: lmax even)
    const bool pairs = stage_pairs(p.iq != 0);
    int lmax = (int)ceil(a.k * spread) + 5 + fold;
    if (pairs) lmax += lmax & 1;
    // The terms read without an index clamp: a lane outside its receive
    // aperture (weight 0) may reach past its window by at most the receive
    // path's extra lateral slope, (1 - srx) times the box's receive-lateral
    // extent (HERCULES: radial; FORCES: x; TPW, VLS: y), into the next window
    // or this zeroed guard
    const double rx_lat = p.mode == BF_HERCULES_3D ? lat : p.mode == BF_FORCES_2D ? E[0] : E[1];
    const int guard = (int)ceil(a.k * (1.0 - srx) * rx_lat) + 3 + 2 * fold;
    const int nthr = 64 * bw[0] * bw[1] * bw[2];
    const int unit = sep ? JC : 1;      // separable modes: JC rows per batch
    int nbb = std::max(nb - nb % unit, unit);
    const size_t lds_cap = lds_cap_bytes();
    const int nwaves = nthr / 64;
    // staging rounds per thread: the batch's quads (real data: pairs of
    // quads) dealt over the workgroup's threads, within the rounds the
    // kernels unroll
    const int max_rounds = stage_rounds(p.mode, p.iq != 0);
    const int per_trace = pairs ? lmax / 2 : lmax;
    auto rounds = [&](int n) { return (n * per_trace + 64 * nwaves - 1) / (64 * nwaves); };
    const int qs = p.iq ? 2 : 1;
    const bool staged = adj == 0 || (adj & 1);    // the RF gradient alone reads no data
    while (nbb >= unit && ((staged && rounds(nbb) > max_rounds) ||
                           lds_bytes(p.n_tx, p.n_ch, nbb, lmax, qs, guard, adj, p.mode) > lds_cap))
        nbb -= unit;
    if (nbb < unit || nthr > 1024) return false;
    cfg->bwx = bw[0];
    cfg->bwy = bw[1];
    cfg->bwz = bw[2];
    cfg->nb = nbb;
    cfg->lmax = lmax;
    cfg->sorted_tx = sorted_tx;
    cfg->uniform_tx = uniform_tx;
    cfg->tx_x0 = tx_x0;
    cfg->tx_inv_dx = tx_inv_dx;
    cfg->inv_lmax = 1.0f / (float)lmax;
    cfg->zp = zp;
    cfg->z_off = z_off;
    cfg->guard = guard;
    cfg->blocks_x = (grid.nx + tx - 1) / tx;
    cfg->blocks_y = (grid.ny + ty - 1) / ty;
    cfg->blocks_z = (grid.nz + z_off + tz - 1) / tz;
    return true;
}

// Wavefront tile and workgroup shape of the RF gradient on the LDS kernel.
// Its terms add to LDS with atomics; lanes of one instruction that hit the
// same entry are serialized, and entries a few apart share LDS banks.  The
// delay grows by about 2 k dz per depth step (two or more samples on the
// usual grids) but hardly changes between laterally adjacent points near a
// trace's own column, so the wavefront runs mostly along depth: 16 lanes
// (measured best against 4 to 64 on the 256 x 256 FORCES plane and the
// 128 x 128 x 256 HERCULES volume), fewer for shallow grids; the rest of the
// lanes and the workgroup's 8 wavefronts lie side by side laterally.
void Frame::adjoint_e_tile(DasArgs *a, int bw_out[3]) const
{
    const int zp = variant == BF_DAS_LDS_Z2 && z2_ok() ? 2 : 1;
    const int nzl = (grid.nz + zp - 1) / zp;
    int lz = 0;
    while (lz < 4 && (1 << lz) < nzl) ++lz;
    const int r = 6 - lz;
    if (grid.ny == 1) {
        a->lx = r;
        a->ly = 0;
        bw_out[0] = 8; bw_out[1] = 1; bw_out[2] = 1;
    } else {
        a->lx = (r + 1) / 2;
        a->ly = r / 2;
        bw_out[0] = 4; bw_out[1] = 2; bw_out[2] = 1;
    }
    a->lz = lz;
    a->tiles_x = (grid.nx + (1 << a->lx) - 1) >> a->lx;
    a->tiles_y = (grid.ny + (1 << a->ly) - 1) >> a->ly;
    a->tiles_z = (grid.nz + (1 << lz) - 1) >> lz;
    a->n_waves = a->tiles_x * a->tiles_y * a->tiles_z;
}

// Two points per lane share their lateral offset to every receiver: HERCULES
// volumes and FORCES planes with real data, and the grid's depth axis along
// the array normal.
bool Frame::z2_ok() const
{
    return (p.mode == BF_HERCULES_3D || p.mode == BF_FORCES_2D) && !p.iq && grid.az[0] == 0.0 &&
           grid.az[1] == 0.0;
}

int Frame::das(const void *e, float *out, double c, hipStream_t s, float *part) const
{
    DasArgs a = das_args(e, out, c);
    if (part) a.part = part;
    LdsCfg cfg;
    hipError_t err;
    if (variant != BF_DAS_GATHER && lds_config(a, &cfg))
        err = launch_das_lds(a, cfg, p.mode, das_et(), p.interp, s);
    else
        err = launch_das(a, p.mode, das_et(), p.interp, s);
    return err == hipSuccess ? BF_OK : hip_fail(err, "DAS launch");
}

// Decode fused into DAS: the LDS kernel of a FORCES plane staging its taps
// from the int16 RF through the plan's H (no decoded-data buffer, one launch
// plus the channel-group sum).  The plan's DAS configuration applies; a
// window that does not fit LDS, the gather variant, a non-FORCES or an IQ
// plan is BF_ERR_UNSUPPORTED.
int Frame::das_fused(const int16_t *rf, float *out, double c, hipStream_t s) const
{
    if (p.mode != BF_FORCES_2D || p.iq)
        return fail(BF_ERR_UNSUPPORTED, "the fused decode + DAS takes FORCES plans with RF data");
    DasArgs a = das_args(rf, out, c);
    a.hf = d_Hf;
    a.hf_ld = 32 * kb;
    LdsCfg cfg;
    if (variant == BF_DAS_GATHER || !lds_config(a, &cfg))
        return fail(BF_ERR_UNSUPPORTED, "the fused decode + DAS needs the LDS kernel "
                                        "(not the gather variant; windows must fit LDS)");
    const hipError_t err = launch_das_lds_fused(a, cfg, p.interp, s);
    return err == hipSuccess ? BF_OK : hip_fail(err, "fused decode + DAS launch");
}

// The per-frame arrays of `a` advanced to frame f0 of a stack.
DasArgs Frame::at_frame(const DasArgs &a, int f0) const
{
    DasArgs b = a;
    const long pts = (long)grid.nx * grid.ny * grid.nz;
    if (b.e) b.e = static_cast<const char *>(b.e) + (size_t)f0 * e_bytes();
    if (b.out) b.out += (size_t)f0 * out_elems();
    if (b.grad_out) b.grad_out += (size_t)f0 * pts;
    if (b.grad_e) b.grad_e += (size_t)f0 * e_elems();
    return b;
}

// A stack of nf frames ([nf][...] arrays) at one sound speed, one launch per
// frame.  (One launch over the stack, grid z = frame, measured no faster on
// the 256 x 256 plane -- its single-frame launch already fills the chip --
// and the frame offsets cost the forward kernels four VGPRs.)
int Frame::das_frames(const void *e, int nf, float *out, double c, hipStream_t s) const
{
    const DasArgs a = das_args(e, out, c);
    for (int f = 0; f < nf; ++f) {
        const DasArgs b = at_frame(a, f);
        const int st = das(b.e, b.out, c, s);
        if (st != BF_OK) return st;
    }
    return BF_OK;
}

// Adjoint of das_frames (grad_out, grad_e: [nf][...]; grad_c: [nf]).
// Linear / cubic reads run the LDS-staged adjoint: dL/de (which reads no
// data) on a depth-major wavefront tile, dL/dc (FP32 data) on the plan's
// tile, as two launches when both are requested, each over a whole stack
// (dL/dc: as many frames per launch as the partial-sum buffer holds).
// Nearest reads, other data types and the gather variant run the gather
// adjoint (FP32 atomics into grad_e) frame by frame.
int Frame::das_adjoint(const void *e, const float *grad_out, double c, float *grad_e,
                       float *grad_c, int nf, hipStream_t s) const
{
    DasArgs a = das_args(e, nullptr, c);
    a.grad_out = grad_out;
    a.grad_e = grad_e;
    const bool lds_ok = p.interp != BF_INTERP_NEAREST && variant != BF_DAS_GATHER;
    DasArgs ae = a;
    LdsCfg ce, cc;
    int bwa[3];
    adjoint_e_tile(&ae, bwa);
    const bool e_lds = grad_e && lds_ok && lds_config(ae, &ce, 2, bwa);
    const bool c_lds = grad_c && lds_ok && p.e_type == BF_E_F32 && lds_config(a, &cc, 1) &&
                       (long)xcd_slab_grid(cc) * a.groups <= max_blocks;
    hipError_t err = hipSuccess;
    if ((grad_e && !e_lds) || (grad_c && !c_lds)) {
        for (int f = 0; f < nf && err == hipSuccess; ++f) {
            DasArgs ag = at_frame(a, f);   // what the LDS kernels do not take, frame f
            if (e_lds) ag.grad_e = nullptr;
            err = launch_das_adjoint(ag, p.mode, p.e_type, p.interp,
                                     c_lds || !grad_c ? nullptr : grad_c + f, s);
        }
    }
    // frames per launch: the whole stack, or as many as the cap allows
    const int cap = stack_cap > 0 ? stack_cap : nf;
    if (e_lds) {
        const int k = std::min(nf, cap);
        for (int f0 = 0; f0 < nf && err == hipSuccess; f0 += k)
            err = launch_das_lds_adjoint(at_frame(ae, f0), ce, p.mode, p.interp, nullptr, s,
                                         std::min(k, nf - f0));
    }
    if (err == hipSuccess && c_lds) {
        DasArgs ac = a;
        ac.grad_e = nullptr;
        // (the dL/dc partials of a launch must fit the plan's partial buffer)
        const int k = (int)std::min<long>(
            std::min(nf, cap), max_blocks / ((long)xcd_slab_grid(cc) * a.groups));
        for (int f0 = 0; f0 < nf && err == hipSuccess; f0 += k)
            err = launch_das_lds_adjoint(at_frame(ac, f0), cc, p.mode, p.interp, grad_c + f0, s,
                                         std::min(k, nf - f0));
    }
    return err == hipSuccess ? BF_OK : hip_fail(err, "DAS adjoint launch");
}

// ---------------------------------------------------------------------------
// Scratch of bf_das_noalloc: the partial images of a channel-split DAS launch
// live in this file-scope device array instead of plan memory.  Each device
// holds its own copy (at its own address) for the life of the process.  Host
// code never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol): the device address is looked up once per device
// with hipGetSymbolAddress and kept in g_scratch.
// ---------------------------------------------------------------------------
constexpr int SCRATCH_MAX_DEVICES = 64;
static __device__ __align__(256) float scratch[BF_DAS_NOALLOC_MAX_BYTES / sizeof(float)];
static std::mutex g_scratch_mu;
static float *g_scratch[SCRATCH_MAX_DEVICES];

// Device address of this device's scratch array (dev must be current).
static int scratch_ptr(int dev, float **out)
{
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES)
        return fail(BF_ERR_UNSUPPORTED, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch[dev] = static_cast<float *>(p);
    }
    *out = g_scratch[dev];
    return BF_OK;
}

}  // namespace bf

using namespace bf;

static int check_plan(bf_plan plan)
{
    if (!plan) return fail(BF_ERR_NULL, "plan is NULL");
    if (plan->magic != BF_PLAN_MAGIC) return fail(BF_ERR_STATE, "not a live plan");
    return BF_OK;
}

static int check_frames(int32_t n_frames)
{
    if (n_frames < 1 || n_frames > BF_MAX_FRAMES)
        return fail(BF_ERR_SHAPE, "n_frames must be 1..%d", BF_MAX_FRAMES);
    return BF_OK;
}

static int check_c(double c)
{
    if (!is_fin(c) || c <= 0.0) return fail(BF_ERR_GEOMETRY, "sound speed must be finite and > 0");
    return BF_OK;
}

extern "C" {

int32_t bf_abi_version(void) { return BF_ABI_VERSION; }

const char *bf_last_error(void) { return g_err.c_str(); }

int bf_validate(const bf_params *params)
{
    g_err.clear();
    return validate_params(params);
}

int bf_plan_create_batch(const bf_params *params, int32_t n_frames, bf_plan *out)
{
    g_err.clear();
    if (!out) return fail(BF_ERR_NULL, "out is NULL");
    *out = nullptr;
    if (!params) return fail(BF_ERR_NULL, "params is NULL");
    if (n_frames < 1 || n_frames > 4096) return fail(BF_ERR_SHAPE, "n_frames=%d not in [1,4096]", n_frames);
    for (int f = 0; f < n_frames; ++f) {
        int st = validate_params(&params[f]);
        if (st != BF_OK) {
            if (n_frames > 1) {
                std::string m = g_err;
                return fail(st, "frame %d: %s", f, m.c_str());
            }
            return st;
        }
    }
    int dev = 0;
    int st = check_device(&dev);
    if (st != BF_OK) return st;
    bf_plan plan = new bf_plan_s();
    plan->device = dev;
    plan->frames.resize(n_frames);
    for (int f = 0; f < n_frames; ++f) {
        plan->frames[f] = new Frame();
        st = plan->frames[f]->init(params[f]);
        if (st != BF_OK) {
            delete plan;
            return st;
        }
    }
    *out = plan;
    return BF_OK;
}

int bf_plan_create(const bf_params *params, bf_plan *out)
{
    return bf_plan_create_batch(params, 1, out);
}

int bf_plan_destroy(bf_plan plan)
{
    g_err.clear();
    if (!plan) return BF_OK;
    if (plan->magic != BF_PLAN_MAGIC) return fail(BF_ERR_STATE, "not a live plan");
    (void)hipDeviceSynchronize();
    delete plan;
    return BF_OK;
}

int bf_plan_get_info(bf_plan plan, bf_plan_info *info)
{
    g_err.clear();
    int st = check_plan(plan);
    if (st != BF_OK) return st;
    if (!info) return fail(BF_ERR_NULL, "info is NULL");
    const Frame &f = *plan->frames[0];
    info->n_frames = (int32_t)plan->frames.size();
    info->tile[0] = 1 << f.lx;
    info->tile[1] = 1 << f.ly;
    info->tile[2] = 1 << f.lz;
    {
        // the kernel bf_das actually runs (LDS windows may not fit: gather)
        LdsCfg cfg;
        const bool lds = f.variant != BF_DAS_GATHER &&
                         f.lds_config(f.das_args(nullptr, nullptr, f.p.c), &cfg);
        info->variant = lds ? (cfg.zp == 2 ? BF_DAS_LDS_Z2 : BF_DAS_LDS) : BF_DAS_GATHER;
        info->nb = lds ? cfg.nb : f.nb;
    }
    info->block[0] = f.bw[0];
    info->block[1] = f.bw[1];
    info->block[2] = f.bw[2];
    info->workspace_bytes = plan->workspace_bytes();
    info->e_elems = f.e_elems();
    info->out_elems = f.out_elems();
    info->channel_groups = f.groups;
    return BF_OK;
}

int bf_set_tile(bf_plan plan, int32_t log2_x, int32_t log2_y, int32_t log2_z)
{
    g_err.clear();
    int st = check_plan(plan);
    if (st != BF_OK) return st;
    if (log2_x < 0 || log2_y < 0 || log2_z < 0 || log2_x + log2_y + log2_z != 6)
        return fail(BF_ERR_SHAPE, "tile log2 sizes must be >= 0 and sum to 6");
    for (Frame *f : plan->frames) {
        if (f->p.mode == BF_FORCES_2D && f->grid.ny == 1 && log2_y != 0)
            return fail(BF_ERR_SHAPE, "a 2D plan needs log2_y = 0");
    }
    for (Frame *f : plan->frames) f->set_tile(log2_x, log2_y, log2_z);
    return BF_OK;
}

int bf_set_das_config(bf_plan plan, int32_t variant, int32_t bw_x, int32_t bw_y, int32_t bw_z,
                      int32_t nb)
{
    g_err.clear();
    int st = check_plan(plan);
    if (st != BF_OK) return st;
    if (plan->batch) return fail(BF_ERR_STATE, "DAS configuration before the first batched launch");
    if (variant != BF_DAS_LDS && variant != BF_DAS_GATHER && variant != BF_DAS_LDS_Z2)
        return fail(BF_ERR_UNSUPPORTED, "unknown DAS variant %d", variant);
    if (bw_x < 1 || bw_y < 1 || bw_z < 1 || bw_x * bw_y * bw_z > 16)
        return fail(BF_ERR_SHAPE, "workgroup must hold 1..16 wavefront tiles");
    if (nb < 4 || nb > 64 || nb % 4 != 0) return fail(BF_ERR_SHAPE, "nb must be 4..64, a multiple of 4");
    for (Frame *f : plan->frames) {
        if (f->p.mode == BF_FORCES_2D && f->grid.ny == 1 && bw_y != 1)
            return fail(BF_ERR_SHAPE, "a 2D plan needs bw_y = 1");
        if (variant == BF_DAS_LDS_Z2 &&
            ((f->p.mode != BF_HERCULES_3D && f->p.mode != BF_FORCES_2D) || f->p.iq))
            return fail(BF_ERR_UNSUPPORTED,
                        "two depth points per lane: HERCULES and FORCES plans with real data only");
    }
    for (Frame *f : plan->frames) {
        f->variant = variant;
        f->bw[0] = bw_x;
        f->bw[1] = bw_y;
        f->bw[2] = bw_z;
        f->nb = nb;
    }
    return BF_OK;
}

int bf_decode(bf_plan plan, const int16_t *rf, void *e, void *stream)
{
    g_err.clear();
    int st = check_plan(plan);
    if (st != BF_OK) return st;
    if (!rf || !e) return fail(BF_ERR_NULL, "rf and e must be non-NULL");
    return plan->frames[0]->decode(rf, e, (hipStream_t)stream);
}

int bf_das(bf_plan plan, const void *e, float *out, double c, void *stream)
{
    g_err.clear();
    int st = check_plan(plan);
    if (st != BF_OK) return st;
    if (!e || !out) return fail(BF_ERR_NULL, "e and out must be non-NULL");
    if ((st = check_c(c)) != BF_OK) return st;
    return plan->frames[0]->das(e, out, c, (hipStream_t)stream);
}

int bf_das_fused(bf_plan plan, const int16_t *rf, float *out, double c, void *stream)
{
    g_err.clear();
    int st = check_plan(plan);
    if (st != BF_OK) return st;
    if (!rf || !out) return fail(BF_ERR_NULL, "rf and out must be non-NULL");
    if ((st = check_c(c)) != BF_OK) return st;
    return plan->frames[0]->das_fused(rf, out, c, (hipStream_t)stream);
}

int bf_das_noalloc(bf_plan plan, const void *e, float *out, double c, void *stream)
{
    g_err.clear();
    int st = check_plan(plan);
    if (st != BF_OK) return st;
    if (!e || !out) return fail(BF_ERR_NULL, "e and out must be non-NULL");
    if ((st = check_c(c)) != BF_OK) return st;
    int dev = 0;
    hipError_t he = hipGetDevice(&dev);
    if (he != hipSuccess) return hip_fail(he, "hipGetDevice");
    if (dev != plan->device)
        return fail(BF_ERR_STATE, "current device %d is not the plan's device %d", dev,
                    plan->device);
    const Frame &f = *plan->frames[0];
    float *part = nullptr;
    if (f.groups > 1) {
        const uint64_t need = (uint64_t)f.groups * (uint64_t)f.out_elems() * sizeof(float);
        if (need > BF_DAS_NOALLOC_MAX_BYTES)
            return fail(BF_ERR_TOO_LARGE, "partial images need %llu bytes, the scratch holds %u",
                        (unsigned long long)need, (unsigned)BF_DAS_NOALLOC_MAX_BYTES);
        if ((st = scratch_ptr(dev, &part)) != BF_OK) return st;
    }
    return f.das(e, out, c, (hipStream_t)stream, part);
}

int bf_das_adjoint(bf_plan plan, const void *e, const float *grad_out, double c, float *grad_e,
                   float *grad_c, void *stream)
{
    return bf_das_adjoint_frames(plan, e, grad_out, 1, c, grad_e, grad_c, stream);
}

int bf_das_frames(bf_plan plan, const void *e, int32_t n_frames, float *out, double c,
                  void *stream)
{
    g_err.clear();
    int st = check_plan(plan);
    if (st != BF_OK) return st;
    if (!e || !out) return fail(BF_ERR_NULL, "e and out must be non-NULL");
    if ((st = check_frames(n_frames)) != BF_OK) return st;
    if ((st = check_c(c)) != BF_OK) return st;
    return plan->frames[0]->das_frames(e, n_frames, out, c, (hipStream_t)stream);
}

int bf_das_adjoint_frames(bf_plan plan, const void *e, const float *grad_out, int32_t n_frames,
                          double c, float *grad_e, float *grad_c, void *stream)
{
    g_err.clear();
    int st = check_plan(plan);
    if (st != BF_OK) return st;
    if (!grad_out) return fail(BF_ERR_NULL, "grad_out is NULL");
    if (grad_c && !e) return fail(BF_ERR_NULL, "e is needed for grad_c");
    if ((st = check_frames(n_frames)) != BF_OK) return st;
    if ((st = check_c(c)) != BF_OK) return st;
    const Frame &f = *plan->frames[0];
    if (f.p.iq) return fail(BF_ERR_UNSUPPORTED, "the adjoint is defined for RF plans only");
    return f.das_adjoint(e, grad_out, c, grad_e, grad_c, n_frames, (hipStream_t)stream);
}

int bf_sharpness(const float *img, int64_t n_per_image, int32_t n_images, float *loss, float *grad,
                 void *stream)
{
    g_err.clear();
    if (!img || !loss) return fail(BF_ERR_NULL, "img and loss must be non-NULL");
    if (n_per_image < 1 || n_images < 1) return fail(BF_ERR_SHAPE, "empty image batch");
    if (n_per_image * (int64_t)n_images >= (int64_t(1) << 31))
        return fail(BF_ERR_TOO_LARGE, "image batch exceeds 2^31 elements");
    int dev = 0;
    int st = check_device(&dev);
    if (st != BF_OK) return st;
    hipError_t err = launch_sharpness(img, (long)n_per_image, n_images, loss, grad,
                                      (hipStream_t)stream);
    return err == hipSuccess ? BF_OK : hip_fail(err, "sharpness launch");
}

double bf_test_hann_poly(double u2) { return (double)hann_u2((float)u2); }

int bf_test_set_stack_cap(bf_plan plan, int32_t cap)
{
    g_err.clear();
    int st = check_plan(plan);
    if (st != BF_OK) return st;
    if (cap < 0) return fail(BF_ERR_SHAPE, "stack cap must be >= 0");
    for (Frame *f : plan->frames) f->stack_cap = cap;
    return BF_OK;
}

}  // extern "C"
