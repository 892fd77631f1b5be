// bf_das_adj.hip -- the adjoint of LDS-staged delay-and-sum: das_block in its
// adjoint form (bf_das_lds_block.h).  dL/dc: one FP64 partial per workgroup,
// then a fixed-order sum.  dL/de: per-trace LDS accumulation windows added
// to grad_e after each batch.
#include "bf_das_lds_block.h"

namespace bf {

hipError_t launch_reduce_partials(const double *partial, int n, float *out, hipStream_t s,
                                  int n_frames = 1);
hipError_t launch_fill(float *p, long n, float v, hipStream_t s);

// Frame fr of a stack of frames of one plan (grid z): the per-frame arrays
// advance by one frame's extent.  e, grad_e: [frames][n_tx][n_ch][S];
// grad_out: [frames][points]; partial: [frames][n_wg] (n_wg workgroups per
// frame).  Null arrays stay null.
__device__ inline void frame_args(DasArgs &a, int fr, long n_wg)
{
    const long traces = (long)fr * a.n_tx * a.n_ch;
    if (a.e) a.e = static_cast<const float *>(a.e) + traces * a.S;
    if (a.grad_out) a.grad_out += (long)fr * a.g.nx * a.g.ny * a.g.nz;
    if (a.grad_e) a.grad_e += traces * a.S;
    if (a.partial) a.partial += fr * n_wg;
}

// ADJ = 1: dL/dc (FP32 data), 2: dL/de (reads no data).  STACK: grid z runs
// a stack of frames (the single-frame kernels keep their registers: the
// frame offsets cost four VGPRs).
template <int MODE, int IP, int ZP, int ADJ, bool STACK>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(WavesPerEu<MODE, ZP>::value)))
void das_lds_adj_kernel(DasArgs a, LdsCfg c)
{
    extern __shared__ float4 smem[];
    if constexpr (STACK) frame_args(a, blockIdx.z, (long)gridDim.x * gridDim.y);
    const int blk = xcd_slab_box(c, blockIdx.x);
    if (blk < 0) {      // past the last slab: an empty partial for dL/dc
        if ((ADJ & 1) && threadIdx.x == 0) a.partial[(long)blockIdx.y * gridDim.x + blockIdx.x] = 0.0;
        return;
    }
    das_block<MODE, ET_F32, IP, ZP, ADJ>(a, c, blk, blockIdx.y, smem);
}

template <int MODE, int IP, int ZP, int ADJ, bool STACK>
static hipError_t launch_adj_lds5(const DasArgs &a, const LdsCfg &c, int nf, size_t shm,
                                  hipStream_t s)
{
    const int nthr = 64 * c.bwx * c.bwy * c.bwz;
    dim3 grid(xcd_slab_grid(c), a.groups, nf);
    if (c.lmax & 1) return hipErrorInvalidValue;        // real data: pairs of quads
    const void *fn = reinterpret_cast<const void *>(&das_lds_adj_kernel<MODE, IP, ZP, ADJ, STACK>);
    hipError_t e = allow_lds(fn, shm);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((das_lds_adj_kernel<MODE, IP, ZP, ADJ, STACK>), grid, dim3(nthr), shm, s, a,
                       c);
    return hipGetLastError();
}

template <int MODE, int IP, int ZP, int ADJ>
static hipError_t launch_adj_lds4(const DasArgs &a, const LdsCfg &c, int nf, size_t shm,
                                  hipStream_t s)
{
    return nf > 1 ? launch_adj_lds5<MODE, IP, ZP, ADJ, true>(a, c, nf, shm, s)
                  : launch_adj_lds5<MODE, IP, ZP, ADJ, false>(a, c, 1, shm, s);
}

template <int MODE, int IP, int ZP>
static hipError_t launch_adj_lds3(const DasArgs &a, const LdsCfg &c, int adj, int nf, size_t shm,
                                  hipStream_t s)
{
    switch (adj) {
        case 1: return launch_adj_lds4<MODE, IP, ZP, 1>(a, c, nf, shm, s);
        case 2: return launch_adj_lds4<MODE, IP, ZP, 2>(a, c, nf, shm, s);
        default: return hipErrorInvalidValue;     // one gradient per launch
    }
}

template <int MODE, int IP>
static hipError_t launch_adj_lds2(const DasArgs &a, const LdsCfg &c, int adj, int nf, size_t shm,
                                  hipStream_t s)
{
    if constexpr (MODE == MODE_HERCULES || MODE == MODE_FORCES)
        if (c.zp == 2) return launch_adj_lds3<MODE, IP, 2>(a, c, adj, nf, shm, s);
    return c.zp == 1 ? launch_adj_lds3<MODE, IP, 1>(a, c, adj, nf, shm, s) : hipErrorInvalidValue;
}

template <int MODE>
static hipError_t launch_adj_lds1(const DasArgs &a, const LdsCfg &c, int ip, int adj, int nf,
                                  size_t shm, hipStream_t s)
{
    switch (ip) {
        case IN_LINEAR: return launch_adj_lds2<MODE, IN_LINEAR>(a, c, adj, nf, shm, s);
        case IN_CUBIC: return launch_adj_lds2<MODE, IN_CUBIC>(a, c, adj, nf, shm, s);
        default: return hipErrorInvalidValue;
    }
}

// The adjoint with the LDS-staged kernel (linear or cubic reads), one of the
// two gradients per call: grad_e (a.grad_e) is cleared and accumulated, or
// grad_c receives the fixed-order sum of the workgroups' partials (FP32
// data).  n_frames > 1: a stack of frames in one launch (grid z), with
// grad_c[n_frames] and [n_frames][...] arrays (frame_args).
hipError_t launch_das_lds_adjoint(const DasArgs &a, const LdsCfg &c, int mode, int ip,
                                  float *grad_c, hipStream_t s, int n_frames)
{
    const int adj = (grad_c ? 1 : 0) | (a.grad_e ? 2 : 0);
    if (adj == 0) return hipSuccess;
    if (adj == 3) return hipErrorInvalidValue;
    const size_t shm = lds_bytes(a.n_tx, a.n_ch, c.nb, c.lmax, 1, c.guard, adj, mode);
    hipError_t err;
    if (a.grad_e) {
        err = launch_fill(a.grad_e, (long)n_frames * a.n_tx * a.n_ch * a.S, 0.f, s);
        if (err != hipSuccess) return err;
    }
    switch (mode) {
        case MODE_FORCES: err = launch_adj_lds1<MODE_FORCES>(a, c, ip, adj, n_frames, shm, s); break;
        case MODE_HERCULES: err = launch_adj_lds1<MODE_HERCULES>(a, c, ip, adj, n_frames, shm, s); break;
        case MODE_TPW: err = launch_adj_lds1<MODE_TPW>(a, c, ip, adj, n_frames, shm, s); break;
        case MODE_VLS: err = launch_adj_lds1<MODE_VLS>(a, c, ip, adj, n_frames, shm, s); break;
        default: return hipErrorInvalidValue;
    }
    if (err != hipSuccess || !grad_c) return err;
    return launch_reduce_partials(a.partial, xcd_slab_grid(c) * a.groups, grad_c, s, n_frames);
}

}  // namespace bf
