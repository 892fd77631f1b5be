// bf_das_lds.hip -- forward delay-and-sum kernels with LDS-staged trace
// windows (gfx950): the single-frame kernel, the persistent batched kernel
// and their launchers.  The workgroup body is das_block in bf_das_lds_block.h.
#include "bf_das_lds_block.h"

namespace bf {

hipError_t launch_sum_groups(const DasArgs &a, hipStream_t s);

template <int MODE, int ET, int IP, int ZP>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(WavesPerEu<MODE, ZP>::value)))
void das_lds_kernel(DasArgs a, LdsCfg c)
{
    extern __shared__ float4 smem[];
    const int blk = xcd_slab_box(c, blockIdx.x);
    if (blk < 0) return;
    das_block<MODE, ET, IP, ZP>(a, c, blk, blockIdx.y, smem);
}

// Persistent form for a batch of frames: each workgroup pulls (frame, box,
// channel group) items from queues until they are empty (a frame with
// channel groups writes one partial image per group, summed afterwards in a
// fixed order).  There is one queue per XCD; the
// host deals whole depth slabs of a frame to the queues (costliest first), so
// the workgroups on one XCD (index b runs on XCD b % 8: the grid is resident
// at once and dispatched round-robin) work on neighbouring boxes that share
// trace windows in that XCD's L2.  A workgroup drains its home queue, then
// takes what is left in the others, so uneven queues still balance.  Every
// workgroup leaves after one failed pull per queue.
template <int MODE, int ET, int IP, int ZP>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(WavesPerEu<MODE, ZP>::value)))
void das_persistent_kernel(const FrameDas *__restrict__ frames,
                                                              const int4 *__restrict__ items,
                                                              QueueSet queues, int *counters,
                                                              void *const *__restrict__ out_ptrs)
{
    extern __shared__ float4 smem[];
    __shared__ int s_item;
    const int home = blockIdx.x % N_XCD_QUEUES;
    for (int r = 0; r < N_XCD_QUEUES; ++r) {
        const int q = (home + r) % N_XCD_QUEUES;
        const int beg = queues.off[q], n = queues.off[q + 1] - beg;
        for (;;) {
            if (threadIdx.x == 0) s_item = atomicAdd(counters + q, 1);
            __syncthreads();
            // the item is workgroup-uniform: keep it (and all it indexes) scalar
            const int item = __builtin_amdgcn_readfirstlane(s_item);
            __syncthreads();
            if (item >= n) break;
            const int fr = __builtin_amdgcn_readfirstlane(items[beg + item].x);
            const int blk = __builtin_amdgcn_readfirstlane(items[beg + item].y);
            const int grp = __builtin_amdgcn_readfirstlane(items[beg + item].z);
            DasArgs a = frames[fr].a;
            a.out = static_cast<float *>(out_ptrs[fr]);
            das_block<MODE, ET, IP, ZP>(a, frames[fr].c, blk, grp, smem);
            __syncthreads();
        }
    }
}


template <int MODE, int ET, int IP, int ZP>
static hipError_t launch_persistent4(const PersistentLaunch &p, hipStream_t s)
{
    const void *fn = reinterpret_cast<const void *>(&das_persistent_kernel<MODE, ET, IP, ZP>);
    hipError_t e = allow_lds(fn, p.shm);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((das_persistent_kernel<MODE, ET, IP, ZP>), dim3(p.grid), dim3(p.threads),
                       p.shm, s, p.frames, p.items, p.queues, p.counters, p.out_ptrs);
    return hipGetLastError();
}

template <int MODE, int ET, int IP>
static hipError_t launch_persistent3(const PersistentLaunch &p, hipStream_t s)
{
    if constexpr (MODE == MODE_HERCULES || MODE == MODE_FORCES)
        if (p.zp == 2) return launch_persistent4<MODE, ET, IP, 2>(p, s);
    return p.zp == 1 ? launch_persistent4<MODE, ET, IP, 1>(p, s) : hipErrorInvalidValue;
}

template <int MODE, int ET>
static hipError_t launch_persistent2(const PersistentLaunch &p, hipStream_t s)
{
    switch (p.ip) {
        case IN_NEAREST: return launch_persistent3<MODE, ET, IN_NEAREST>(p, s);
        case IN_LINEAR: return launch_persistent3<MODE, ET, IN_LINEAR>(p, s);
        case IN_CUBIC: return launch_persistent3<MODE, ET, IN_CUBIC>(p, s);
        default: return hipErrorInvalidValue;
    }
}

template <int MODE>
static hipError_t launch_persistent1(const PersistentLaunch &p, hipStream_t s)
{
    switch (p.et) {
        case ET_F32: return launch_persistent2<MODE, ET_F32>(p, s);
        case ET_BF16: return launch_persistent2<MODE, ET_BF16>(p, s);
        case ET_I32: return launch_persistent2<MODE, ET_I32>(p, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_das_persistent(const PersistentLaunch &p, hipStream_t s)
{
    switch (p.mode) {
        case MODE_FORCES: return launch_persistent1<MODE_FORCES>(p, s);
        case MODE_HERCULES: return launch_persistent1<MODE_HERCULES>(p, s);
        case MODE_TPW: return launch_persistent1<MODE_TPW>(p, s);
        case MODE_VLS: return launch_persistent1<MODE_VLS>(p, s);
        default: return hipErrorInvalidValue;
    }
}

// Workgroups of the persistent DAS kernel that fit on the device at once.
int persistent_das_blocks(int mode, int et, int ip, int zp, int threads, size_t shm)
{
    int dev = 0, cus = 0, per = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const void *fn = nullptr;
    if (mode == 0 && et == ET_F32 && ip == IN_CUBIC)
        fn = zp == 2 ? reinterpret_cast<const void *>(&das_persistent_kernel<0, ET_F32, IN_CUBIC, 2>)
                     : reinterpret_cast<const void *>(&das_persistent_kernel<0, ET_F32, IN_CUBIC, 1>);
    else if (mode == 1 && et == ET_F32 && ip == IN_CUBIC)
        fn = zp == 2 ? reinterpret_cast<const void *>(&das_persistent_kernel<1, ET_F32, IN_CUBIC, 2>)
                     : reinterpret_cast<const void *>(&das_persistent_kernel<1, ET_F32, IN_CUBIC, 1>);
    if (fn && allow_lds(fn, shm) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, threads, shm) == hipSuccess && per > 0)
        return cus * per;
    return cus * 2;
}

template <int MODE, int ET, int IP, int ZP>
static hipError_t launch_lds4(const DasArgs &a, const LdsCfg &c, size_t shm, hipStream_t s)
{
    const int nthr = 64 * c.bwx * c.bwy * c.bwz;
    dim3 grid(xcd_slab_grid(c), a.groups);
    if (stage_pairs(ET == ET_CF32) && (c.lmax & 1)) return hipErrorInvalidValue;   // pairs of quads
    hipError_t e = allow_lds(reinterpret_cast<const void *>(&das_lds_kernel<MODE, ET, IP, ZP>), shm);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((das_lds_kernel<MODE, ET, IP, ZP>), grid, dim3(nthr), shm, s, a, c);
    return hipGetLastError();
}

template <int MODE, int ET, int IP>
static hipError_t launch_lds_zp(const DasArgs &a, const LdsCfg &c, size_t shm, hipStream_t s)
{
    if constexpr ((MODE == MODE_HERCULES || MODE == MODE_FORCES) && ET != ET_CF32)
        if (c.zp == 2) return launch_lds4<MODE, ET, IP, 2>(a, c, shm, s);
    return c.zp == 1 ? launch_lds4<MODE, ET, IP, 1>(a, c, shm, s) : hipErrorInvalidValue;
}

template <int MODE, int ET>
static hipError_t launch_lds_ip(const DasArgs &a, const LdsCfg &c, int ip, size_t shm,
                                hipStream_t s)
{
    switch (ip) {
        case IN_NEAREST: return launch_lds_zp<MODE, ET, IN_NEAREST>(a, c, shm, s);
        case IN_LINEAR: return launch_lds_zp<MODE, ET, IN_LINEAR>(a, c, shm, s);
        case IN_CUBIC: return launch_lds_zp<MODE, ET, IN_CUBIC>(a, c, shm, s);
        default: return hipErrorInvalidValue;
    }
}

template <int MODE>
static hipError_t launch_lds_et(const DasArgs &a, const LdsCfg &c, int et, int ip, size_t shm,
                                hipStream_t s)
{
    switch (et) {
        case ET_F32: return launch_lds_ip<MODE, ET_F32>(a, c, ip, shm, s);
        case ET_BF16: return launch_lds_ip<MODE, ET_BF16>(a, c, ip, shm, s);
        case ET_I32: return launch_lds_ip<MODE, ET_I32>(a, c, ip, shm, s);
        case ET_CF32: return launch_lds_ip<MODE, ET_CF32>(a, c, ip, shm, s);
        default: return hipErrorInvalidValue;
    }
}

// Decode fused into DAS: FORCES planes from int16 RF (a.e) and the FP32 H
// table (a.hf); the same LDS kernel with the decode in its staging.
hipError_t launch_das_lds_fused(const DasArgs &a, const LdsCfg &c, int ip, hipStream_t s);

size_t lds_bytes(int n_tx, int n_ch, int nb, int lmax, int qs, int guard, int adj, int mode)
{
    const bool stage = adj == 0 || (adj & 1);     // data windows staged
    // tx_x and rx_c (and the separable modes' path bounds: one more of each)
    const int tables = (mode == MODE_HERCULES ? 1 : 2) * (((n_tx + 3) & ~3) + ((n_ch + 3) & ~3));
    return (size_t)(tables + 2 * ((nb + 3) & ~3)) * 4 +
           (mode == MODE_HERCULES ? (size_t)HANN_TAB_PAD * 8 : 0) +
           (stage ? (2 * (size_t)nb * lmax + guard) * qs * 16 : 0) +
           ((adj & 2) ? 2 * (size_t)nb * (lmax + 3) * 8 + 16 * 4 : 0);
}

hipError_t launch_das_lds_fused(const DasArgs &a, const LdsCfg &c, int ip, hipStream_t s)
{
    const size_t shm = lds_bytes(a.n_tx, a.n_ch, c.nb, c.lmax, 1, c.guard, 0, MODE_FORCES);
    const hipError_t err = launch_lds_ip<MODE_FORCES, ET_RF16>(a, c, ip, shm, s);
    if (err != hipSuccess || a.groups <= 1) return err;
    return launch_sum_groups(a, s);
}

hipError_t launch_das_lds(const DasArgs &a, const LdsCfg &c, int mode, int et, int ip,
                          hipStream_t s)
{
    const size_t shm = lds_bytes(a.n_tx, a.n_ch, c.nb, c.lmax, a.cx ? 2 : 1, c.guard, 0, mode);
    hipError_t err;
    switch (mode) {
        case MODE_FORCES: err = launch_lds_et<MODE_FORCES>(a, c, et, ip, shm, s); break;
        case MODE_HERCULES: err = launch_lds_et<MODE_HERCULES>(a, c, et, ip, shm, s); break;
        case MODE_TPW: err = launch_lds_et<MODE_TPW>(a, c, et, ip, shm, s); break;
        case MODE_VLS: err = launch_lds_et<MODE_VLS>(a, c, et, ip, shm, s); break;
        default: return hipErrorInvalidValue;
    }
    if (err != hipSuccess || a.groups <= 1) return err;
    return launch_sum_groups(a, s);
}

}  // namespace bf
