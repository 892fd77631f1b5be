// bf_batch.hip -- batched decode + DAS over many frames with persistent
// kernels, its hipGraph replay, and the DAS workgroup autotuner.
//
// A batch holds frames with their own descriptions (uFORCES / uHERCULES
// transmit subsets of different sizes, 2D and 3D outputs).  Frames are
// grouped into kernel classes: decode by (32-wide K blocks, output type) and
// DAS by (mode, data type, interpolation).  Each class runs as ONE persistent
// launch whose workgroups pull work items from atomic queues: decode items
// are (frame, channel, 256 samples); DAS items are (frame, workgroup box),
// grouped into depth slabs that are dealt to one queue per XCD in decreasing
// cost, so the tail is made of short items and the boxes that run together
// on an XCD share trace windows in its L2.  Decoded data stays in plan-owned workspaces; the caller's RF and
// output buffers are passed through a device pointer table refreshed before
// every launch, so a captured graph never needs re-capture for new buffers.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "bf_plan.h"

namespace bf {

hipError_t launch_decode_persistent(const DecLaunch &p, hipStream_t s);
hipError_t launch_das_persistent(const PersistentLaunch &p, hipStream_t s);
int persistent_das_blocks(int mode, int et, int ip, int zp, int threads, size_t shm);
hipError_t launch_fill(float *p, long n, float v, hipStream_t s);
hipError_t launch_sum_groups(const DasArgs &a, hipStream_t s);

__global__ void reset_counters_kernel(int *c, int n)
{
    for (int q = threadIdx.x; q < n; q += blockDim.x) c[q] = 0;
}

struct DecClass {
    int kb, ot;
    std::vector<int2> items;
    int2 *d_items = nullptr;
    int grid = 0;
};

struct DasItem {
    double cost;    // per-item cost of its frame
    int slab;       // box depth index (bz)
    int grp;        // channel group
    int4 item;      // (frame, box, channel group, -)
};

struct DasClass {
    int mode, et, ip, zp, threads;
    size_t shm = 0;
    std::vector<DasItem> items;
    int4 *d_items = nullptr;
    int n_items = 0;
    QueueSet queues{};
    int grid = 0;
};

constexpr int RING = 4;

struct Batch {
    int F = 0;
    FrameDec *d_fdec = nullptr;
    FrameDas *d_fdas = nullptr;
    std::vector<FrameDas> h_fdas;     // host copy of the DAS frame table
    void **d_ptrs = nullptr;          // [2F]: rf pointers, then out pointers
    int *d_counters = nullptr;
    std::vector<DecClass> dec;
    std::vector<DasClass> das;
    std::vector<int> gather_frames;   // frames on the gather kernel (windows too long for LDS)
    std::vector<int> split_frames;    // persistent frames with channel groups (partial images)
    std::vector<int> frame_lds;       // frames on their own LDS launch (BF_BATCH_FRAME_LDS)
    std::vector<bf_batch_frame_info> info;   // how each frame runs
    void **h_stage[RING] = {};
    hipEvent_t ev[RING] = {};
    int ring = 0;
    // the pointers of the last staged copy and its stream: a call with the
    // same buffers on the same stream finds them in the device table already
    // (that copy is ordered before it), so it stages nothing
    std::vector<void *> last_ptrs;
    hipStream_t last_stream = nullptr;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<void *> allocs;

    ~Batch()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
        for (int k = 0; k < RING; ++k) {
            if (ev[k]) (void)hipEventDestroy(ev[k]);
            if (h_stage[k]) (void)hipHostFree(h_stage[k]);
        }
        for (void *p : allocs) (void)hipFree(p);
    }
    void *alloc(size_t bytes)
    {
        void *p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
        allocs.push_back(p);
        return p;
    }
};

static int build_batch(bf_plan plan)
{
    Batch *b = new Batch();
    plan->batch = b;
    const int F = (int)plan->frames.size();
    b->F = F;
    std::vector<FrameDec> fdec(F);
    std::vector<FrameDas> fdas(F);
    int dev0 = 0, cus0 = 0;
    (void)hipGetDevice(&dev0);
    (void)hipDeviceGetAttribute(&cus0, hipDeviceAttributeMultiprocessorCount, dev0);
    // LDS frames of a kernel class run as one persistent launch over their
    // (box, channel group) items.  A class with few boxes (e.g. a pair of
    // small planes) splits the channel sum of its frames over G groups, so
    // that it still gives about four items per CU; each group writes a
    // partial image and a second kernel adds them in a fixed order.
    const long target_items = 4L * cus0;
    std::vector<int> lds_ok(F, 0), groups(F, 1);
    {
        std::vector<std::pair<long, long>> cls_boxes;   // (class key, boxes)
        std::vector<long> key(F, -1);
        for (int f = 0; f < F; ++f) {
            Frame &fr = *plan->frames[f];
            DasArgs a = fr.das_args(nullptr, nullptr, fr.p.c);
            LdsCfg c;
            if (fr.variant == BF_DAS_GATHER || !fr.lds_config(a, &c)) continue;
            lds_ok[f] = 1;
            key[f] = ((((long)fr.p.mode * 8 + fr.p.e_type) * 8 + fr.p.interp) * 4 + c.zp) * 2048 +
                     64 * c.bwx * c.bwy * c.bwz;
            const long nblk = (long)c.blocks_x * c.blocks_y * c.blocks_z;
            bool found = false;
            for (auto &kb : cls_boxes)
                if (kb.first == key[f]) { kb.second += nblk; found = true; }
            if (!found) cls_boxes.push_back({key[f], nblk});
        }
        for (int f = 0; f < F; ++f)
            for (auto &kb : cls_boxes)
                if (key[f] >= 0 && kb.first == key[f] && kb.second < target_items) {
                    const long G = (target_items + kb.second - 1) / kb.second;
                    const long gmax = std::max(1, plan->frames[f]->p.n_ch / 4);
                    groups[f] = (int)std::min<long>(std::min<long>(G, 16), gmax);
                }
    }
    for (int f = 0; f < F; ++f) {
        Frame &fr = *plan->frames[f];
        if (!fr.d_e) {
            fr.d_e = fr.alloc(fr.e_bytes());
            if (!fr.d_e) return fail(BF_ERR_HIP, "decoded-data workspace allocation failed");
        }
        fdec[f].a = fr.decode_args(nullptr, fr.d_e);
        DasArgs a = fr.das_args(fr.d_e, nullptr, fr.p.c);
        a.groups = 1;
        a.part = nullptr;
        LdsCfg c;
        bf_batch_frame_info fi;
        fi.das_path = BF_BATCH_GATHER;
        fi.das_class = -1;
        fi.channel_groups = 1;
        fi.decode_class = -1;
        fi.das_items = 0;
        if (!lds_ok[f] || !fr.lds_config(a, &c)) {
            b->gather_frames.push_back(f);
            memset(&c, 0, sizeof c);
        } else if (groups[f] > 1 &&
                   (long)c.blocks_x * c.blocks_y * c.blocks_z * fr.groups >= 2L * cus0) {
            // A frame of a class that would need the channel split, whose own
            // launch (the single-frame kernel with the frame's channel groups)
            // already gives two workgroups per CU: that launch, captured in
            // the pass like the others, measured faster than its share of the
            // persistent launch (a pair of 256 x 256 planes from 128 x 128
            // traces: 1.35 ms per pass persistent).
            b->frame_lds.push_back(f);
            fi.das_path = BF_BATCH_FRAME_LDS;
            fi.channel_groups = fr.groups;
            fi.das_items = (int64_t)c.blocks_x * c.blocks_y * c.blocks_z * fr.groups;
            memset(&c, 0, sizeof c);
        } else {
            const int G = groups[f];
            if (G > 1) {
                a.groups = G;
                a.part = (float *)b->alloc((size_t)G * fr.out_elems() * sizeof(float));
                if (!a.part) return fail(BF_ERR_HIP, "partial-image allocation failed");
                b->split_frames.push_back(f);
            }
            const int threads = 64 * c.bwx * c.bwy * c.bwz;
            const size_t shm = lds_bytes(a.n_tx, a.n_ch, c.nb, c.lmax, 1, c.guard, 0, fr.p.mode);
            DasClass *cls = nullptr;
            for (DasClass &d : b->das)
                if (d.mode == fr.p.mode && d.et == fr.p.e_type && d.ip == fr.p.interp &&
                    d.zp == c.zp && d.threads == threads)
                    cls = &d;
            if (!cls) {
                DasClass d;
                d.mode = fr.p.mode;
                d.et = fr.p.e_type;
                d.ip = fr.p.interp;
                d.zp = c.zp;
                d.threads = threads;
                b->das.push_back(d);
                cls = &b->das.back();
            }
            cls->shm = std::max(cls->shm, shm);
            const int nblk = c.blocks_x * c.blocks_y * c.blocks_z;
            // an item's cost: its traces times its points
            const double cost = (double)fr.p.n_tx * fr.p.n_ch / G * threads;
            for (int g = 0; g < G; ++g)
                for (int q = 0; q < nblk; ++q)
                    cls->items.push_back({cost, q % c.blocks_z, g, make_int4(f, q, g, 0)});
            fi.das_path = BF_BATCH_PERSISTENT_LDS;
            fi.das_class = (int)(cls - b->das.data());
            fi.channel_groups = G;
            fi.das_items = (int64_t)nblk * G;
        }
        if (c.lmax & 1) return fail(BF_ERR_STATE, "frame %d: odd LDS window length", f);
        fdas[f].a = a;
        fdas[f].c = c;
        // decode classes
        if (fr.p.decode_algo == BF_DECODE_MFMA_I8) {
            DecClass *cls = nullptr;
            for (DecClass &d : b->dec)
                if (d.kb == fr.kb && d.ot == fr.p.e_type) cls = &d;
            if (!cls) {
                DecClass d;
                d.kb = fr.kb;
                d.ot = fr.p.e_type;
                b->dec.push_back(d);
                cls = &b->dec.back();
            }
            const int n_chunks = (fr.p.n_samples + 63) / 64;
            const int n_cg = (n_chunks + 3) / 4;
            for (int j = 0; j < fr.p.n_ch; ++j)
                for (int g = 0; g < n_cg; ++g) cls->items.push_back(make_int2(f, j * n_cg + g));
            fi.decode_class = (int)(cls - b->dec.data());
        }
        if (fi.das_path == BF_BATCH_GATHER) fi.das_items = 1;   // one launch of the gather kernel
        b->info.push_back(fi);
    }
    const int n_counters = (int)(b->dec.size() + b->das.size() * N_XCD_QUEUES);
    b->d_fdec = (FrameDec *)b->alloc(sizeof(FrameDec) * F);
    b->d_fdas = (FrameDas *)b->alloc(sizeof(FrameDas) * F);
    b->d_ptrs = (void **)b->alloc(sizeof(void *) * 2 * F);
    b->d_counters = (int *)b->alloc(sizeof(int) * (n_counters > 0 ? n_counters : 1));
    if (!b->d_fdec || !b->d_fdas || !b->d_ptrs || !b->d_counters)
        return fail(BF_ERR_HIP, "batch table allocation failed");
    hipError_t e;
    if ((e = hipMemcpy(b->d_fdec, fdec.data(), sizeof(FrameDec) * F, hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (e = hipMemcpy(b->d_fdas, fdas.data(), sizeof(FrameDas) * F, hipMemcpyHostToDevice)) !=
            hipSuccess)
        return hip_fail(e, "batch table upload");
    b->h_fdas = fdas;
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    for (DecClass &d : b->dec) {
        d.d_items = (int2 *)b->alloc(sizeof(int2) * d.items.size());
        if (!d.d_items) return fail(BF_ERR_HIP, "batch item allocation failed");
        if ((e = hipMemcpy(d.d_items, d.items.data(), sizeof(int2) * d.items.size(),
                           hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "batch item upload");
        d.grid = std::min<int>((int)d.items.size(), cus * 8);
    }
    for (DasClass &d : b->das) {
        // Depth slabs (frame, channel group, bz) in decreasing cost (costlier
        // frames, then deeper slabs: wider apertures) dealt round-robin to the
        // per-XCD queues; a slab's boxes stay together in its queue (they
        // stage nearly the same trace windows).
        std::stable_sort(d.items.begin(), d.items.end(), [](const DasItem &x, const DasItem &y) {
            if (x.cost != y.cost) return x.cost > y.cost;
            if (x.item.x != y.item.x) return x.item.x < y.item.x;
            if (x.grp != y.grp) return x.grp < y.grp;
            return x.slab > y.slab;
        });
        std::vector<std::vector<int4>> per(N_XCD_QUEUES);
        int next = 0;
        for (size_t q = 0; q < d.items.size(); ++q) {
            if (q > 0 && (d.items[q].item.x != d.items[q - 1].item.x ||
                          d.items[q].grp != d.items[q - 1].grp ||
                          d.items[q].slab != d.items[q - 1].slab))
                next = (next + 1) % N_XCD_QUEUES;
            per[next].push_back(d.items[q].item);
        }
        std::vector<int4> it;
        for (int q = 0; q < N_XCD_QUEUES; ++q) {
            d.queues.off[q] = (int)it.size();
            it.insert(it.end(), per[q].begin(), per[q].end());
        }
        d.queues.off[N_XCD_QUEUES] = (int)it.size();
        d.n_items = (int)it.size();
        d.d_items = (int4 *)b->alloc(sizeof(int4) * it.size());
        if (!d.d_items) return fail(BF_ERR_HIP, "batch item allocation failed");
        if ((e = hipMemcpy(d.d_items, it.data(), sizeof(int4) * it.size(), hipMemcpyHostToDevice)) !=
            hipSuccess)
            return hip_fail(e, "batch item upload");
        d.grid = std::min(d.n_items, persistent_das_blocks(d.mode, d.et, d.ip, d.zp, d.threads, d.shm));
    }
    for (int k = 0; k < RING; ++k) {
        if ((e = hipHostMalloc((void **)&b->h_stage[k], sizeof(void *) * 2 * F)) != hipSuccess)
            return hip_fail(e, "pinned staging allocation");
        if ((e = hipEventCreateWithFlags(&b->ev[k], hipEventDisableTiming)) != hipSuccess)
            return hip_fail(e, "event creation");
    }
    return BF_OK;
}

// Copy the frame pointers to the device table (ordered on `s` before the
// kernels that read it).  A ring of pinned buffers keeps earlier, still
// pending copies intact.
static int stage_pointers(Batch *b, const int16_t *const *rf, float *const *out, hipStream_t s)
{
    bool same = !b->last_ptrs.empty() && b->last_stream == s;
    for (int f = 0; same && f < b->F; ++f)
        same = b->last_ptrs[f] == (const void *)rf[f] && b->last_ptrs[b->F + f] == (void *)out[f];
    if (same) return BF_OK;
    const int k = b->ring;
    b->ring = (b->ring + 1) % RING;
    hipError_t e = hipEventSynchronize(b->ev[k]);
    if (e != hipSuccess) return hip_fail(e, "pointer staging wait");
    for (int f = 0; f < b->F; ++f) {
        b->h_stage[k][f] = (void *)rf[f];
        b->h_stage[k][b->F + f] = (void *)out[f];
    }
    if ((e = hipMemcpyAsync(b->d_ptrs, b->h_stage[k], sizeof(void *) * 2 * b->F,
                            hipMemcpyHostToDevice, s)) != hipSuccess)
        return hip_fail(e, "pointer table copy");
    if ((e = hipEventRecord(b->ev[k], s)) != hipSuccess) return hip_fail(e, "event record");
    b->last_ptrs.assign(b->h_stage[k], b->h_stage[k] + 2 * b->F);
    b->last_stream = s;
    return BF_OK;
}

// All kernels of one batched pass, in stream order.
static int enqueue(bf_plan plan, hipStream_t s)
{
    Batch *b = plan->batch;
    const int n_counters = (int)(b->dec.size() + b->das.size() * N_XCD_QUEUES);
    hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(64), 0, s, b->d_counters,
                       n_counters);
    int ci = 0;
    for (DecClass &d : b->dec) {
        DecLaunch L;
        L.kb = d.kb;
        L.ot = d.ot;
        L.grid = d.grid;
        L.frames = b->d_fdec;
        L.items = d.d_items;
        L.n_items = (int)d.items.size();
        L.counter = b->d_counters + ci++;
        L.rf_ptrs = b->d_ptrs;
        hipError_t e = launch_decode_persistent(L, s);
        if (e != hipSuccess) return hip_fail(e, "persistent decode launch");
    }
    for (DasClass &d : b->das) {
        PersistentLaunch L;
        L.mode = d.mode;
        L.et = d.et;
        L.ip = d.ip;
        L.zp = d.zp;
        L.grid = d.grid;
        L.threads = d.threads;
        L.shm = d.shm;
        L.frames = b->d_fdas;
        L.items = d.d_items;
        L.queues = d.queues;
        L.counters = b->d_counters + ci;
        ci += N_XCD_QUEUES;
        L.out_ptrs = b->d_ptrs + b->F;
        hipError_t e = launch_das_persistent(L, s);
        if (e != hipSuccess) return hip_fail(e, "persistent DAS launch");
    }
    // frames split over channel groups: add their partial images in a fixed
    // order into the output (its pointer read from the device table)
    for (int f : b->split_frames) {
        DasArgs a = b->h_fdas[f].a;
        a.out = nullptr;
        a.out_ref = reinterpret_cast<float *const *>(b->d_ptrs + b->F + f);
        hipError_t e = launch_sum_groups(a, s);
        if (e != hipSuccess) return hip_fail(e, "partial-image sum launch");
    }
    return BF_OK;
}

static int check_batch(bf_plan plan, const int16_t *const *rf, float *const *out)
{
    if (!plan) return fail(BF_ERR_NULL, "plan is NULL");
    if (plan->magic != BF_PLAN_MAGIC) return fail(BF_ERR_STATE, "not a live plan");
    if (!rf || !out) return fail(BF_ERR_NULL, "rf and out pointer arrays must be non-NULL");
    for (size_t f = 0; f < plan->frames.size(); ++f)
        if (!rf[f] || !out[f]) return fail(BF_ERR_NULL, "frame %zu has a NULL buffer", f);
    for (Frame *fr : plan->frames) {
        if (fr->p.decode_algo != BF_DECODE_MFMA_I8)
            return fail(BF_ERR_UNSUPPORTED, "batched path runs the int8 decode only");
        if (fr->p.iq) return fail(BF_ERR_UNSUPPORTED, "batched path takes RF frames only");
    }
    if (!plan->batch) {
        int st = build_batch(plan);
        if (st != BF_OK) {
            delete plan->batch;
            plan->batch = nullptr;
            return st;
        }
    }
    return BF_OK;
}

// Frames on their own LDS launch, and frames whose windows do not fit in
// LDS (the direct-gather kernel), run after the persistent kernels; they read
// their output pointer from the device table too, so they are captured in
// the same graph.
static int enqueue_gather(bf_plan plan, hipStream_t s)
{
    Batch *b = plan->batch;
    for (int f : b->frame_lds) {
        const Frame &fr = *plan->frames[f];
        DasArgs a = fr.das_args(fr.d_e, nullptr, fr.p.c);
        a.out_ref = reinterpret_cast<float *const *>(b->d_ptrs + b->F + f);
        LdsCfg c;
        if (!fr.lds_config(a, &c)) return fail(BF_ERR_STATE, "frame %d lost its LDS configuration", f);
        hipError_t e = launch_das_lds(a, c, fr.p.mode, fr.p.e_type, fr.p.interp, s);
        if (e != hipSuccess) return hip_fail(e, "DAS launch");
    }
    for (int f : b->gather_frames) {
        const Frame &fr = *plan->frames[f];
        DasArgs a = fr.das_args(fr.d_e, nullptr, fr.p.c);
        a.out_ref = reinterpret_cast<float *const *>(b->d_ptrs + b->F + f);
        hipError_t e = launch_das(a, fr.p.mode, fr.p.e_type, fr.p.interp, s);
        if (e != hipSuccess) return hip_fail(e, "DAS launch");
    }
    return BF_OK;
}

}  // namespace bf

using namespace bf;

bf_plan_s::~bf_plan_s()
{
    magic = 0;
    delete batch;
    for (Frame *f : frames) delete f;
}

int64_t bf_plan_s::workspace_bytes() const
{
    int64_t b = 0;
    for (const Frame *f : frames) b += f->total_bytes;
    return b;
}

// ---------------------------------------------------------------------------
// Autotuner
// ---------------------------------------------------------------------------
namespace {

struct TileCand {
    int lx, ly, lz, bwx, bwy, bwz, nb, variant;
};

std::vector<TileCand> candidates(const Frame &f)
{
    std::vector<TileCand> c;
    if (f.p.mode == BF_FORCES_2D && (f.grid.ny == 1 || f.grid.nx == 1)) {
        // a plane along x (ny = 1) or along y (nx = 1): tiles and workgroups
        // spread over that lateral axis and depth only
        const bool along_x = f.grid.ny == 1;
        const int tiles[][2] = {{3, 3}, {2, 4}, {4, 2}, {1, 5}, {5, 1}};
        const int blocks[][2] = {{2, 2}, {4, 1}, {1, 4}, {2, 1}, {4, 4}, {2, 8}};
        // two depth points per lane (real data): half the wavefronts per box
        const bool z2 = !f.p.iq && f.grid.nz >= 2;
        const int blocks2[][2] = {{2, 4}, {2, 2}, {4, 2}, {2, 8}, {4, 4}};
        for (auto &t : tiles) {
            const int lx = along_x ? t[0] : 0, ly = along_x ? 0 : t[0];
            c.push_back({lx, ly, t[1], 1, 1, 1, 4, BF_DAS_GATHER});
            for (auto &b : blocks)
                for (int nb : {4, 8, 16})
                    c.push_back({lx, ly, t[1], along_x ? b[0] : 1, along_x ? 1 : b[0], b[1], nb,
                                 BF_DAS_LDS});
            if (z2)
                for (auto &b : blocks2)
                    for (int nb : {8, 16, 24})
                        c.push_back({lx, ly, t[1], along_x ? b[0] : 1, along_x ? 1 : b[0], b[1],
                                     nb, BF_DAS_LDS_Z2});
        }
    } else {
        const int tiles[][3] = {{3, 3, 0}, {2, 3, 1}, {2, 2, 2}};
        const int blocks[][3] = {{2, 2, 3}, {2, 2, 2}, {4, 2, 1}, {3, 2, 2}, {2, 3, 2}, {2, 2, 1}};
        // two depth points per lane (HERCULES, real data): boxes twice as deep
        const bool z2 = f.p.mode == BF_HERCULES_3D && !f.p.iq && f.grid.nz >= 2;
        const int blocks2[][3] = {{2, 2, 3}, {2, 2, 2}, {4, 2, 1}, {2, 2, 1}, {3, 2, 2}};
        for (auto &t : tiles) {
            c.push_back({t[0], t[1], t[2], 1, 1, 1, 4, BF_DAS_GATHER});
            for (auto &b : blocks)
                for (int nb : {8, 16, 24, 32, 40})
                    c.push_back({t[0], t[1], t[2], b[0], b[1], b[2], nb, BF_DAS_LDS});
            if (z2)
                for (auto &b : blocks2)
                    for (int nb : {16, 24, 32, 40})
                        c.push_back({t[0], t[1], t[2], b[0], b[1], b[2], nb, BF_DAS_LDS_Z2});
        }
    }
    return c;
}

std::string tune_key(const Frame &f, const char *arch)
{
    char buf[256];
    snprintf(buf, sizeof buf, "%s|m%d|tx%d|ch%d|S%d|%dx%dx%d|ip%d|et%d%s", arch, f.p.mode,
             f.p.n_tx, f.p.n_ch, f.p.n_samples, f.grid.nx, f.grid.ny, f.grid.nz, f.p.interp,
             f.p.e_type, f.p.iq ? "|iq" : "");
    return buf;
}

bool cache_lookup(const char *path, const std::string &key, TileCand *out)
{
    FILE *fp = fopen(path, "r");
    if (!fp) return false;
    char line[512];
    bool found = false;
    while (fgets(line, sizeof line, fp)) {
        char k[300];
        TileCand t;
        if (sscanf(line, "%299s %d %d %d %d %d %d %d %d", k, &t.lx, &t.ly, &t.lz, &t.bwx, &t.bwy,
                   &t.bwz, &t.nb, &t.variant) == 9 &&
            key == k) {
            *out = t;
            found = true;      // last entry wins
        }
    }
    fclose(fp);
    return found;
}

// Scratch decoded data for timing: a hash of the index scaled to the int16
// range, stored in the plan's element type (FP32, BF16 or int32).
__global__ void scratch_fill_kernel(void *p, long n, int et)
{
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (long)gridDim.x * blockDim.x) {
        uint32_t h = (uint32_t)q * 2654435761u;
        h ^= h >> 13;
        h *= 0x5bd1e995u;
        h ^= h >> 15;
        const int v = (int)(h & 0xFFFF) - 32768;
        if (et == ET_F32)
            static_cast<float *>(p)[q] = (float)v;
        else if (et == ET_BF16)
            static_cast<uint16_t *>(p)[q] = (uint16_t)(__float_as_uint((float)v) >> 16);
        else
            static_cast<int *>(p)[q] = v;
    }
}

}  // namespace

extern "C" {

int bf_batch_run(bf_plan plan, const int16_t *const *rf, float *const *out, void *stream)
{
    int st = check_batch(plan, rf, out);
    if (st != BF_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if ((st = stage_pointers(plan->batch, rf, out, s)) != BF_OK) return st;
    if ((st = enqueue(plan, s)) != BF_OK) return st;
    return enqueue_gather(plan, s);
}

int bf_graph_launch(bf_plan plan, const int16_t *const *rf, float *const *out, void *stream)
{
    int st = check_batch(plan, rf, out);
    if (st != BF_OK) return st;
    Batch *b = plan->batch;
    hipStream_t s = (hipStream_t)stream;
    if ((st = stage_pointers(b, rf, out, s)) != BF_OK) return st;
    hipError_t e;
    if (!b->exec) {
        if (!b->cap && (e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking)) != hipSuccess)
            return hip_fail(e, "capture stream");
        if ((e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return hip_fail(e, "graph capture begin");
        st = enqueue(plan, b->cap);
        if (st == BF_OK) st = enqueue_gather(plan, b->cap);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(b->cap, &g);
        if (st != BF_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return hip_fail(e, "graph capture end");
        b->graph = g;
        if ((e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0)) != hipSuccess)
            return hip_fail(e, "graph instantiate");
    }
    if ((e = hipGraphLaunch(b->exec, s)) != hipSuccess) return hip_fail(e, "graph launch");
    return BF_OK;
}

int bf_batch_get_frame_info(bf_plan plan, int32_t frame, bf_batch_frame_info *info)
{
    clear_err();
    if (!plan) return fail(BF_ERR_NULL, "plan is NULL");
    if (plan->magic != BF_PLAN_MAGIC) return fail(BF_ERR_STATE, "not a live plan");
    if (!info) return fail(BF_ERR_NULL, "info is NULL");
    if (!plan->batch) return fail(BF_ERR_STATE, "no batched launch yet");
    if (frame < 0 || frame >= (int32_t)plan->batch->info.size())
        return fail(BF_ERR_SHAPE, "frame %d outside the batch", frame);
    *info = plan->batch->info[frame];
    return BF_OK;
}

int bf_autotune(bf_plan plan, const char *cache_path)
{
    if (!plan) return fail(BF_ERR_NULL, "plan is NULL");
    if (plan->magic != BF_PLAN_MAGIC) return fail(BF_ERR_STATE, "not a live plan");
    if (plan->batch) return fail(BF_ERR_STATE, "autotune before the first batched launch");
    hipDeviceProp_t prop;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(e, "device query");
    // Frames of one problem shape (the tune key: mode, transmits, channels,
    // samples, grid, interpolation, element type) form a class: the first
    // frame of each class is tuned on scratch data of its own element type
    // and its choice applies to the whole class.
    std::vector<std::string> keys;
    // (a batch plan tunes under keys of its own: its candidates are restricted, below)
    const bool batch = plan->frames.size() > 1;
    for (Frame *f : plan->frames)
        keys.push_back(tune_key(*f, prop.gcnArchName) + (batch ? "|batch" : ""));
    std::vector<int> done(plan->frames.size(), 0);
    for (size_t c0 = 0; c0 < plan->frames.size(); ++c0) {
        if (done[c0]) continue;
        Frame *f0 = plan->frames[c0];
        const std::string &key = keys[c0];
        TileCand best{};
        bool have = cache_path && cache_lookup(cache_path, key, &best);
        if (!have) {
            void *e_buf = nullptr;
            float *o_buf = nullptr;
            const size_t o_bytes = (size_t)f0->out_elems() * 4;
            if (hipMalloc(&e_buf, f0->e_bytes()) != hipSuccess) return fail(BF_ERR_HIP, "scratch alloc");
            if (hipMalloc(&o_buf, o_bytes) != hipSuccess) {
                (void)hipFree(e_buf);
                return fail(BF_ERR_HIP, "scratch alloc");
            }
            // (IQ data: the real and imaginary parts of a sample as two FP32 values)
            hipLaunchKernelGGL(scratch_fill_kernel, dim3(4096), dim3(256), 0, 0, e_buf,
                               (long)f0->e_elems(), f0->p.iq ? (int)ET_F32 : f0->p.e_type);
            const int saved[7] = {f0->lx, f0->ly, f0->lz, f0->bw[0], f0->bw[1], f0->bw[2], f0->nb};
            const int saved_variant = f0->variant;
            hipEvent_t t0, t1;
            (void)hipEventCreate(&t0);
            (void)hipEventCreate(&t1);
            float best_ms = 1e30f;
            // the plan's own configuration first: tuning never ends slower
            std::vector<TileCand> cands{
                {saved[0], saved[1], saved[2], saved[3], saved[4], saved[5], saved[6], saved_variant}};
            const std::vector<TileCand> more = candidates(*f0);
            cands.insert(cands.end(), more.begin(), more.end());
            // A batch plan runs each kernel class (mode, type, interpolation,
            // points per lane, workgroup size) as one persistent launch: its
            // candidates keep the workgroup size, the points per lane and the
            // LDS kernel, so that tuning one class does not split it into
            // separate launches that run one after the other.
            const int threads0 = saved[3] * saved[4] * saved[5];
            for (const TileCand &t : cands) {
                if (batch && (t.bwx * t.bwy * t.bwz != threads0 || t.variant != saved_variant))
                    continue;
                f0->set_tile(t.lx, t.ly, t.lz);
                f0->bw[0] = t.bwx;
                f0->bw[1] = t.bwy;
                f0->bw[2] = t.bwz;
                f0->nb = t.nb;
                f0->variant = t.variant;
                LdsCfg cfg;
                if (t.variant != BF_DAS_GATHER &&
                    !f0->lds_config(f0->das_args(e_buf, o_buf, f0->p.c), &cfg))
                    continue;
                if (f0->das(e_buf, o_buf, f0->p.c, 0) != BF_OK) continue;   // warm-up
                (void)hipEventRecord(t0, 0);
                for (int r = 0; r < 3; ++r) (void)f0->das(e_buf, o_buf, f0->p.c, 0);
                (void)hipEventRecord(t1, 0);
                (void)hipEventSynchronize(t1);
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, t0, t1);
                if (ms < best_ms) {
                    best_ms = ms;
                    best = t;
                }
            }
            (void)hipEventDestroy(t0);
            (void)hipEventDestroy(t1);
            (void)hipFree(e_buf);
            (void)hipFree(o_buf);
            if (best_ms >= 1e30f)
                best = {saved[0], saved[1], saved[2], saved[3], saved[4], saved[5], saved[6],
                        saved_variant};
            else if (cache_path) {
                FILE *fp = fopen(cache_path, "a");
                if (fp) {
                    fprintf(fp, "%s %d %d %d %d %d %d %d %d\n", key.c_str(), best.lx, best.ly,
                            best.lz, best.bwx, best.bwy, best.bwz, best.nb, best.variant);
                    fclose(fp);
                }
            }
        }
        for (size_t f = c0; f < plan->frames.size(); ++f)
            if (keys[f] == key) {
                Frame *fr = plan->frames[f];
                fr->set_tile(best.lx, best.ly, best.lz);
                fr->bw[0] = best.bwx;
                fr->bw[1] = best.bwy;
                fr->bw[2] = best.bwz;
                fr->nb = best.nb;
                fr->variant = best.variant;
                done[f] = 1;
            }
    }
    return BF_OK;
}

}  // extern "C"
