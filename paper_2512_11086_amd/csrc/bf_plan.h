// bf_plan.h -- internal plan and frame objects of libbf (host side).
#pragma once

#include <stdint.h>

#include <vector>

#include "bf.h"
#include "bf_common.h"

namespace bf {

int fail(int code, const char *fmt, ...);
void clear_err();
int hip_fail(hipError_t e, const char *what);
int validate_params(const bf_params *p);

// One frame of a plan: its description, host copies of the tables and the
// device tables the kernels read.
struct Frame {
    bf_params p;                 // copy; pointer members cleared
    std::vector<int8_t> H;       // [n_tx][n_tx]
    std::vector<int> tx, ch;     // element column / channel element
    int kb = 1;                  // 32-wide K blocks of the int8 decode
    Grid grid;
    int lx = 2, ly = 2, lz = 2;  // DAS wavefront tile (log2)
    int bw[3] = {4, 4, 1};       // wavefront tiles per LDS workgroup (x, y, z)
    int nb = 16;                 // traces per staged batch
    int variant = 0;             // BF_DAS_LDS, BF_DAS_GATHER or BF_DAS_LDS_Z2
    int sorted_tx = 0;           // transmit columns ascending
    int uniform_tx = 0;          // transmit columns equally spaced (ascending)
    float tx_x0 = 0.f, tx_inv_dx = 0.f;
    double tpw_smax = 0.0;       // TPW: largest |sin| of the transmit angles
    int groups = 1;              // channel groups of the DAS launch (small grids)
    int stack_cap = 0;           // frames per adjoint launch of a stack (0: no cap)
    float *d_part = nullptr;     // [groups][points] partial images
    float2 *d_hann = nullptr;    // Hann weight table (HANN_N + 1 entries)
    long max_blocks = 0;
    int8_t *d_At = nullptr;
    int *d_colsum = nullptr;
    float *d_Hf = nullptr;
    float *d_tx_x = nullptr, *d_rx_c = nullptr;
    float2 *d_tx_sc = nullptr;   // TPW: (sin, cos - 1) per transmit
    double *d_partial = nullptr;
    void *d_e = nullptr;         // batch plans: decoded-data workspace
    std::vector<void *> allocs;
    int64_t total_bytes = 0;

    ~Frame();
    void *alloc(size_t bytes);
    int init(const bf_params &src);
    void set_tile(int lx, int ly, int lz);
    int64_t e_elems() const;
    int64_t out_elems() const;
    int das_et() const;          // element type of the DAS kernels (ET_CF32 for IQ plans)
    size_t e_bytes() const;
    DecodeArgs decode_args(const int16_t *rf, void *e) const;
    DasArgs das_args(const void *e, float *out, double c) const;
    bool lds_config(const DasArgs &a, LdsCfg *cfg, int adj = 0, const int *bw_adj = nullptr) const;
    void adjoint_e_tile(DasArgs *a, int bw_out[3]) const;   // the RF gradient's lane tile
    bool z2_ok() const;          // two depth points per lane apply to this frame
    int decode(const int16_t *rf, void *e, hipStream_t s) const;
    // part: partial images of a channel-split launch (nullptr: the plan's own)
    int das(const void *e, float *out, double c, hipStream_t s, float *part = nullptr) const;
    // decode fused into DAS (FORCES planes with real data, LDS path): rf int16
    int das_fused(const int16_t *rf, float *out, double c, hipStream_t s) const;
    DasArgs at_frame(const DasArgs &a, int f0) const;
    int das_frames(const void *e, int nf, float *out, double c, hipStream_t s) const;
    int das_adjoint(const void *e, const float *grad_out, double c, float *grad_e, float *grad_c,
                    int nf, hipStream_t s) const;
};

struct Batch;   // persistent batched path state (bf_batch.hip)

hipError_t launch_das(const DasArgs &a, int mode, int et, int ip, hipStream_t s);
hipError_t launch_das_lds(const DasArgs &a, const LdsCfg &c, int mode, int et, int ip,
                          hipStream_t s);
hipError_t launch_das_lds_fused(const DasArgs &a, const LdsCfg &c, int ip, hipStream_t s);
size_t lds_bytes(int n_tx, int n_ch, int nb, int lmax, int qs, int guard, int adj, int mode);
hipError_t launch_das_lds_adjoint(const DasArgs &a, const LdsCfg &c, int mode, int ip,
                                  float *grad_c, hipStream_t s, int n_frames = 1);

constexpr uint32_t BF_PLAN_MAGIC = 0xBF0C0DE5u;

}  // namespace bf

struct bf_plan_s {
    uint32_t magic = bf::BF_PLAN_MAGIC;
    int device = 0;
    std::vector<bf::Frame *> frames;
    bf::Batch *batch = nullptr;
    ~bf_plan_s();
    int64_t workspace_bytes() const;
};
