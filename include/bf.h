/*
 * bf.h -- C ABI of libbf: Hadamard aperture decoding and delay-and-sum (DAS)
 * beamforming of row-column / TOBE array channel data on AMD MI355X (gfx950).
 *
 * Method: arXiv 2512.11086, "An Open Source Realtime GPU Beamformer for RCA
 * and TOBE Arrays".  The path is: int16 RF channel data -> Hadamard decode
 * across transmits (Sec. IV-A; Sec. VII-E) -> DAS with receive apodization
 * (Eqs. 1-3; Sec. VII-F) and fractional-delay interpolation (Sec. IV-B).
 * Optionally the RF is first demodulated to complex baseband (IQ), filtered
 * and decimated (Eq. 4; Sec. VII-D), decoded as complex int16 and
 * beamformed as IQ data with a per-term phase rotation.
 *
 * Conventions shared by every entry point
 *  - Every function returns a bf_status (0 = BF_OK, < 0 = error).  Nothing
 *    aborts or throws.  On error, bf_last_error() returns a message for the
 *    calling thread.  Arguments are validated before any device work is
 *    queued, so a failed call leaves device memory untouched.
 *  - Data pointers marked "device" are device memory owned by the caller,
 *    contiguous in the documented layout.  Pointers marked "host" are read
 *    during the call only (the library copies what it keeps).
 *  - All device work is queued on the caller's stream (`stream` is a
 *    hipStream_t; NULL = the legacy default stream) and is asynchronous.
 *    Faults inside kernels surface on later HIP calls on that stream.
 *  - A plan owns its device tables and workspaces; bf_plan_destroy frees
 *    them.  A plan must not be used concurrently from two host threads, and
 *    two streams must not run calls of the same plan at the same time (the
 *    calls share the plan's workspaces).
 *  - No buffer may exceed 2^31 elements (the paper's limit is 2 GB of data
 *    per call, Table I): larger requests fail with BF_ERR_TOO_LARGE.
 *
 * Layouts
 *  rf   int16            [n_tx][n_ch][n_samples]   encoded channel data, sample fastest
 *  e    f32 | bf16 | i32 [n_tx][n_ch][n_samples]   decoded data (type = params.e_type)
 *  out  f32              [Ny][Nx][Nz]              image / volume, z (depth) fastest
 * IQ plans (params.iq = 1) add a trailing (re, im) pair to each:
 *  rf   int16 [n_tx][n_ch][n_samples][2],  e  f32 [n_tx][n_ch][n_samples][2],
 *  out  f32   [Ny][Nx][Nz][2]
 */
#ifndef BF_H
#define BF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BF_ABI_VERSION 8

/* Largest frame count of bf_das_frames / bf_das_adjoint_frames. */
#define BF_MAX_FRAMES 4096

typedef enum {
    BF_OK = 0,
    BF_ERR_NULL = -1,          /* a required pointer is NULL                          */
    BF_ERR_SHAPE = -2,         /* a count is out of range or inconsistent             */
    BF_ERR_NOT_HADAMARD = -3,  /* an entry is not +-1 or H H^T != N I                 */
    BF_ERR_GEOMETRY = -4,      /* non-finite or non-physical geometry / timing value  */
    BF_ERR_UNSUPPORTED = -5,   /* a valid request this library does not implement     */
    BF_ERR_TOO_LARGE = -6,     /* a buffer would exceed 2^31 elements                 */
    BF_ERR_HIP = -7,           /* a HIP runtime call failed                           */
    BF_ERR_NO_DEVICE = -8,     /* no gfx950 device is available                       */
    BF_ERR_STATE = -9          /* call does not fit the plan (e.g. batch on 1 frame)  */
} bf_status;

/* Acquisition method (Table I).  uFORCES / uHERCULES are the same modes with a
 * sparse transmit subset in tx_elements.  TPW and VLS are the conventional
 * row-column volume methods (Sec. II capabilities): columns transmit tilted
 * plane waves (TPW) or waves through virtual line sources (VLS), rows receive
 * (a row is a line element along x at y_j, receiving in the y-z plane). */
enum { BF_FORCES_2D = 0, BF_HERCULES_3D = 1, BF_TPW_3D = 2, BF_VLS_3D = 3 };
/* Fractional-delay interpolation (Sec. IV-B; Table I). */
enum { BF_INTERP_NEAREST = 0, BF_INTERP_LINEAR = 1, BF_INTERP_CUBIC = 2 };
/* Element type of decoded data (written by bf_decode, read by bf_das). */
enum { BF_E_F32 = 0, BF_E_BF16 = 1, BF_E_I32 = 2 };
/* Decode arithmetic: exact int8 matrix-core product, or FP32 FMA (also exact
 * for |values| < 2^24, i.e. for every int16 input with n_tx <= 256). */
enum { BF_DECODE_MFMA_I8 = 0, BF_DECODE_FMA_F32 = 1 };

/* Problem description: the data description and beamforming parameters of
 * Sec. VI-B (array pitch, 4x4 transform, transmit sequence and Hadamard
 * order, sampling rate, sound speed, output region and resolution, channel
 * mapping). */
typedef struct {
    int32_t mode;              /* BF_FORCES_2D, BF_HERCULES_3D, BF_TPW_3D, BF_VLS_3D     */
    int32_t n_tx;              /* transmits per frame = Hadamard order, 1..256          */
    int32_t n_ch;              /* receive data channels, 1..1024                        */
    int32_t n_samples;         /* samples per channel, 1..65536                         */
    int32_t n_elem[2];         /* element columns (x), rows (y) of the array            */
    double  pitch[2];          /* column pitch (x), row pitch (y), metres, > 0          */
    /* Row-major 4x4 affine from the global frame to the array frame, whose origin
     * is the centre of the corner element and whose z axis is the array normal.
     * The last row must be 0 0 0 1.  A single centred array uses a translation
     * by ((n_elem[0]-1)/2 pitch[0], (n_elem[1]-1)/2 pitch[1], 0). */
    double  xdc_transform[16];
    /* host, n_tx*n_tx, row-major: hadamard[k*n_tx+i] = polarity (+-1) of element
     * i in transmit k.  Any matrix with H H^T = N I is accepted (checked exactly).
     * NULL: the acquisition is not encoded and decoding is the identity. */
    const int8_t  *hadamard;
    /* host, n_tx: element column behind decoded transmit i; NULL = 0..n_tx-1.
     * A sparse subset gives uFORCES / uHERCULES. */
    const int32_t *tx_elements;
    /* host, n_ch: element column (FORCES) or row (HERCULES, TPW, VLS) of data
     * channel j; NULL = 0..n_ch-1. */
    const int32_t *channel_map;
    double  fs;                /* sampling rate, Hz, > 0                                */
    double  fc;                /* centre frequency, Hz (informational for RF data)      */
    double  c;                 /* default sound speed, m/s, > 0                         */
    double  t0;                /* time of sample 0 relative to the transmit, s          */
    /* Transmit focus, the paper's focal point that encodes the emitted wave:
     * HERCULES: +INFINITY = plane wave; finite < 0 = diverging wave from the
     *   virtual point source (array centre, depth focal_depth), zero delay at
     *   the array centre: tx = |p - v| - |focal_depth|.
     * VLS: depth z_f of the virtual line sources (x of column tx_elements[i],
     *   parallel to y), finite: tx = z_f + sgn(z - z_f) |(x - x_i, z - z_f)|.
     * Ignored by FORCES and TPW. */
    double  focal_depth;
    double  f_number;          /* receive F# of the Hann apodization (Eq. 2); 0 = none  */
    int32_t interp;            /* BF_INTERP_*                                           */
    int32_t e_type;            /* BF_E_*                                                */
    int32_t decode_algo;       /* BF_DECODE_*                                           */
    int32_t out_dims[3];       /* Nx, Ny, Nz output points (Ny = 1 for a B-scan)        */
    double  out_min[3];        /* inclusive region bounds in the global frame, metres:  */
    double  out_max[3];        /*   point k on axis a = min + k (max-min)/(N-1)         */
    /* 0: real RF samples.  1: complex baseband (IQ) samples as written by
     * bf_demodulate (layouts above); fs is then the IQ sampling rate, fc the
     * demodulation frequency fd of Eq. 4, and e_type must be BF_E_F32.  DAS reads
     * the complex trace with the plan's interpolator (real and imaginary parts
     * alike) and rotates each term by exp(+j 2 pi fd (tof - t0)), the phase the
     * demodulation removed at that record time.  IQ plans support bf_decode,
     * bf_das, bf_set_* and bf_autotune; bf_das_adjoint and the batched entry
     * points return BF_ERR_UNSUPPORTED. */
    int32_t iq;
    /* TPW only: host, n_tx tilt angles in radians (|angle| < pi/2) of the plane
     * wave of each transmit in the x-z plane, zero delay at the array centre:
     * tx = (x - x_c) sin(angle) + z cos(angle).  Ignored otherwise. */
    const double *tx_angles;
} bf_params;

typedef struct bf_plan_s *bf_plan;   /* opaque, owned by libbf */

/* DAS kernel variants: LDS-staged trace windows, the direct gather kernel
 * (used automatically when a window would not fit in LDS), or LDS-staged
 * windows with two adjacent depth points per lane (HERCULES and FORCES plans
 * with real data; a wavefront then covers tile[0] x tile[1] x 2 tile[2]
 * points, the default for such plans; a grid whose depth axis is not along
 * the array normal runs BF_DAS_LDS instead, as bf_plan_get_info reports).
 * Results agree to FP32 rounding; the variants differ only in speed. */
enum { BF_DAS_LDS = 0, BF_DAS_GATHER = 1, BF_DAS_LDS_Z2 = 2 };

/* Read-only facts about a plan. */
typedef struct {
    int32_t n_frames;
    int32_t tile[3];           /* DAS voxels per wavefront along x, y, z               */
    int32_t variant;           /* BF_DAS_* kernel bf_das runs for frame 0 (after the
                                  LDS-fit check at the plan's sound speed)              */
    int32_t block[3];          /* wavefront tiles per LDS workgroup along x, y, z      */
    int32_t nb;                /* traces per staged batch (as run: the requested count
                                  trimmed to the LDS budget)                           */
    int64_t workspace_bytes;   /* device memory held by the plan                       */
    int64_t e_elems;           /* elements of decoded data per frame (frame 0; IQ
                                  plans count the two FP32 parts of a sample)          */
    int64_t out_elems;         /* output values per frame (frame 0; IQ: 2 per point)   */
    int32_t channel_groups;    /* workgroup sets the channel sum of bf_das is split over
                                  (small grids; > 1: partial images summed in a fixed
                                  order by a second kernel)                            */
} bf_plan_info;

/* ABI version of the loaded library (BF_ABI_VERSION). */
int32_t bf_abi_version(void);

/* Thread-local message describing the last error of the calling thread
 * ("" if none).  The pointer stays valid until the thread's next bf_ call. */
const char *bf_last_error(void);

/* Validate a problem description without touching the GPU: sizes, geometry,
 * element indices, and the exact Hadamard check H H^T = N I (Sec. VII-E:
 * decoding is a product across transmits).  Returns the status bf_plan_create
 * would return for the same description before its first device call. */
int bf_validate(const bf_params *params);

/* Create a single-frame plan: validates (as bf_validate), selects the
 * kernels, and uploads the geometry and Hadamard tables to the current device.
 * Errors: BF_ERR_NULL / SHAPE / NOT_HADAMARD / GEOMETRY / UNSUPPORTED /
 * TOO_LARGE from validation; BF_ERR_NO_DEVICE if the current device is not a
 * gfx950; BF_ERR_HIP if an allocation or copy fails.  *out is NULL on error. */
int bf_plan_create(const bf_params *params, bf_plan *out);

/* Create a plan for a batch of n_frames (1..4096) frames, each with its own
 * description (params[f]; modes, transmit counts, grids may differ).  The plan
 * owns one decoded-data workspace per frame.  Used by bf_batch_run and
 * bf_graph_launch; bf_decode / bf_das / bf_das_adjoint act on frame 0. */
int bf_plan_create_batch(const bf_params *params, int32_t n_frames, bf_plan *out);

/* Free a plan and its device memory (waits for the device first).  NULL is a no-op. */
int bf_plan_destroy(bf_plan plan);

int bf_plan_get_info(bf_plan plan, bf_plan_info *info);

/* Choose the DAS wavefront tile of the plan by timing the candidate shapes on
 * the device (synchronous; uses scratch data).  If cache_path is non-NULL the
 * choice is read from / appended to that text file, keyed by device and problem
 * shape.  Returns the chosen shape through bf_plan_get_info. */
int bf_autotune(bf_plan plan, const char *cache_path);
/* Set the DAS wavefront tile explicitly: log2 of voxels along x, y, z; they must
 * sum to 6 (64 lanes).  For 2D plans log2_y must be 0. */
int bf_set_tile(bf_plan plan, int32_t log2_x, int32_t log2_y, int32_t log2_z);

/* Select the DAS kernel and its LDS workgroup: variant BF_DAS_*, wavefront
 * tiles per workgroup (product 1..16; bw_y = 1 for 2D plans) and traces per
 * staged batch nb (4..64, multiple of 4; FORCES, TPW and VLS round it down
 * to a multiple of their rows per batch, 4).  Applies to every frame;
 * BF_DAS_LDS_Z2 on a frame that is not HERCULES or FORCES with real data is
 * BF_ERR_UNSUPPORTED; after the first bf_batch_run / bf_graph_launch of the
 * plan it is BF_ERR_STATE. */
int bf_set_das_config(bf_plan plan, int32_t variant, int32_t bw_x, int32_t bw_y, int32_t bw_z,
                      int32_t nb);

/* Decode (Sec. VII-E):  e[i][j][t] = sum_k H[k][i] * rf[k][j][t]  (unscaled, so
 * decoding an encoded set returns N times the element responses).
 * rf: device int16 [n_tx][n_ch][n_samples];  e: device, type params.e_type,
 * same layout.  Exact for BF_E_F32 / BF_E_I32 (|e| <= 256 * 32768 < 2^24);
 * BF_E_BF16 rounds to nearest even.  rf and e must not overlap. */
int bf_decode(bf_plan plan, const int16_t *rf, void *e, void *stream);

/* DAS (Eq. 1 with Eqs. 2-3; Sec. VII-F):
 *   out[p] = sum_i sum_j a(p,i,j) * interp(e[i][j], (tof_ij(p) - t0) * fs)
 * FORCES:   tof = (|p - col(tx_i)|_xz + |p - col(ch_j)|_xz) / c,
 *           a = W(F# |x - x_j| / z)
 * HERCULES: tof = (tx(p) + |p - (x_i, y_j, 0)|) / c,  a = W(F# rho / z), rho radial,
 *           tx = z (plane) or |p - v| - f (diverging, see focal_depth)
 * TPW, VLS: tof = (tx_i(p) + |(y - y_j, z)|) / c,  a = W(F# |y - y_j| / z),
 *           tx_i per tx_angles / focal_depth
 * W is the Hann window (Eq. 3); points with z <= 0 give 0.  Samples outside
 * [0, n_samples) read as 0.  e: device, type params.e_type; out: device f32
 * [Ny][Nx][Nz], overwritten.  c: sound speed for this call (m/s, finite, > 0;
 * the autofocus loop varies it).  Accumulation is FP32 in a fixed order per
 * point, so repeated calls give bit-identical results. */
int bf_das(bf_plan plan, const void *e, float *out, double c, void *stream);

/* bf_das for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and the same result bit for bit, but the partial images of a
 * channel-split launch (grids with fewer than 8192 wavefronts of points; see
 * bf_plan_info.channel_groups) go to a static device array of
 * BF_DAS_NOALLOC_MAX_BYTES per GPU, which the library holds until the process
 * ends, instead of plan memory.  The call itself allocates nothing (the plan
 * is created beforehand, with its tables).  Every call on a GPU shares that
 * GPU's array, so calls that overlap on one GPU (other streams, other host
 * threads) race; calls queued on one stream do not.  The current device must
 * be the plan's (BF_ERR_STATE otherwise).  BF_ERR_TOO_LARGE if the plan's
 * partial images exceed the array (the channel split keeps them below 8 MiB
 * for every plan).  Other errors as bf_das. */
#define BF_DAS_NOALLOC_MAX_BYTES (8u << 20)
int bf_das_noalloc(bf_plan plan, const void *e, float *out, double c, void *stream);

/* Decode fused into DAS (Sec. VII-C's decode -> beamform order in one
 * kernel; decode Sec. VII-E, DAS Eq. 1): FORCES planes only.  Each staged tap
 * of decoded trace (i, j) is formed from the RF as sum_k H[k][i] rf[k][j][n]
 * inside the LDS DAS kernel, so no decoded data is written or read; the sums
 * are exact in FP32, and out equals bf_decode followed by bf_das bit for bit
 * when the plan's e_type is BF_E_F32 or BF_E_I32 (exact decoded values; a
 * BF_E_BF16 plan's bf_decode rounds, the fused taps do not).  rf: device int16 [n_tx][n_ch][n_samples];
 * out: device f32 [Ny][Nx][Nz], overwritten; c as bf_das.  The decode is
 * repeated for every workgroup box that stages a window, so on the
 * workloads measured here this is slower than the two calls (the bench's
 * decode_share object times both).  BF_ERR_UNSUPPORTED for HERCULES, TPW,
 * VLS or IQ plans, the gather variant, or windows that do not fit LDS. */
int bf_das_fused(bf_plan plan, const int16_t *rf, float *out, double c, void *stream);

/* Adjoint of bf_das for the same e and c, given grad_out = dL/d(out)
 * (device f32 [Ny][Nx][Nz]).  The paper defines only the forward sum (Eq. 1
 * with Eqs. 2-3 and the Hermite read of Sec. IV-B); this is its exact
 * transpose in e, and its derivative in c through the delays of Eq. 1 (the
 * apodization of Eq. 2 does not depend on c):
 *   grad_e (device f32 [n_tx][n_ch][n_samples], nullable, overwritten) =
 *       transpose of the linear map e -> out, applied to grad_out;
 *   grad_c (device f32 scalar, nullable, overwritten) =
 *       sum_p grad_out[p] * d out[p] / dc, with d s / dc = -tof * fs / c.
 * e may be NULL when grad_c is NULL (grad_e does not depend on the data).
 * grad_out must be finite.  Linear and cubic reads run on the LDS-staged
 * kernel: grad_c as FP64 workgroup partials summed in a fixed order
 * (bit-identical between calls); grad_e per workgroup in 64-bit fixed point
 * (scaled by the workgroup's largest |grad_out|), then FP32 atomics across
 * workgroups, so its low bits may vary between calls.  Nearest reads, data
 * types other than FP32 (for grad_c) and the BF_DAS_GATHER variant run the
 * gather adjoint (FP32 atomics per term). */
int bf_das_adjoint(bf_plan plan, const void *e, const float *grad_out, double c,
                   float *grad_e, float *grad_c, void *stream);

/* bf_das for a stack of n_frames frames of this plan's geometry, all at
 * sound speed c (e.g. the frames of one sound-speed autofocus batch):
 *   out[f] = bf_das(e[f]) for f < n_frames, bit for bit.
 * e: device, type params.e_type, [n_frames][n_tx][n_ch][n_samples];
 * out: device f32 [n_frames][Ny][Nx][Nz], overwritten.  n_frames in
 * 1..BF_MAX_FRAMES (BF_ERR_SHAPE otherwise).  One launch per frame on the
 * given stream; no allocation. */
int bf_das_frames(bf_plan plan, const void *e, int32_t n_frames, float *out, double c,
                  void *stream);

/* bf_das_adjoint for a stack of frames at one c: grad_out [n_frames][Ny][Nx][Nz],
 * grad_e [n_frames][n_tx][n_ch][n_samples] (nullable), grad_c device f32
 * [n_frames] (nullable): grad_c[f] = sum_p grad_out[f][p] d out[f][p] / dc, the
 * frame's own term (a loss summed over frames has dL/dc = sum_f grad_c[f]).
 * The LDS-staged adjoint takes the whole stack in one launch per gradient
 * (dL/dc: as many frames per launch as the plan's partial-sum buffer holds);
 * the gather adjoint runs frame by frame.  grad_c[f] is bit-identical to
 * bf_das_adjoint on frame f alone; grad_e matches it up to the order of its
 * FP32 atomics.  No allocation.  Errors as bf_das_frames and bf_das_adjoint. */
int bf_das_adjoint_frames(bf_plan plan, const void *e, const float *grad_out, int32_t n_frames,
                          double c, float *grad_e, float *grad_c, void *stream);

/* Image-sharpness loss for n_images images of n_per_image points each (the
 * objective of the sound-speed autofocus; not a step of the paper's
 * pipeline, which images at a given c):
 *   loss[f] = -sum I^4 / (sum I^2)^2   (device f32 [n_images], overwritten)
 *   grad[f][p] = d loss[f] / d I[f][p] (device f32, nullable, overwritten)
 * Sums are accumulated in FP64.  An all-zero image gives loss 0, gradient 0. */
int bf_sharpness(const float *img, int64_t n_per_image, int32_t n_images, float *loss,
                 float *grad, void *stream);

/* Batched decode + DAS of every frame of a batch plan with persistent
 * kernels (one decode launch per Hadamard-order class and one DAS launch per
 * kernel class, each pulling work items from queues).  The frames are the
 * paper's parameter sets (Sec. VI-B: several sets, e.g. cross-plane views or
 * transmit subsets, imaged from one acquisition stream), each decoded
 * (Sec. VII-E) and beamformed (Eq. 1; Sec. VII-F) as by bf_decode + bf_das.
 * rf[f]: device int16 of frame f; out[f]: device f32 of frame f (host arrays of
 * n_frames device pointers).  Decoded data goes to the plan's workspaces. */
int bf_batch_run(bf_plan plan, const int16_t *const *rf, float *const *out, void *stream);

/* Same work as bf_batch_run, recorded once into a hipGraph and replayed on
 * later calls.  The frame pointers are copied into the plan's device table
 * before each replay, so new buffers need no re-capture; a call with the same
 * buffers on the same stream as the last copy (of either entry point) finds
 * them there and copies nothing.  Calls of one plan on different streams must
 * not overlap: they share the table. */
int bf_graph_launch(bf_plan plan, const int16_t *const *rf, float *const *out, void *stream);

/* How the batched path runs frame f of a batch plan (after its first
 * bf_batch_run or bf_graph_launch; BF_ERR_STATE before, BF_ERR_SHAPE for f
 * out of range). */
enum { BF_BATCH_PERSISTENT_LDS = 0, BF_BATCH_GATHER = 1, BF_BATCH_FRAME_LDS = 2 };
typedef struct {
    int32_t das_path;          /* BF_BATCH_PERSISTENT_LDS, BF_BATCH_GATHER or
                                  BF_BATCH_FRAME_LDS (its own LDS launch, in the same
                                  pass and graph: a frame of a kernel class too small
                                  for the persistent launch without a channel split,
                                  whose own launch fills the GPU)                       */
    int32_t das_class;         /* index of its persistent DAS launch (-1: otherwise)     */
    int32_t channel_groups;    /* work items per box along the channel sum (>= 1)        */
    int32_t decode_class;      /* index of its persistent decode launch                  */
    int64_t das_items;         /* DAS work items of the frame                            */
} bf_batch_frame_info;
int bf_batch_get_frame_info(bf_plan plan, int32_t frame, bf_batch_frame_info *info);

/* ---------------------------------------------------------------------------
 * Demodulation (Eq. 4; Sec. VII-D): the stage before decoding.
 *   y[n]  = sum_{k=0}^{N_f-1} h[k] x[n-k] exp(-j 2 pi fd (n-k) / fs),  x[n<0] = 0
 *   iq[q] = y[q D],   q = 0 .. n_out-1,  n_out = ceil(n_samples / D)
 * i.e. mix every sample with the carrier (n counted from sample 0 of the
 * record), filter with h (the baseband matched filter, which also acts as the
 * low-pass; real or complex taps), then keep every D-th output (decimation
 * after the low-pass).  The filter is causal and not delay-compensated: fold
 * its group delay into the t0 of the IQ plan if wanted.  Computed in FP32;
 * BF_IQ_I16 output is rounded to nearest (ties to even) and saturated to int16,
 * which loses nothing for filters with gain <= 1 (the paper's convention), so
 * the data do not grow for the next stage.
 *   rf: device int16 [n_traces][n_samples] (n_traces = n_tx * n_ch of a frame)
 *   iq: device [n_traces][n_out][2] (re, im), int16 or f32 per out_type; for
 *       int16 this is exactly the rf layout of an IQ plan with n_samples = n_out.
 * ------------------------------------------------------------------------- */
enum { BF_IQ_I16 = 0, BF_IQ_F32 = 1 };

typedef struct {
    int32_t n_traces;          /* traces per call, >= 1                                */
    int32_t n_samples;         /* input samples per trace, 1..65536                    */
    int32_t decimation;        /* D, 1..16                                             */
    int32_t n_taps;            /* filter length N_f, 1..1024                           */
    const double *taps_re;     /* host, n_taps: real parts of h (copied at create)     */
    const double *taps_im;     /* host, n_taps, or NULL for a real filter              */
    double fs;                 /* input sampling rate, Hz, > 0                         */
    double fd;                 /* demodulation frequency, Hz, finite                   */
    int32_t out_type;          /* BF_IQ_I16 or BF_IQ_F32                               */
} bf_demod_params;

typedef struct bf_demod_s *bf_demod;   /* opaque, owned by libbf */

/* Validate, then upload the filter (folded with the mix, FP64 -> FP32) and the
 * output rotations to the current device.  Errors as bf_plan_create (SHAPE for
 * counts out of range, GEOMETRY for non-finite fs / fd / taps). */
int bf_demod_create(const bf_demod_params *params, bf_demod *out);
/* Free a demodulator (waits for the device first).  NULL is a no-op. */
int bf_demod_destroy(bf_demod d);
/* Output samples per trace, ceil(n_samples / D). */
int bf_demod_out_samples(bf_demod d, int32_t *n_out);
/* Demodulate one frame on `stream` (asynchronous).  rf and iq must not overlap. */
int bf_demodulate(bf_demod d, const int16_t *rf, void *iq, void *stream);

/* ---------------------------------------------------------------------------
 * Envelope and display compression: the stage after DAS (the paper applies a
 * Hilbert transform to the beamformed image and shows it on a log scale with
 * an adjustable dynamic range or on a power scale with an adjustable
 * threshold).
 *   RF image (iq = 0): env = |x_a|, x_a the analytic signal of each depth
 *     column: X = DFT_N(x), X_a[k] = h[k] X[k] with h = 1 at DC and at N/2,
 *     2 for 0 < k < N/2, 0 above; x_a = IDFT_N(X_a) (circular over the
 *     column's N samples, no padding).
 *   IQ image (iq = 1): env = |z|.
 *   compress BF_COMPRESS_NONE:  y = env
 *            BF_COMPRESS_LOG:   y = max(20 log10(env / ref), -param)  (param: dynamic range, dB)
 *            BF_COMPRESS_POWER: y = min(env / ref, 1)^param          (ref: threshold, param: exponent)
 *   ref > 0 is used as given; ref <= 0 takes the maximum envelope of the image
 *   (computed on the device; an all-zero image gives -param / 0).
 * img: device f32 [n_cols][n] (depth fastest: a [Ny][Nx][Nz] volume has
 * n_cols = Ny*Nx, n = Nz) or, for iq = 1, complex f32 [n_cols][n][2];
 * out: device f32 [n_cols][n] (must not overlap img).  FP32 arithmetic: for
 * power-of-two n from 64 to 1024 a register-resident FFT per pair of columns
 * (two real columns as one complex transform: the inverse DFT of
 * -j sgn(k) DFT(x1 + j x2) is H{x1} + j H{x2}, and env = sqrt(x^2 + H{x}^2));
 * other powers of two a radix-2 FFT in LDS; a direct circular sum otherwise.
 * A plan holds its tables and a partial-maximum buffer, so calls of one plan
 * must not overlap on the device.
 * ------------------------------------------------------------------------- */
enum { BF_COMPRESS_NONE = 0, BF_COMPRESS_LOG = 1, BF_COMPRESS_POWER = 2 };

typedef struct bf_env_s *bf_env;      /* opaque, owned by libbf */

/* n_cols >= 1, n in 1..4096, iq 0 or 1.  Errors: SHAPE, UNSUPPORTED, TOO_LARGE,
 * NO_DEVICE, HIP. */
int bf_env_create(int64_t n_cols, int32_t n, int32_t iq, bf_env *out);
/* Free an envelope plan (waits for the device first).  NULL is a no-op. */
int bf_env_destroy(bf_env e);
/* Envelope + compression on `stream` (asynchronous).  GEOMETRY if ref is not
 * finite or, when compressing, param is not finite and > 0. */
int bf_envelope(bf_env e, const float *img, float *out, int32_t compress, double ref,
                double param, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* BF_H */
