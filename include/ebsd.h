/*
 * ebsd.h -- C ABI of the MI355X (gfx950) demons-based HR-EBSD remapping library.
 *
 * Method: Zhu, Kaufmann & Vecchio, "Novel Remapping Approach for HR-EBSD based
 * on Demons Registration" (arXiv:1907.05993).  For every scan point a test
 * pattern is registered against its reference pattern by multi-resolution
 * demons (section 1, Eq. (1)); the displacement field sampled at the ROI
 * centres gives shifts q (section 2), from which the deformation gradient F is
 * solved through the projective model of Eq. (2) by minimising Eq. (3); its
 * rotation R_finite = P Q^T (Eq. (4)-(5)) remaps the reference, a second-pass
 * ROI cross-correlation (section 2) measures the residual shifts, and
 * F = F_inf R_finite (Eq. (12)).  The rotation is reported as a rotation vector
 * (the axis-angle form after Eq. (5), Eq. (6)).
 *
 * Conventions
 *   - Patterns are H x W fp32, row-major, x = column, y = row, pixel centres
 *     at integers.  Pattern centre: x* = pc_x W - 0.5, y* = pc_y H - 0.5,
 *     detector distance Z* = pc_z W (px); r(x) = (x - x*, y - y*, Z*),
 *     k = (0, 0, 1).
 *   - Displacement field: [2][H][W] fp32 on the reference grid, channel 0
 *     along x, channel 1 along y, in full-resolution px, defined by
 *     test(x + u(x)) ~ ref(x); u at a ROI centre is the shift q of Eq. (2).
 *   - F, R: 3 x 3 row-major fp64 in the detector frame above; det F = 1
 *     (the shifts fix F only up to scale; the isochoric normalisation stands in
 *     for the traction-free condition).
 *
 * Memory and streams
 *   - Every pattern, field and result pointer is HIP device memory owned by the
 *     caller.  The pair array itself is host memory, read during the call.
 *   - The handle owns its workspace (device memory it allocates and grows on
 *     demand) and a small pinned staging buffer.  Growing the workspace
 *     synchronises the device first.
 *   - Calls are asynchronous on `stream` (a hipStream_t; NULL = the default
 *     stream): outputs are valid once the stream has completed.  A handle is
 *     used by one host thread at a time; different handles may run in
 *     different threads at once (the library keeps its graph captures apart
 *     from its device-wide waits, workspace growth and frees).
 *   - Errors: every call validates all of its arguments before anything is
 *     enqueued and returns a negative EBSD_E* code (outputs untouched).
 *     Numerical outcomes never fail a batch: they are reported per pair in
 *     the status bits.  No exception or abort crosses the ABI.
 */
#ifndef EBSD_H
#define EBSD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EBSD_ABI_VERSION 5
#define EBSD_MAX_LEVELS 8

/* return codes */
enum {
    EBSD_OK = 0,
    EBSD_EINVAL = -1,   /* bad argument (NULL pointer, n < 0, bad parameter value) */
    EBSD_ESHAPE = -2,   /* pattern size not supported (coarsest level under 4 x 4, over 16384) */
    EBSD_EROI = -3,     /* a ROI falls outside the pattern, or ROI size is not 32/64/128/256 */
    EBSD_ENOMEM = -4,   /* device or pinned allocation failed */
    EBSD_EDEVICE = -5,  /* a HIP runtime call failed */
    EBSD_ENOTSUP = -6,  /* feature not available in this library */
    EBSD_ENOMODEL = -7, /* warm start requested but no network parameters loaded */
    EBSD_EVERSION = -8, /* ebsd_params.struct_size does not match this library */
    EBSD_EIO = -9,      /* a parameter file could not be read or written */
    EBSD_ETOOBIG = -10  /* input larger than an allocation-free entry point's fixed device buffer */
};

/* per-pair status bits */
enum {
    EBSD_CONVERGED = 1,         /* tol > 0 and every level stopped on the tolerance */
    EBSD_HIT_CAP = 2,           /* tol > 0 and some level ran to its iteration cap */
    EBSD_WARM_USED = 4,         /* warm start: the network's field started demons */
    EBSD_WARM_FALLBACK = 8,     /* warm start: the field failed the Eq. (2) fit test; demons started from zero */
    EBSD_SOLVE_ILLCOND = 16,    /* an Eq. (3) solve was ill-conditioned (cond(J^T J) > 1e12) */
    EBSD_NONFINITE_INPUT = 32,  /* a pattern held NaN/Inf (treated as all-zero) */
    EBSD_DEGENERATE_INPUT = 64  /* a pattern had no contrast (treated as all-zero) */
};

typedef struct ebsd_params {
    uint32_t struct_size;                 /* sizeof(ebsd_params) */
    int32_t levels;                       /* pyramid levels, 1..8 (multi-resolution demons); level l is the
                                             pattern halved l times, sizes rounding up (an odd size keeps
                                             its last pixel), and must keep 4 x 4 pixels */
    int32_t max_iters[EBSD_MAX_LEVELS];   /* demons iterations per level, [0] = finest */
    float sigma_px;                       /* Gaussian smoothing of the accumulated field, 0 <= sigma <= 1.3 */
    float tol_px;                         /* stop a level when 2^l RMS|u_new - u| < tol (full-res px); 0 = fixed count */
    double pc_x, pc_y, pc_z;              /* pattern centre fractions */
    int32_t n_roi;                        /* ROIs: 1 at the pattern centre + (n_roi - 1) on a ring, 5..256 */
    int32_t roi_size;                     /* 32, 64, 128 or 256 (the paper's size) */
    double roi_radius_frac;               /* ring radius / W */
    int32_t window;                       /* 1 = Hann window on each ROI (section 2), 0 = none */
    int32_t second_pass;                  /* 1 = remap + XCF second pass (Eq. (12)); 0 = demons only */
    int32_t warm_start;                   /* square 128, 256 or 512 px, 3 levels: 1 = start demons from the
                                             network's field, 2 = from the Eq. (2) field fitted to it; 0 = zero */
    float fallback_residual_px;           /* warm start: largest RMS misfit of the Eq. (2) fit, in
                                             full-resolution px of the registered pattern (0.5) */
    int32_t remap_interp;                 /* remap before the XCF (section 2, before Eq. (12)): 3 = cubic
                                             B-spline interpolation (the paper's cubic scheme), 1 = bilinear */
    int32_t xcf_passes;                   /* remap + XCF + Eq. (12) passes, 1..16: pass 1 remaps by R_finite
                                             and composes with it (the paper's method), pass k > 1 remaps by
                                             pass k-1's F and composes with that F */
    int32_t first_pass;                   /* 0 = demons (the paper's method); 1 = the conventional first
                                             pass it is compared with (sections 1 and 3): q1 is the ROI
                                             cross-correlation of the unremapped patterns, no demons run,
                                             the field output is not written and iters are 0; needs
                                             warm_start = 0 */
    float bandpass_lo_px;                 /* pre-filter of every raw pattern before normalisation (section
                                             3.3: low-pass against noise, high-pass against background):
                                             sigma of the Gaussian low-pass, 0 = off, <= 32 */
    float bandpass_hi_px;                 /* sigma of the Gaussian background estimate subtracted, 0 = off,
                                             <= 32; the filtered pattern is G_lo * p - G_hi * p (taps
                                             exp(-j^2 / 2 sigma^2), |j| <= floor(3 sigma + 0.5), unit sum,
                                             replicated border) */
    int32_t background_static;            /* background correction before the pre-filter (section 3.3):
                                             1 = divide every raw pattern by the static background, the
                                             pixelwise mean of the size bucket's test patterns; 0 = off */
    float background_dynamic_px;          /* then divide by the pattern's own Gaussian blur of this sigma
                                             (the pre-filter's taps; 0 = off, <= 32); a non-positive
                                             divisor gives 0 */
} ebsd_params;

/* One scan point.  ref/test: device pointers to H x W fp32 patterns.  Pairs
 * with the same ref_id >= 0 share one reference (same pointer and size) whose
 * pyramid is built once; ref_id < 0 means "not shared". */
typedef struct ebsd_pair {
    const float* ref;
    const float* test;
    int32_t H, W;
    int32_t ref_id;
} ebsd_pair;

/* Outputs (device memory, caller-allocated; any pointer may be NULL). */
typedef struct ebsd_outputs {
    float* field;               /* final displacement field, [2][H][W] per pair, full-res px */
    const int64_t* field_offset;/* HOST array [n]: float offset of pair i's field; NULL = i*2*H*W */
    double* F;                  /* [n][9] total deformation gradient, det F = 1 (Eq. (12)) */
    double* R;                  /* [n][9] rotation of F (Eq. (4)-(5)) */
    double* rotvec;             /* [n][3] rotation vector theta*m, rad */
    double* R_finite;           /* [n][9] first-pass rotation used for the remap */
    double* F_first;            /* [n][9] first-pass deformation gradient (det 1) */
    float* q1;                  /* [n][n_roi][2] first-pass shifts (field at ROI centres) */
    float* q2;                  /* [n][n_roi][2] second-pass XCF shifts */
    float* peak_height;         /* [n][n_roi] normalised XCF peak height */
    int32_t* iters;             /* [n][levels] demons iterations run per level */
    uint32_t* status;           /* [n] status bits */
    float* warm_field;          /* [n][64][64][2] network output (warm start), px of the 256 x 256 image it saw */
    float* warm_misfit;         /* [n] RMS misfit of the Eq. (2) fit to warm_field, in the same px */
    double* mae_first;          /* [n] mean angular error of the first fit (F_first to q1), rad */
    double* mae;                /* [n] mean angular error of the last fit (F_inf to the last pass's q2;
                                   F_first to q1 without a second pass), rad.  Mean angular error:
                                   the mean over the ROIs of the angle between F r_i and r_i + q_i
                                   (the quality figure section 3 compares the methods by) */
    double* ssim;               /* [n] structural similarity of the registration (the SSIM section 3
                                   reports for demons): mean over the pixels whose 11 x 11 window fits
                                   (Gaussian, sigma 1.5 px) of SSIM(R, T(x + u(x))) between the
                                   normalised reference and the test warped by the final field,
                                   C1 = (0.01 L)^2, C2 = (0.03 L)^2, L = 6 (z-scored patterns); NaN with
                                   the XCF first pass or a pattern of 10 px or less; computed only when
                                   this pointer is set */
    double* omega;              /* [n][9] Eq. (6)'s rotation tensor of rotvec (theta):
                                   omega_ij = -eps_ijk theta_k, row-major, rad (the cross-product
                                   matrix of theta, the logarithm of R) */
} ebsd_outputs;

/* Library ABI version (EBSD_ABI_VERSION). */
int ebsd_version(void);

/* Fill *p with the defaults: 3 levels x 150 iterations, sigma 1 px, tol 0,
 * pattern centre (0.5, 0.5, 0.7), 20 ROIs of 64 px on a ring of 0.3 W, Hann
 * window, second pass on (cubic B-spline remap, one pass), demons first
 * pass, warm start off (fallback misfit 0.5 px).  Returns EBSD_OK or
 * EBSD_EINVAL (p == NULL). */
int ebsd_params_default(ebsd_params* p);

/* Human-readable text of a return code (static storage). */
const char* ebsd_strerror(int code);

typedef struct ebsd_handle ebsd_handle;

/* Create a handle bound to HIP device `device` with parameters *p (copied).
 * Returns EBSD_EVERSION if p->struct_size != sizeof(ebsd_params),
 * EBSD_EINVAL for an invalid parameter, EBSD_EDEVICE if the device cannot be
 * selected.  On success *out receives the handle (no device memory yet). */
int ebsd_create(const ebsd_params* p, int device, ebsd_handle** out);

/* Release the handle, its workspace and staging buffers after synchronising
 * the device.  NULL is accepted. */
int ebsd_destroy(ebsd_handle* h);

/* Copy the handle's parameters into *out. */
int ebsd_get_params(const ebsd_handle* h, ebsd_params* out);

/* ROI layout used by the handle's parameters for an H x W pattern (section 2:
 * ROIs evenly spaced on a ring around the pattern centre plus one at the
 * centre).  ROI 0 is at the pattern centre, ROI j >= 1 at angle
 * 2 pi (j-1)/(n_roi-1) from +x toward +y on a ring of radius frac W; top-left
 * x0 = floor(c - (N-1)/2 + 0.5); the centre used in Eq. (2) is x0 + (N-1)/2.
 * cx, cy (double) and x0, y0 are HOST arrays of n_roi entries (any may be
 * NULL).  Returns EBSD_EROI if a ROI leaves the pattern. */
int ebsd_roi_layout(const ebsd_params* p, int32_t H, int32_t W, double* cx, double* cy,
                    int32_t* x0, int32_t* y0);

/* The whole path for n pairs: per-pattern normalisation, pyramids, demons
 * (Eq. (1)) coarse to fine, q1 at the ROI centres, F_first by Eq. (3),
 * R_finite = polar(F_first) (Eq. (4)-(5)), remap + ROI XCF (section 2), F_inf
 * by Eq. (3), F = F_inf R_finite (Eq. (12)), R = polar(F), rotation vector.
 * pairs: HOST array of n descriptors (device pattern pointers); pairs of
 * different sizes are processed in size buckets, in order of first
 * appearance.  n == 0 is a no-op.  stream: hipStream_t or NULL. */
int ebsd_register_batch(ebsd_handle* h, const ebsd_pair* pairs, int32_t n,
                        const ebsd_outputs* out, void* stream);

/* Same as ebsd_register_batch, but demons starts on the coarsest level from
 * the caller's field u_init (device, [n][2][h][w] fp32, h x w the coarsest
 * level's size: H and W halved L-1 times rounding up, in
 * full-resolution px) instead of zero: the warm start.  All pairs must have
 * the same size.  u_init == NULL behaves as ebsd_register_batch. */
int ebsd_register_batch_init(ebsd_handle* h, const ebsd_pair* pairs, int32_t n,
                             const float* u_init, const ebsd_outputs* out, void* stream);

/* Pipelined registration (throughput of a stream of batches).  A pipeline
 * owns `depth` (1..8) registration handles created with the same parameters,
 * each with its own stream, workspace, captured graphs and host thread.
 * Batches submitted in turn go to the handles round-robin and run back to back
 * on each, so `depth` batches are in flight at once: one batch's network
 * forward, coarse levels and second pass overlap another's finest demons
 * level.  Each batch is an ebsd_register_batch call on its handle: outputs
 * are identical bit for bit.
 * The pipeline's memory is depth times one handle's.
 *
 * ebsd_pipeline_create: EBSD_EINVAL unless 1 <= depth <= 8 (and as
 * ebsd_create).  ebsd_pipeline_handle: the handle of slot 0 <= slot < depth,
 * owned by the pipeline, for configuration (ebsd_load_model, ebsd_autotune,
 * ebsd_set_graphs, ...) while no batch is pending; do not destroy it or call
 * its registration functions directly.  ebsd_pipeline_submit: validates as
 * ebsd_register_batch, copies `pairs` and `*out` (and the host field_offset
 * array) and returns without waiting; the batch starts after the work already
 * on `stream`; the caller keeps the patterns and outputs alive and unchanged
 * until `stream` has passed the point at which a later ebsd_pipeline_wait made
 * it wait (work enqueued on `stream` after that call sees the results).
 * Errors of a submitted batch are reported
 * by the next ebsd_pipeline_wait.  ebsd_pipeline_wait: blocks until every
 * submitted batch has been issued, then makes `stream` wait for their
 * completion; returns the first error since the previous wait.
 * ebsd_pipeline_destroy: waits for the submitted batches (host side), then
 * frees everything; NULL is a no-op. */
typedef struct ebsd_pipeline ebsd_pipeline;
int ebsd_pipeline_create(const ebsd_params* p, int device, int32_t depth, ebsd_pipeline** out);
int ebsd_pipeline_handle(ebsd_pipeline* pl, int32_t slot, ebsd_handle** h);
int ebsd_pipeline_submit(ebsd_pipeline* pl, const ebsd_pair* pairs, int32_t n, const ebsd_outputs* out,
                         void* stream);
int ebsd_pipeline_wait(ebsd_pipeline* pl, void* stream);
int ebsd_pipeline_destroy(ebsd_pipeline* pl);

/* Second pass only (section 2, Eq. (12)): remap each reference by the
 * caller's R_finite (device, [n][9] fp64, row-major), ROI XCF against the
 * test, F_inf by Eq. (3), F = F_inf R_finite, det F = 1, R, rotation vector.
 * Fills F, R, rotvec, q2, peak_height, status (and copies R_finite) of out. */
int ebsd_second_pass_batch(ebsd_handle* h, const ebsd_pair* pairs, int32_t n,
                           const double* R_finite, const ebsd_outputs* out, void* stream);

/* Autotuner for the demons kernel: on this batch (same validation as
 * ebsd_register_batch), times every supported strip height (rows per
 * workgroup: 16, 32, 64, 128) of the row-marching demons kernel for each
 * pyramid level (wider than 512 px: column segments, and also the 2-D tile
 * kernel as strip height 0), and keeps the fastest per level size for
 * later calls of this handle whose size bucket holds at least a quarter as
 * many pairs as the tuned batch (smaller batches use the default rule of
 * ebsd_get_strip_height).  If the environment variable EBSD_TUNE_CACHE
 * named a file when the handle was created, the table is read from it then
 * and written back here (lines "gfx950 <h> <w> <rows> <two-iteration rows>",
 * through a temporary file renamed over the cache, so a reader never sees a
 * partial table).  Synchronises
 * `stream`.  Demons results are unaffected (the strip height only changes the
 * work decomposition). */
int ebsd_autotune(ebsd_handle* h, const ebsd_pair* pairs, int32_t n, void* stream);

/* Graph replay (default on): the demons iterations of each pyramid level
 * (one launch per iteration) form a static sequence for a given batch
 * configuration (pair size, batch size, distinct references, parameters,
 * strip height); it is captured once into a HIP graph and replayed on later
 * calls, the per-call pointers travelling in a descriptor copied before the
 * replay.  enable = 0 makes later calls launch every kernel directly.
 * Results are identical either way. */
int ebsd_set_graphs(ebsd_handle* h, int enable);

/* Demons levels of at most 64 x 64 pixels of a size bucket of at most 256
 * pairs run in one launch per level (default, enable = 1): one workgroup per
 * pair keeps the level's reference, test and field in LDS and iterates to the
 * cap or to its own tolerance (multi-resolution demons, section 1).  Larger
 * buckets, and enable = 0, run them like the finer levels, one or two
 * iterations per launch.  The fields are bit-identical either way; the squared
 * update is summed in another order, so a stop on the tolerance can differ
 * only when the RMS update lies within rounding of it. */
int ebsd_set_resident(ebsd_handle* h, int enable);

/* Per-pair convergence across launches (multi-resolution demons, section 1,
 * run to a tolerance per pair).  Every demons launch skips the pairs that
 * have stopped, but a level's launches up to the cap would still be issued.
 * With a tolerance (tol_px > 0) and chunk_launches > 0 (default 8), a
 * level's launches are issued in chunks of chunk_launches; after each chunk
 * a one-workgroup kernel writes the number of pairs still iterating into
 * pinned host memory.  With chunks c - 1 and c queued behind it, the host
 * waits for chunk c - 2's count and issues no further chunk once it is
 * zero, so a level ends within two chunks of its last pair's stop and the
 * device never waits for the host.  The call then
 * returns only after the gated levels have been issued (the host thread
 * waits on the stream between chunks); a stream being captured by the
 * caller is never gated.  chunk_launches = 0 issues every launch and never
 * waits.  Results are identical either way (a skipped launch would have
 * exited at once for every pair).  EBSD_EINVAL for a negative value. */
int ebsd_set_gating(ebsd_handle* h, int32_t chunk_launches);

/* Demons launches of the last registration call per pyramid level, summed
 * over its size buckets (host arrays of EBSD_MAX_LEVELS, either may be NULL):
 * issued[l] were issued, planned[l] is the full sequence to the cap (one or
 * two iterations per launch).  Levels run level-resident count neither. */
int ebsd_get_launch_counts(const ebsd_handle* h, int32_t* issued, int32_t* planned);

/* Strip height used for a pyramid level of level_h x level_w px (levels
 * wider than 512 px run in column segments of 256 or 512 lanes, each
 * recomputing 9 columns on either side, or, at strip height 0, on the 2-D
 * tile kernel when the autotuner found that faster): the tuned or forced
 * value, else 64.  Untuned levels of a batch with fewer than 512
 * strips of 64 rows use 32 or 16 rows (more workgroups for small batches). */
int ebsd_get_strip_height(const ebsd_handle* h, int32_t level_h, int32_t level_w);

/* Force the strip height (16, 32, 64 or 128; 0 = the 2-D tile kernel, for
 * levels wider than 512 px only) for a level size. */
int ebsd_set_strip_height(ebsd_handle* h, int32_t level_h, int32_t level_w, int32_t rows);

/* Two demons iterations per launch (temporal blocking): the row-marching
 * kernel can run iteration k + 1 on the rows of iteration k while they are
 * still on chip, reading the field once and writing it once per two
 * iterations.  The second iteration of a launch runs before the stop
 * decision on the first is known; the next launch takes the decisions in
 * iteration order and recomputes the field of a pair that should have
 * stopped in between, so iteration counts, status and fields are identical to
 * one iteration per launch.  ebsd_autotune times strip heights 8 (levels at
 * most 128 px wide), 16, 32, 64, 128 of this kernel against the
 * single-iteration kernel and keeps it for a level size where it is faster.
 * ebsd_get_fused_height returns the strip height used for a level size (0 =
 * one iteration per launch); ebsd_set_fused_height forces it (0, 16, 32, 64 or
 * 128, or 8 for levels at most 128 px wide; EBSD_EINVAL otherwise). */
int ebsd_get_fused_height(const ebsd_handle* h, int32_t level_h, int32_t level_w);
int ebsd_set_fused_height(ebsd_handle* h, int32_t level_h, int32_t level_w, int32_t rows);

/* Timing of the demons iterations, for measurement tools.  enable != 0 makes
 * later calls record HIP events on their stream around each pyramid level's
 * demons launches and around the whole call (of its last size bucket). */
int ebsd_set_timing(ebsd_handle* h, int enable);

/* Waits for the last timed call to complete and reports level_ms[l] (host,
 * [levels]): the time of level l's demons launches (left unwritten with the
 * XCF first pass, which runs none), and *total_ms: the whole call.
 * EBSD_EINVAL if no timed call has been made. */
int ebsd_get_timing(ebsd_handle* h, double* level_ms, double* total_ms);

/* ---- warm-start network ------------------------------------------------------
 *
 * The demons iteration of section 1 starts from zero on the coarsest level.
 * The warm start replaces that zero by the field a convolutional network
 * predicts from the pair: a 4-level encoder (two 3 x 3 convolutions with ReLU
 * per level, 32/64/128/256 channels at 256/128/64/32 px, 2 x 2 max pooling
 * between levels) and a decoder at 64 x 64 px (nearest 2x upsampling of the
 * 32 px features, concatenation with the 64 px encoder features, two 3 x 3
 * convolutions of 128 channels with ReLU, a 1 x 1 convolution to 2 channels).
 * Its output is the displacement field (x, y) at the coarse grid points, whose
 * full-resolution coordinates are 4 i + 1.5, in full-resolution px.  Inputs
 * are the z-scored reference and test patterns (256 x 256).
 *
 * Arithmetic: bf16 operands on the matrix cores with fp32 accumulation;
 * activations are stored as bf16 (round to nearest even); biases, the 1 x 1
 * head, the loss and the optimiser are fp32.  Training minimises the mean
 * squared endpoint error against a label field with Adam (fp32 master
 * parameters).
 *
 * Parameters: a flat fp32 vector of EBSD_CNN_PARAMS values; for each 3 x 3
 * convolution in the order c1a, c1b, c2a, c2b, c3a, c3b, c4a, c4b, d1, d2 its
 * weights [3][3][cin][cout] then its bias [cout]; then the head weights
 * [128][2] and bias [2].  Files written by ebsd_cnn_save hold the 8 bytes
 * "EBSDCNN1", an int64 count and the vector (little-endian).
 *
 * Patterns of 512 x 512 reach the network as their pyramid level 1, patterns
 * of 128 x 128 as their level 0 upsampled x2 (bilinear); the fit below works
 * in the 256 x 256 frame (Eq. (2) is unchanged by a common scaling of the
 * detector coordinates), and the starting field is evaluated on, or resampled
 * to, the pattern's own coarse grid.
 *
 * Fallback rule (warm start inside ebsd_register_batch): the Eq. (2) model is
 * fitted (Eq. (3): direct linear start, Gauss-Newton, det F = 1) to the
 * predicted field at the grid points within roi_radius_frac * W of the
 * pattern centre; if the RMS endpoint misfit, in full-resolution px of the
 * registered pattern (the 256-px frame's misfit times N / 256 for an N-px
 * pattern), exceeds fallback_residual_px the pair
 * starts from zero (EBSD_WARM_FALLBACK), otherwise (EBSD_WARM_USED) from
 * the predicted field (warm_start = 1) or from the field of the fitted model
 * (warm_start = 2: the network's estimate projected onto Eq. (2)).
 */
#define EBSD_CNN_PARAMS 1762306

typedef struct ebsd_cnn ebsd_cnn;

/* EBSD_CNN_PARAMS. */
int64_t ebsd_cnn_num_params(void);

/* Network on HIP device `device`, for batches of at most max_batch pairs
 * (1..4096; device buffers of about 45 MB per pair are allocated here).
 * Parameters start at zero; set or load them before use. */
int ebsd_cnn_create(int device, int32_t max_batch, ebsd_cnn** out);
int ebsd_cnn_destroy(ebsd_cnn* c);

/* Copy the flat fp32 parameter vector from / to HOST memory (n must equal
 * EBSD_CNN_PARAMS).  Setting parameters also resets the optimiser state. */
int ebsd_cnn_set_params(ebsd_cnn* c, const float* host, int64_t n);
int ebsd_cnn_get_params(const ebsd_cnn* c, float* host, int64_t n);
/* Gradients of the last ebsd_cnn_train_step, same layout, HOST memory. */
int ebsd_cnn_get_grads(const ebsd_cnn* c, float* host, int64_t n);

/* Parameter files (format above).  EBSD_EIO on a read/write failure or a
 * malformed file. */
int ebsd_cnn_load(ebsd_cnn* c, const char* path);
int ebsd_cnn_save(const ebsd_cnn* c, const char* path);

/* Forward pass for n pairs: ref, test device [n][H][W] fp32 raw patterns,
 * z-scored here; out device [n][H/4][W/4][2] fp32 (x, y) full-res px.
 * n <= max_batch.  The warm start uses H = W = 256; other sizes with H a
 * multiple of 64, W a multiple of 256 and H * W <= 65536 are accepted
 * (EBSD_ESHAPE otherwise). */
int ebsd_cnn_forward(ebsd_cnn* c, const float* ref, const float* test, int32_t n, int32_t H,
                     int32_t W, float* out, void* stream);

/* One training step on n pairs (sizes as for ebsd_cnn_forward): forward,
 * loss against label (device [n][H/4][W/4][2] fp32), backward and, if
 * update != 0, one Adam step with
 * learning rate lr (beta1 0.9, beta2 0.999, eps 1e-8).  *loss (HOST) receives
 * the mean squared endpoint error before the update; the call synchronises
 * `stream`. */
int ebsd_cnn_train_step(ebsd_cnn* c, const float* ref, const float* test, const float* label,
                        int32_t n, int32_t H, int32_t W, float lr, int32_t update, float* loss,
                        void* stream);

/* Kernels of the inference forward pass (ebsd_cnn_forward and the warm
 * start): on = 1 (the default) runs fused kernels (the first block's two
 * convolutions and pooling in one pass, activations kept on chip); on = 0
 * runs one kernel per layer, as the training step does.  Both give the same
 * output bit for bit; the switch exists to measure and test the fusion.
 * EBSD_EINVAL unless on is 0 or 1. */
int ebsd_cnn_set_fusion(ebsd_cnn* c, int32_t on);

/* Restart Adam (moments zero, step count 0). */
int ebsd_cnn_reset_optimizer(ebsd_cnn* c);

/* Adam's state, for checkpointing a training run: first and second moments
 * (HOST, n = ebsd_cnn_num_params() floats each, parameter layout) and the
 * step count that sets the bias corrections.  get: any of m, v, step may be
 * NULL (zero moments before the first training step); set: m and v are
 * required, step >= 0.  EBSD_EINVAL for a wrong n or a negative step. */
int ebsd_cnn_get_optimizer(const ebsd_cnn* c, float* m, float* v, int64_t n, int64_t* step);
int ebsd_cnn_set_optimizer(ebsd_cnn* c, const float* m, const float* v, int64_t n, int64_t step);

/* Parameters used by the warm start of a registration handle: from a file
 * (ebsd_load_model) or copied from a network object (ebsd_set_model). */
int ebsd_load_model(ebsd_handle* h, const char* path);
int ebsd_set_model(ebsd_handle* h, const ebsd_cnn* c);

/* ---- single-stage entry points (one kernel each; device pointers) ------- */

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, hosts that forbid allocation): the same
 * pre-filter as ebsd_stage_bandpass, bit for bit, with its row pass (2 n H W
 * floats) in a fixed device buffer of 8 Mi floats (32 MiB) that the library
 * holds on each device it runs on until the process ends, instead of a
 * temporary.  It calls no allocator and does not wait on the stream.
 * EBSD_ETOOBIG when 2 n H W exceeds 8 Mi floats (e.g. at most 64 patterns of
 * 256 x 256 or 3 of 1244 x 1024 per call); other errors as ebsd_stage_bandpass.
 * Every call on one device shares that buffer: calls that may overlap on one
 * device (other streams, other threads) race and must be ordered by the
 * caller. */
int ebsd_stage_bandpass_static(const float* in, int32_t n, int32_t H, int32_t W, float lo_px, float hi_px,
                               float* out, void* stream);

/* z-score each of n contiguous patterns of `elems` fp32 values:
 * out = (in - mean) / std (population std, FP64 statistics).  flags (device,
 * [n] uint32, may be NULL) receive EBSD_DEGENERATE_INPUT / EBSD_NONFINITE_INPUT;
 * such patterns are written as zeros. */
int ebsd_stage_normalize(const float* in, int32_t n, int64_t elems, float* out, uint32_t* flags,
                         void* stream);

/* The pre-filter of ebsd_params (bandpass_lo_px, bandpass_hi_px) on n raw
 * images in [n][H][W] -> out [n][H][W] (device fp32; 2 <= W <= 16384,
 * H <= 65535, n <= 65535; both sigmas in [0, 32]).  Allocates a temporary
 * of 2 n H W floats. */
int ebsd_stage_bandpass(const float* in, int32_t n, int32_t H, int32_t W, float lo_px, float hi_px, float* out,
                        void* stream);

/* Factor-2 restriction of n images [n][H][W] -> [n][ceil(H/2)][ceil(W/2)]
 * with the separable [1,3,3,1]/8 filter, clamped borders (H, W >= 2; an odd
 * size's last output reads the border through the clamp). */
int ebsd_stage_restrict(const float* in, int32_t n, int32_t H, int32_t W, float* out, void* stream);

/* One demons iteration (Eq. (1) force with the reference gradient, then
 * Gaussian smoothing of the accumulated field with sigma_px) for n image
 * pairs at one level: R, T [n][H][W] (normalised), u_in, u_out [n][2][H][W]
 * in px of this level (u_in != u_out).  rms (device, [n] fp64, may be NULL)
 * receives RMS|u_out - u_in| per pair. */
int ebsd_stage_demons_iter(const float* R, const float* T, int32_t n, int32_t H, int32_t W,
                           const float* u_in, float sigma_px, float* u_out, double* rms,
                           void* stream);

/* Field prolongation [n][2][h][w] -> [n][2][2h][2w]: bilinear with the
 * half-pixel-centre map, values doubled.  EBSD_ESHAPE unless 1 <= h, w <= 8192
 * (outputs of at most 16384 px a side) and n <= 65535. */
int ebsd_stage_prolong(const float* u, int32_t n, int32_t h, int32_t w, float* out, void* stream);

/* ROI cross-correlation of n ROI pairs (section 2): A (reference) and B
 * (test), [n][N][N] fp32, N in {32, 64, 128, 256}; per-ROI zero mean, optional
 * Hann window, C = IFFT(FFT(B w) conj FFT(A w)), integer peak (ties to the
 * lowest row-major index), 2-D quadratic sub-pixel fit.  q: [n][2] (x, y)
 * shift of B relative to A; ph: [n] normalised peak height (may be NULL).
 * N = 256 (the paper's ROI size) allocates a device temporary of 768 KiB per
 * ROI in flight (at most 512 ROIs: 384 MiB) and waits on the stream before
 * it returns; smaller N run in LDS and never wait. */
int ebsd_stage_xcf(const float* A, const float* B, int32_t n, int32_t N, int32_t window, float* q,
                   float* ph, void* stream);

/* Remap of n images (section 2, before Eq. (12)): out(x') = img(pi(R^T
 * r(x'))) with r(x) = (x - xs, y - ys, zs), pi(v) = (xs + zs v_x / v_z,
 * ys + zs v_y / v_z), the sample position clamped to the image.  img, out:
 * [n][H][W] fp32 (device); R: [n][9] fp64 row-major (device); pattern centre
 * (xs, ys) and detector distance zs in px.  interp 3: cubic B-spline
 * interpolation (whole-sample mirror extension); coef (device, [n][H][W]
 * fp32, required) receives the B-spline coefficients of each image.  interp
 * 1: bilinear; coef is not used (may be NULL).  H, W >= 3, n <= 65535. */
int ebsd_stage_remap(const float* img, int32_t n, int32_t H, int32_t W, const double* R, double xs,
                     double ys, double zs, int32_t interp, float* coef, float* out, void* stream);

/* Eq. (13)'s detector-to-sample rotation R_tilt for a tilt of theta rad, as
 * printed (a rotation about z): S = [[cos, sin, 0], [-sin, cos, 0], [0, 0, 1]],
 * written to S (HOST, 9 fp64, row-major).  EBSD_EINVAL for a NULL S or a
 * theta that is not finite. */
int ebsd_tilt_rotation(double theta, double* S);

/* Eq. (3) under the traction-free equality constraint, with the strain and
 * stress it implies (section 2; Eq. (13)-(16); supplementary Eq. (2.1)-(2.11)).
 * For each of n shift sets q [n][n_roi][2] (fp32, device) at the ROI centres
 * cx, cy ([n_roi] fp64, device), pattern centre (xs, ys) and detector
 * distance zs in px: F_inf minimises the Eq. (3) objective subject to zero
 * traction on the sample surface, sigma_S33 = sigma_S23 = sigma_S13 = 0, for
 * the total F = F_inf M (detector frame), where
 *   F_S = S F S^T                   (Eq. (14); S: detector-to-sample rotation,
 *                                    HOST, 9 fp64 row-major, e.g. Eq. (13)'s
 *                                    R_tilt),
 *   eps_S = (F_S F_S^T - I) / 2     (Eq. (15), its first form: free of the
 *                                    rotation in F),
 *   sigma_S = g^T (C : (g eps_S g^T)) g  (Eq. (16) with the stiffness taken
 *                                    to the sample frame, supplementary
 *                                    Eq. (2.4)-(2.11); C cubic with C11, C12,
 *                                    C44 in any stress unit; g [n][9] fp64,
 *                                    device: the passive orientation taking
 *                                    sample to crystal coordinates, Eq. (2.1)).
 * The shifts fix F_inf up to scale; the constraint fixes the scale (and two
 * more directions).  M [n][9] (device) is what the fit composes with:
 * R_finite for the shifts q2 of a single second pass, NULL (identity) for a
 * first-pass fit (q1).  Outputs (device): F [n][9] the total F, eps_S and
 * sigma_S [n][9] (may be NULL), status [n] (may be NULL; SOLVE_ILLCOND when
 * a step fails or the steps do not converge).  EBSD_EINVAL for NULL inputs,
 * n_roi outside 5..256, zs <= 0, an S that is not a rotation, or a stiffness
 * that is not positive definite (C44 > 0, C11 > C12, C11 + 2 C12 > 0). */
int ebsd_traction_free(const float* q, int32_t n, int32_t n_roi, const double* cx, const double* cy,
                       double xs, double ys, double zs, const double* M, const double* g, const double* S,
                       double C11, double C12, double C44, double* F, double* eps_S, double* sigma_S,
                       uint32_t* status, void* stream);

/* Eq. (3) solve for n shift sets: q [n][n_roi][2] fp32 at ROI centres
 * cx, cy (device, [n_roi] fp64), pattern centre (xs, ys, zs) in px.
 * Writes F [n][9] (det 1) and, if R != NULL, R = polar(F) [n][9] (fp64);
 * status [n] may be NULL. */
int ebsd_stage_solve(const float* q, int32_t n, int32_t n_roi, const double* cx, const double* cy,
                     double xs, double ys, double zs, double* F, double* R, uint32_t* status,
                     void* stream);

/* ---- synthetic pattern pairs ---------------------------------------------------
 *
 * Training and benchmark inputs with ground truth.  A pattern is the gnomonic
 * view (pattern centre and Z* as above) of the 25 FCC plane normals of
 * {111}, {200}, {220}, {311}: a band profile (1 + cos(pi phi / theta_B)) / 2
 * for |phi| <= theta_B, theta_B = asin((lambda / 2a) |hkl|), lambda / a =
 * 0.02438, plus the background 1 + 0.2 (gx (x/(W-1) - 1/2) + gy (y/(H-1) -
 * 1/2)); I = background + 0.5 sum(profiles).  The test pattern is rendered
 * by pull-back through F^-1, so its exact shift field is q(x) = pi(F r(x)) - x
 * (the projective model of Eq. (2)).  Each pattern is scaled to a mean of
 * `counts` and, if noise != 0, replaced by Poisson draws: the uniforms of
 * pixel p of stream s (0 reference, 1 test) come from Philox4x32-10 with
 * counter (p, attempt, s, 0) and key (key[0], key[1]); the sampler is PTRS
 * (transformed rejection with squeeze) for means >= 10, inversion below.
 * Rendering is FP64, outputs fp32. */
typedef struct ebsd_gen_spec {
    double G[9];      /* crystal -> detector orientation of the reference, row-major */
    double F[9];      /* applied deformation gradient (detector frame), row-major */
    double gx, gy;    /* background gradient coefficients */
    double counts;    /* mean count of each pattern (<= 0: unscaled) */
    uint32_t key[2];  /* noise key */
    int32_t noise;    /* 1 = Poisson noise */
    int32_t bands;    /* 1 = the FCC bands, 0 = background only */
} ebsd_gen_spec;

/* n pairs of H x W: ref, test device [n][H][W] fp32; label (device, may be
 * NULL; needs H % 4 == 0 and W % 4 == 0) [n][H/4][W/4][2] fp32, the shift
 * field (x, y) at the coarse grid points 4 i + 1.5 (full-res px).  specs is
 * a HOST array.  EBSD_EINVAL for a singular F or non-finite values.
 * Allocates temporaries and synchronises `stream`. */
int ebsd_gen_pairs(const ebsd_gen_spec* specs, int32_t n, int32_t H, int32_t W, double pc_x, double pc_y,
                   double pc_z, float* ref, float* test, float* label, void* stream);

/* ---- single-kernel entry points of the warm-start network -------------------
 * bf16 tensors are uint16_t bit patterns (the upper half of an IEEE float),
 * NHWC.  Weights are fp32 [3][3][Cin][Cout] (rounded to bf16 here).  Shapes:
 * H % 8 == 0, W % 32 == 0, Cin % 32 == 0 or Cin == 8, Cout % 32 == 0, Cin and
 * Cout <= 512 (EBSD_ESHAPE otherwise).  These calls allocate a temporary
 * device buffer and synchronise `stream`; they exist to check the kernels
 * one at a time. */

/* 3 x 3 convolution with zero padding 1 of x [n][H][W][Cin]: mode 0 writes
 * bf16 max(conv + bias, 0) to out [n][H][W][Cout] (uint16_t); mode 1 writes
 * the fp32 convolution (bias unused). */
int ebsd_stage_conv3x3(const uint16_t* x, int32_t n, int32_t H, int32_t W, int32_t Cin, const float* w,
                       const float* bias, int32_t Cout, int32_t mode, void* out, void* stream);

/* Input gradient of that convolution: dx [n][H][W][Cin] fp32 from the output
 * gradient dz [n][H][W][Cout] (bf16) and w [3][3][Cin][Cout]. */
int ebsd_stage_conv3x3_dgrad(const uint16_t* dz, int32_t n, int32_t H, int32_t W, int32_t Cout,
                             const float* w, int32_t Cin, float* dx, void* stream);

/* Weight gradient dw [3][3][Cin][Cout] fp32 = sum over pixels of
 * x[p + tap offset][ci] dz[p][co] (x, dz bf16); also needs H % 4 == 0. */
int ebsd_stage_conv3x3_wgrad(const uint16_t* x, const uint16_t* dz, int32_t n, int32_t H, int32_t W,
                             int32_t Cin, int32_t Cout, float* dw, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* EBSD_H */
