// Internal declarations of the gfx950 demons/XCF library: per-bucket device
// descriptors and the host launchers that each kernel file exports.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <mutex>
#include <shared_mutex>

namespace ebsd {

// Stream capture in one host thread and a call that waits for the whole device
// in another (hipDeviceSynchronize, and the frees and pinned allocations that
// synchronise implicitly) must not overlap: the wait would take in the stream
// being captured, which fails the call or invalidates the capture.  Several
// handles run in their own threads in a pipeline, so captures hold this lock
// shared and every device-wide wait or (de)allocation of the library holds it
// exclusively.
inline std::shared_mutex& capture_mutex()
{
    static std::shared_mutex m;
    return m;
}
using DeviceWideLock = std::unique_lock<std::shared_mutex>;

// Raises a kernel's dynamic LDS limit on the current device, once per device:
// a host-side function attribute (not a stream operation).  `done` holds one
// bit per device ordinal below 64 and may be shared by concurrent callers.
inline hipError_t ensure_dynamic_lds(const void* fn, int bytes, std::atomic<uint64_t>& done)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const uint64_t bit = (dev >= 0 && dev < 64) ? (uint64_t{1} << dev) : 0;
    if (bit && (done.load(std::memory_order_acquire) & bit)) return hipSuccess;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess && bit) done.fetch_or(bit, std::memory_order_acq_rel);
    return e;
}

constexpr int kMaxLevels = 8;
constexpr int kMaxPipelineDepth = 8;  // handles (streams) of one ebsd_pipeline
constexpr int kMaxRadius = 4;     // Gaussian half-width supported by the demons kernel
constexpr int kDemonsTX = 64;     // demons output tile: 64 columns (one wavefront per row)
constexpr int kDemonsTY = 16;     // ... x 16 rows
constexpr int kDemonsThreads = 256;

// Normalised Gaussian taps w[0..2r] for offsets -r..r.
struct Taps {
    float w[2 * kMaxRadius + 1];
};

// Per-pattern statistics from the normalisation pass.
struct PatStat {
    double mean;
    double inv_std;
    uint32_t flags;  // EBSD_DEGENERATE_INPUT / EBSD_NONFINITE_INPUT
    uint32_t pad;
};

// Per-pair demons state (one entry per pair of a bucket).  No kernel
// synchronises across workgroups: within a level, iteration k reads the field
// from buffer (base + k) & 1, and every workgroup of a pair derives the stop
// decision for iteration k from the per-tile sums of iteration k - 1 itself.
struct PairState {
    int32_t base;       // buffer holding the field at iteration 0 of the current level
    int32_t stop;       // -1 while iterating, else the iteration count at which it stopped
    int32_t cur;        // buffer holding the pair's field after the level ended
    uint32_t convmask;  // bit l set when level l stopped on the tolerance
};

// Caller output pointers (any may be NULL), indexed by the caller's pair index.
struct OutPtrs {
    double* F;
    double* R;
    double* rotvec;
    double* Rfin;
    double* F1;
    float* q1;
    float* q2;
    float* ph;
    int32_t* iters;
    uint32_t* status;
    float* warm_field;   // [n][h][w][2] network field (warm start)
    float* warm_misfit;  // [n]
    double* mae1;        // [n] mean angular error of the first fit
    double* mae;         // [n] mean angular error of the last fit
    double* ssim;        // [n] structural similarity of the registration
    double* omega;       // [n][9] Eq. (6)'s rotation tensor of rotvec
};
// Everything a bucket's kernels need, in device memory (one copy per bucket).
struct Bucket {
    int32_t nb;                 // pairs in the bucket
    int32_t nref;               // distinct reference patterns
    int32_t H, W, L;            // finest size and number of levels
    int32_t lvl_off[kMaxLevels];// float offset of level l inside one pyramid (multiple of 64)
    int32_t lh[kMaxLevels];     // level sizes: lh[0] = H, lh[l] = ceil(lh[l-1] / 2)
    int32_t lw[kMaxLevels];     // lw[0] = W, lw[l] = ceil(lw[l-1] / 2)
    int64_t pyr_elems;          // floats per pyramid (all levels)
    const float* const* test_in;// [nb] caller test patterns
    const float* const* ref_in; // [nref] caller reference patterns
    const int32_t* ref_slot;    // [nb] reference slot of each pair
    const int32_t* pair_index;  // [nb] index of the pair in the caller's arrays
    float* test_pyr;            // [nb][pyr_elems]
    float* ref_pyr;             // [nref][pyr_elems]
    PatStat* test_stat;         // [nb]
    PatStat* ref_stat;          // [nref]
    float* field[2];            // [nb][2][H][W] each (level l uses the leading 2 h w)
    PairState* state;           // [nb]
    float* partial;             // [4][nb][max tiles] per-tile sums of squared updates (slot k & 1 for one
                                // iteration per launch, k & 3 for two)
    int32_t max_tiles;          // tiles of the finest level
    int32_t* iters;             // [nb][L]
    int32_t n_roi, roi_N;
    const double* roi_c;        // [n_roi][2] ROI centres (x, y)
    const int32_t* roi_xy;      // [n_roi][2] ROI top-left (x0, y0)
    double xs, ys, zs;          // pattern centre and detector distance, px
    float* q1;                  // [nb][n_roi][2]
    float* q2;                  // [nb][n_roi][2]
    float* ph;                  // [nb][n_roi]
    double* F1;                 // [nb][9]
    double* Rfin;               // [nb][9]
    double* F;                  // [nb][9]
    double* R;                  // [nb][9]
    double* rotvec;             // [nb][3]
    uint32_t* status;           // [nb]
    double* mae1;               // [nb] mean angular error of the first fit (F1 to q1), rad
    double* mae;                // [nb] mean angular error of the last fit, rad
    int32_t prefilter;          // 1: level 0 holds the pre-filtered patterns before normalisation
    double* ssim;               // [nb] structural similarity of the registration (NULL: not computed)
    double* ssim_part;          // [nb][ssim tiles] per-tile sums
    float* ref_coef;            // [nref][H][W] cubic B-spline coefficients of level 0 (NULL: bilinear remap)
    float* coef_tmp;            // [nref][H][W] row pass of the coefficients
    float* xcf_scratch;         // ROIs of 256: xcf_scratch_floats(256, nb n_roi) floats (else NULL)
    // per-call caller pointers (so that a bucket's launch sequence is static
    // and can be replayed from a captured graph)
    OutPtrs out;                // results, scattered by pair_index
    const float* u_init;        // [nb][2][h][w] coarsest initial field or NULL
    float* const* field_dst;    // [nb] destination of each final field or NULL
    const double* rfin_in;      // [caller n][9] R_finite for the second-pass-only entry
    // warm start (NULL when off): network field [nb][h][w][2], fit misfit [nb],
    // status bit (EBSD_WARM_USED / EBSD_WARM_FALLBACK) [nb]
    const float* warm_field;
    const float* warm_misfit;
    const uint32_t* warm_flag;
};

// ---- launchers (defined next to their kernels) -------------------------------

// Normalisation statistics for nb test patterns and nref reference patterns.
hipError_t launch_stats(const Bucket* d_bk, int nb, int nref, hipStream_t s);
// Normalise level 0 of every pyramid and build levels 1..L-1.
hipError_t launch_pyramids(const Bucket* d_bk, const Bucket& hb, hipStream_t s);
// Reset per-pair state and set the coarsest-level initial field
// (bk->u_init [nb][2][h][w] in full-res px, or zero).
hipError_t launch_demons_init(const Bucket* d_bk, const Bucket& hb, hipStream_t s);
// Iteration k (0-based) of level l for every pair that has not stopped; ty =
// strip height of the row-marching kernel.
hipError_t launch_demons_iter(const Bucket* d_bk, const Bucket& hb, int level, int k,
                              const float* taps, int radius, float tol, int ty, hipStream_t s);
// Launch L of level l run two iterations at a time (strip height ty of the
// fused row-marching kernel; cap = the level's iteration cap).
hipError_t launch_demons_iter2(const Bucket* d_bk, const Bucket& hb, int level, int L, const float* taps,
                               int radius, float tol, int cap, int ty, hipStream_t s);
// A whole level of at most 64 x 64 pixels in one launch, one workgroup per
// pair iterating in LDS to the cap or the tolerance; leaves the final field,
// the iteration count and the pair state as launch_level_end does.
bool demons_resident_ok(int h, int w);
hipError_t launch_demons_resident(const Bucket* d_bk, const Bucket& hb, int level, const float* taps, int radius,
                                  float tol, int cap, hipStream_t s);
// *out = number of pairs whose demons state has not recorded a stop (out may
// be pinned host memory mapped into the device's address space).
hipError_t launch_count_active(const Bucket* d_bk, int32_t* out, hipStream_t s);
// Close level l: iteration counts, convergence of the last iteration, final buffer.
hipError_t launch_level_end(const Bucket* d_bk, const Bucket& hb, int level, int cap, float tol,
                            int ty, bool fused, hipStream_t s);
// Prolong the field of every pair from level l to level l-1 and re-arm the pairs.
hipError_t launch_prolong_level(const Bucket* d_bk, const Bucket& hb, int level, hipStream_t s);
// Sample the finest field at the ROI centres -> q1.
hipError_t launch_sample_q1(const Bucket* d_bk, const Bucket& hb, hipStream_t s);
// Copy the finest field to the caller (bk->field_dst[i] = destination of pair i or NULL).
hipError_t launch_copy_field(const Bucket* d_bk, const Bucket& hb, hipStream_t s);
// First-pass solve: F1 from q1 (Eq. (3)), Rfin = polar(F1), mae1; status
// from the input flags and, when tol > 0, the per-level convergence.
hipError_t launch_solve_first(const Bucket* d_bk, const Bucket& hb, float tol, hipStream_t s);
// Status from the input flags only (second-pass-only entry).
hipError_t launch_status_inputs(const Bucket* d_bk, const Bucket& hb, hipStream_t s);
// Cubic B-spline coefficients of level 0 of every reference -> bk->ref_coef.
hipError_t launch_bspline_coef(const Bucket* d_bk, const Bucket& hb, hipStream_t s);
// Remap + ROI XCF for every (pair, ROI) -> q2, ph.  interp 3: cubic B-spline
// from bk->ref_coef, 1: bilinear; pass 0 remaps by Rfin, pass k > 0 by F.
hipError_t launch_xcf_pairs(const Bucket* d_bk, const Bucket& hb, int window, int interp, int pass,
                            hipStream_t s);
// The conventional first pass: ROI XCF of the unremapped level-0 patterns ->
// q1, ph.
hipError_t launch_xcf_first(const Bucket* d_bk, const Bucket& hb, int window, hipStream_t s);
// Pre-filter (Gaussian low-pass minus Gaussian background) of raw patterns.
// Pattern p reads src + p src_stride (src != NULL) or src_a[p] (p < na) /
// src_b[p - na], and writes dst_a + p dst_stride (p < na) or dst_b + (p - na)
// dst_stride; tmp holds 2 x npat x H x W floats.  Taps: r < 0 turns a filter off.
constexpr int kBandMaxR = 96;
struct BandTaps {
    float lo[2 * kBandMaxR + 1];
    float hi[2 * kBandMaxR + 1];
    int rlo, rhi;
};
struct BandIO {
    const float* const* src_a;
    const float* const* src_b;
    const float* src;
    int64_t src_stride;
    // src == NULL and src_a == NULL: pattern p reads srcb_a + p srcb_stride (p < na)
    // or srcb_b + (p - na) srcb_stride (in place over a pyramid's level 0, say)
    const float* srcb_a;
    const float* srcb_b;
    int64_t srcb_stride;
    float* dst_a;
    float* dst_b;
    int64_t dst_stride;
    int na, npat, H, W;
    float* tmp;
};
BandTaps make_band_taps(double lo, double hi);
hipError_t launch_bandpass(const BandIO& io, const BandTaps& tp, hipStream_t s);
// Background correction: bg [H][W] = pixelwise mean of the nb patterns src_a[0..nb)
// (the static background); dst(p) = src(p) / bg (bg == NULL: a copy); dst(p) /=
// blur + p H W (the dynamic step, in place).  A non-positive divisor gives 0.
hipError_t launch_mean_pattern(const float* const* src, int nb, int64_t hw, float* bg, hipStream_t s);
hipError_t launch_bg_static(const BandIO& io, const float* bg, hipStream_t s);
hipError_t launch_bg_dynamic(const BandIO& io, const float* blur, hipStream_t s);
// Structural similarity of the normalised reference and the test warped by the
// final field (11 x 11 Gaussian window, sigma 1.5; L = 6) -> bk->ssim, via
// per-tile sums in bk->ssim_part.
int ssim_tiles(int H, int W);
hipError_t launch_ssim(const Bucket* d_bk, const Bucket& hb, hipStream_t s);
// iters[b][l] = 0 for every pair and level (no demons iterations run).
hipError_t launch_zero_iters(const Bucket* d_bk, const Bucket& hb, hipStream_t s);
// Rfin[b] = bk->rfin_in[pair_index[b]] (second-pass-only entry).
hipError_t launch_gather_rfin(const Bucket* d_bk, const Bucket& hb, hipStream_t s);
hipError_t launch_scatter(const Bucket* d_bk, const Bucket& hb, hipStream_t s);
// Copy the warm-start field and misfit of every pair to the caller's outputs.
hipError_t launch_scatter_warm(const Bucket* d_bk, const Bucket& hb, hipStream_t s);
// Second-pass solve: F_inf from q2, F = F_inf M, det 1, R = polar(F), rotvec,
// with M = Rfin for pass 0 and M = F (the previous pass's) after.
// second_pass == 0: F = F1.  mae: of the F_inf fit (of F1 without a second pass).
hipError_t launch_solve_second(const Bucket* d_bk, const Bucket& hb, int second_pass, int pass,
                               hipStream_t s);

// ---- stage launchers -----------------------------------------------------------
hipError_t launch_stage_normalize(const float* in, int n, int64_t elems, float* out,
                                  uint32_t* flags, hipStream_t s);
hipError_t launch_stage_restrict(const float* in, int n, int H, int W, float* out, hipStream_t s);
hipError_t launch_stage_demons_iter(const float* R, const float* T, int n, int H, int W,
                                    const float* u_in, const float* taps, int radius,
                                    float* u_out, double* rms, hipStream_t s);
hipError_t launch_stage_prolong(const float* u, int n, int h, int w, float* out, hipStream_t s);
// N in {32, 64, 128}: LDS-resident; N = 256: scratch holds xcf_scratch_floats(256, n) floats.
hipError_t launch_stage_xcf(const float* A, const float* B, int n, int N, int window, float* q,
                            float* ph, float* scratch, hipStream_t s);
// Global scratch the XCF of `rois` ROIs of N x N needs (0 below N = 256).
int64_t xcf_scratch_floats(int N, int64_t rois);
hipError_t launch_stage_remap(const float* ref, int n, int H, int W, const double* R, double xs, double ys,
                              double zs, int interp, float* coef, float* out, hipStream_t s);
hipError_t launch_stage_solve(const float* q, int n, int n_roi, const double* cx,
                              const double* cy, double xs, double ys, double zs, double* F,
                              double* R, uint32_t* status, hipStream_t s);
// Detector-to-sample rotation S (Eq. (13)-(14)) and the cubic stiffness of
// the crystal frame, for the traction-free solve.
struct TractionFrame {
    double S[9];
    double c11, c12, c44;
};
// Eq. (3) under the traction-free constraint for n shift sets; M [n][9]
// (NULL = identity), g [n][9]; F, eps, sig [n][9] (eps, sig may be NULL).
hipError_t launch_traction_free(const float* q, int n, int n_roi, const double* cx, const double* cy,
                                double xs, double ys, double zs, const double* M, const double* g,
                                const TractionFrame& tf, double* F, double* eps, double* sig,
                                uint32_t* status, hipStream_t s);

// Number of demons tiles of an h x w level (2-D tile kernel).
inline int demons_tiles(int h, int w)
{
    return ((w + kDemonsTX - 1) / kDemonsTX) * ((h + kDemonsTY - 1) / kDemonsTY);
}

// Row-marching kernel: wavefronts per row (0 = not applicable), supported
// strip heights, number of strips, and its launchers (false if not
// applicable).  Levels wider than 512 px run in column segments of 512
// lanes: each segment recomputes kSegHalo columns on either side (enough for
// two iterations of the widest smoothing) and writes the 512 - 2 kSegHalo
// columns between them.
int rows_cpl(int w);
constexpr int kSegHalo = 2 * kMaxRadius + 1;
__host__ __device__ inline int rows_segs(int w, int nw)
{
    const int lanes = 64 * nw, ww = lanes - 2 * kSegHalo;
    return w <= lanes ? 1 : (w + ww - 1) / ww;
}
// Columns of segment `seg`: lanes start at column sx0; columns [ws, we) are written.
__host__ __device__ inline void rows_seg_cols(int seg, int nsegs, int w, int nw, int& sx0, int& ws, int& we)
{
    if (nsegs == 1) {
        sx0 = 0;
        ws = 0;
        we = w;
        return;
    }
    const int ww = 64 * nw - 2 * kSegHalo;
    ws = seg * ww;
    we = ws + ww < w ? ws + ww : w;
    sx0 = ws - kSegHalo;
}
bool rows_ty_supported(int ty);
// Two iterations per launch (temporal blocking) at strip heights 16, 32, 64, 128 (and 8 on
// levels at most 128 px wide):
// launch L of a level runs iterations 2L and 2L + 1 (see k_demons_rows2);
// ceil(cap / 2) launches, plus one more when tol > 0 and cap is even.
bool rows2_ty_supported(int ty);
bool rows2_ty_ok(int w, int ty);  // ty supported for a level w px wide (8 only up to 128 px)
bool launch_demons_rows2(const Bucket* d_bk, const Bucket& hb, int level, int L, const Taps& tp, int radius,
                         float tol, int cap, int ty, hipStream_t s);
int rows_units(int h, int ty);
bool launch_demons_rows(const Bucket* d_bk, const Bucket& hb, int level, int k, const Taps& tp,
                        int radius, float tol, int ty, hipStream_t s);
bool launch_demons_rows_stage(const float* R, const float* T, int n, int h, int w, const float* u,
                              const Taps& tp, int radius, float* un, double* rms, hipStream_t s);

constexpr int kDefaultStripTY = 64;
constexpr int kMinStripTY = 16;
constexpr int kMinStripTY2 = 8;  // two-iteration kernel on rows of at most 128 px (latency of small batches)

// Work units (and per-pair partial sums) of one demons iteration at h x w
// with strip height ty (row-marching kernel: strips x column segments) or
// 2-D tiles (ty = 0, which levels wider than 512 px may select).
inline int demons_units(int h, int w, int ty)
{
    const int nw = rows_cpl(w);
    return nw && ty > 0 ? rows_units(h, ty) * rows_segs(w, nw) : demons_tiles(h, w);
}
// Strip heights a level accepts: the row kernel's, and 0 (2-D tiles) above 512 px.
inline bool strip_ty_ok(int w, int ty) { return rows_ty_supported(ty) || (ty == 0 && w > 512); }

}  // namespace ebsd
