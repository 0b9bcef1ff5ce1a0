// Row-marching demons kernels: choice of the row width (wavefronts per row)
// and of the strip heights; the kernels are in demons_rows_impl.h, instantiated
// per row width in k_demons_rows_w<NW>.hip.
#include "ebsd_internal.h"

namespace ebsd {

// one row width per translation unit
bool demons_rows_nw1(const Bucket* d_bk, int nb, int h, int w, int level, int k, const Taps& tp, int radius, float tol,
                      int ty, hipStream_t s);
bool demons_rows2_nw1(const Bucket* d_bk, int nb, int h, int w, int level, int L, const Taps& tp, int radius, float tol,
                       int cap, int ty, hipStream_t s);
bool demons_rows_stage_nw1(const float* R, const float* T, int n, int h, int w, const float* u, const Taps& tp,
                            int radius, float* un, double* rms, hipStream_t s);
bool demons_rows_nw2(const Bucket* d_bk, int nb, int h, int w, int level, int k, const Taps& tp, int radius, float tol,
                      int ty, hipStream_t s);
bool demons_rows2_nw2(const Bucket* d_bk, int nb, int h, int w, int level, int L, const Taps& tp, int radius, float tol,
                       int cap, int ty, hipStream_t s);
bool demons_rows_stage_nw2(const float* R, const float* T, int n, int h, int w, const float* u, const Taps& tp,
                            int radius, float* un, double* rms, hipStream_t s);
bool demons_rows_nw4(const Bucket* d_bk, int nb, int h, int w, int level, int k, const Taps& tp, int radius, float tol,
                      int ty, hipStream_t s);
bool demons_rows2_nw4(const Bucket* d_bk, int nb, int h, int w, int level, int L, const Taps& tp, int radius, float tol,
                       int cap, int ty, hipStream_t s);
bool demons_rows_stage_nw4(const float* R, const float* T, int n, int h, int w, const float* u, const Taps& tp,
                            int radius, float* un, double* rms, hipStream_t s);
bool demons_rows_nw8(const Bucket* d_bk, int nb, int h, int w, int level, int k, const Taps& tp, int radius, float tol,
                      int ty, hipStream_t s);
bool demons_rows2_nw8(const Bucket* d_bk, int nb, int h, int w, int level, int L, const Taps& tp, int radius, float tol,
                       int cap, int ty, hipStream_t s);
bool demons_rows_stage_nw8(const float* R, const float* T, int n, int h, int w, const float* u, const Taps& tp,
                            int radius, float* un, double* rms, hipStream_t s);

int rows_cpl(int w)
{
    if (w <= 64) return 1;
    if (w <= 128) return 2;
    if (w <= 256) return 4;
    if (w <= 512) return 8;
    // wider levels: column segments of 256 or 512 lanes, whichever leaves
    // fewer lanes idle (512 on a tie: fewer recomputed columns)
    const double u4 = (double)w / (rows_segs(w, 4) * 256), u8 = (double)w / (rows_segs(w, 8) * 512);
    return u4 > u8 ? 4 : 8;
}

bool rows_ty_supported(int ty) { return ty == 16 || ty == 32 || ty == 64 || ty == 128; }

bool rows2_ty_supported(int ty) { return ty == 8 || ty == 16 || ty == 32 || ty == 64 || ty == 128; }

bool rows2_ty_ok(int w, int ty) { return rows2_ty_supported(ty) && rows_cpl(w) && (ty != 8 || rows_cpl(w) <= 2); }

bool launch_demons_rows2(const Bucket* d_bk, const Bucket& hb, int level, int L, const Taps& tp, int radius,
                         float tol, int cap, int ty, hipStream_t s)
{
    const int h = hb.lh[level], w = hb.lw[level];
    switch (rows_cpl(w)) {
    case 1: return demons_rows2_nw1(d_bk, hb.nb, h, w, level, L, tp, radius, tol, cap, ty, s);
    case 2: return demons_rows2_nw2(d_bk, hb.nb, h, w, level, L, tp, radius, tol, cap, ty, s);
    case 4: return demons_rows2_nw4(d_bk, hb.nb, h, w, level, L, tp, radius, tol, cap, ty, s);
    case 8: return demons_rows2_nw8(d_bk, hb.nb, h, w, level, L, tp, radius, tol, cap, ty, s);
    default: return false;
    }
}

int rows_units(int h, int ty) { return (h + ty - 1) / ty; }

bool launch_demons_rows(const Bucket* d_bk, const Bucket& hb, int level, int k, const Taps& tp,
                        int radius, float tol, int ty, hipStream_t s)
{
    if (ty == 0) return false;  // the 2-D tile kernel
    const int h = hb.lh[level], w = hb.lw[level];
    switch (rows_cpl(w)) {
    case 1: return demons_rows_nw1(d_bk, hb.nb, h, w, level, k, tp, radius, tol, ty, s);
    case 2: return demons_rows_nw2(d_bk, hb.nb, h, w, level, k, tp, radius, tol, ty, s);
    case 4: return demons_rows_nw4(d_bk, hb.nb, h, w, level, k, tp, radius, tol, ty, s);
    case 8: return demons_rows_nw8(d_bk, hb.nb, h, w, level, k, tp, radius, tol, ty, s);
    default: return false;
    }
}

bool launch_demons_rows_stage(const float* R, const float* T, int n, int h, int w, const float* u,
                              const Taps& tp, int radius, float* un, double* rms, hipStream_t s)
{
    if (w > 512) return false;  // one segment per row only (the 2-D tile kernel takes wider images)
    switch (rows_cpl(w)) {
    case 1: return demons_rows_stage_nw1(R, T, n, h, w, u, tp, radius, un, rms, s);
    case 2: return demons_rows_stage_nw2(R, T, n, h, w, u, tp, radius, un, rms, s);
    case 4: return demons_rows_stage_nw4(R, T, n, h, w, u, tp, radius, un, rms, s);
    case 8: return demons_rows_stage_nw8(R, T, n, h, w, u, tp, radius, un, rms, s);
    default: return false;
    }
}

}  // namespace ebsd
