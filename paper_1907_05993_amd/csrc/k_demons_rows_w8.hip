// Instantiations of the row-marching demons kernels for rows of 512 threads
// (8 wavefronts): one translation unit per row width keeps compile times short.
#include "demons_rows_impl.h"

namespace ebsd {

bool demons_rows_nw8(const Bucket* d_bk, int nb, int h, int w, int level, int k, const Taps& tp, int radius, float tol,
                      int ty, hipStream_t s)
{
    return dispatch_rad<8>(d_bk, nb, h, w, level, k, tp, radius, tol, ty, s);
}

bool demons_rows2_nw8(const Bucket* d_bk, int nb, int h, int w, int level, int L, const Taps& tp, int radius, float tol,
                       int cap, int ty, hipStream_t s)
{
    return dispatch_rad2<8>(d_bk, nb, h, w, level, L, tp, radius, tol, cap, ty, s);
}

bool demons_rows_stage_nw8(const float* R, const float* T, int n, int h, int w, const float* u, const Taps& tp,
                            int radius, float* un, double* rms, hipStream_t s)
{
    return dispatch_rad_stage<8>(R, T, n, h, w, u, tp, radius, un, rms, s);
}

}  // namespace ebsd
