// Level-resident demons (multi-resolution demons, section 1, Eq. (1)): a level of
// at most 64 x 64 pixels is iterated to its cap or tolerance inside one
// workgroup per pair (lane = column, wavefront = row, eight rows per pass).
// The reference, the test and the field of the level stay in LDS for all
// iterations, so a coarse level costs one launch instead of one or two
// iterations per launch, and each pair stops on its own tolerance.
//
// Per iteration, three phases separated by workgroup barriers:
//   1. force: v = u + a grad R / (|grad R|^2 + a^2), a = R - T(x + u), with the
//      bilinear gather clamped to the level and blended with lerp_ends;
//   2. horizontal Gaussian taps of v (border columns replicated);
//   3. vertical taps (border rows replicated) into u, the squared update summed.
// Every pixel's arithmetic is that of the row-marching kernels (same gradient,
// gather, force, reciprocal and tap order), so the fields are bit-identical to
// theirs; the update's sum is reduced in another order, which can move a stop
// decision only when the RMS update lies within rounding of the tolerance.
#include <hip/hip_runtime.h>

#include "dev_util.h"
#include "ebsd_internal.h"
#include "../../include/ebsd.h"

namespace ebsd {

namespace {

constexpr int kResThreads = 512;
constexpr int kResRows = kResThreads / 64;  // rows per pass
constexpr int kResMaxPx = 64 * 64;
constexpr size_t kResLdsBytes = sizeof(float) * 8 * kResMaxPx;  // R, T, u (2), v (2), row taps (2)

// The three phases of an iteration over the rows a thread owns (y0, y0 + 8, ...), as
// functions whose LDS operands are restrict-qualified: the arrays are disjoint parts of
// the level's LDS, and with that known the compiler issues the reads of a group of four
// rows together instead of waiting for each row's stores before the next row's reads (an
// empty asm with a memory clobber between the two groups bounds the registers this takes).
constexpr int kResMaxRows = 64 / kResRows;
constexpr int kResGroup = kResMaxRows / 2;  // rows whose reads are issued together

__device__ __forceinline__ void res_force(const float* __restrict__ sR, const float* __restrict__ sT,
                                          const float* __restrict__ ux, const float* __restrict__ uy,
                                          float* __restrict__ vx, float* __restrict__ vy, int h, int w, int x,
                                          int y0, bool col, int xm, int xp, float sx, float wm1, float hm1,
                                          float wm2, float hm2, float wf, int ddx, int ddy)
{
#pragma unroll
    for (int j = 0; j < kResMaxRows; j++) {
        if (j == kResGroup) asm volatile("" ::: "memory");  // two groups of rows: bounded registers
        const int y = y0 + kResRows * j;
        if (y < h && col) {
            const int i = y * w + x;
            const int ym = max(y - 1, 0), yp = min(y + 1, h - 1);
            const float sy = (yp - ym == 2) ? 0.5f : 1.0f;
            const float gxr = (sR[y * w + xp] - sR[y * w + xm]) * sx;
            const float gyr = (sR[yp * w + x] - sR[ym * w + x]) * sy;
            const float u0 = ux[i], u1 = uy[i];
            const float xc = fminf(fmaxf((float)x + u0, 0.0f), wm1);
            const float yc = fminf(fmaxf((float)y + u1, 0.0f), hm1);
            const float xf = fminf(floorf(xc), wm2), yf = fminf(floorf(yc), hm2);
            const float fx = xc - xf, fy = yc - yf;
            const int o = (int)fmaf(yf, wf, xf);
            const float wv =
                lerp_ends(lerp_ends(sT[o], sT[o + ddx], fx), lerp_ends(sT[o + ddy], sT[o + ddx + ddy], fx), fy);
            const float a = sR[i] - wv;
            const float den = fmaf(gxr, gxr, fmaf(gyr, gyr, a * a));
            float v0 = u0, v1 = u1;
            if (den > 1e-9f) {
                const float q = a * __builtin_amdgcn_rcpf(den);
                v0 = fmaf(q, gxr, u0);
                v1 = fmaf(q, gyr, u1);
            }
            vx[i] = v0;
            vy[i] = v1;
        }
    }
}

template <int RAD>
__device__ __forceinline__ void res_taps_h(const float* __restrict__ vx, const float* __restrict__ vy,
                                           float* __restrict__ hx, float* __restrict__ hy, const Taps& tp, int h,
                                           int w, int x, int y0, bool col)
{
#pragma unroll
    for (int j = 0; j < kResMaxRows; j++) {
        if (j == kResGroup) asm volatile("" ::: "memory");  // two groups of rows: bounded registers
        const int y = y0 + kResRows * j;
        if (y < h && col) {
            const int i = y * w + x;
            float ax = 0.0f, ay = 0.0f;
#pragma unroll
            for (int t = 0; t <= 2 * RAD; t++) {
                const int c = y * w + clampi(x - RAD + t, 0, w - 1);
                ax = fmaf(tp.w[t], vx[c], ax);
                ay = fmaf(tp.w[t], vy[c], ay);
            }
            hx[i] = ax;
            hy[i] = ay;
        }
    }
}

// returns this thread's sum of squared updates
template <int RAD>
__device__ __forceinline__ float res_taps_v(const float* __restrict__ hx, const float* __restrict__ hy,
                                            float* __restrict__ ux, float* __restrict__ uy, const Taps& tp, int h,
                                            int w, int x, int y0, bool col)
{
    float ss = 0.0f;
#pragma unroll
    for (int j = 0; j < kResMaxRows; j++) {
        if (j == kResGroup) asm volatile("" ::: "memory");  // two groups of rows: bounded registers
        const int y = y0 + kResRows * j;
        if (y < h && col) {
            const int i = y * w + x;
            float ox = 0.0f, oy = 0.0f;
#pragma unroll
            for (int t = 0; t <= 2 * RAD; t++) {
                const int r = clampi(y - RAD + t, 0, h - 1) * w + x;
                ox = fmaf(tp.w[t], hx[r], ox);
                oy = fmaf(tp.w[t], hy[r], oy);
            }
            const float dx = ox - ux[i], dy = oy - uy[i];
            ss = fmaf(dx, dx, fmaf(dy, dy, ss));
            ux[i] = ox;
            uy[i] = oy;
        }
    }
    return ss;
}

template <int RAD>
__global__ void __launch_bounds__(kResThreads)
    k_demons_resident(const Bucket* __restrict__ bk, int level, Taps tp, float tol, int cap)
{
    extern __shared__ float lds[];
    __shared__ float red[kResThreads / 64];
    const int b = blockIdx.x;
    PairState st = bk->state[b];
    const int h = bk->lh[level], w = bk->lw[level], n = h * w;
    float* sR = lds;
    float* sT = sR + n;
    float* ux = sT + n;
    float* uy = ux + n;
    float* vx = uy + n;
    float* vy = vx + n;
    float* hx = vy + n;
    float* hy = hx + n;
    const float* __restrict__ Rg = bk->ref_pyr + (int64_t)bk->ref_slot[b] * bk->pyr_elems + bk->lvl_off[level];
    const float* __restrict__ Tg = bk->test_pyr + (int64_t)b * bk->pyr_elems + bk->lvl_off[level];
    const int64_t slot = (int64_t)b * 2 * bk->H * bk->W;
    const float* __restrict__ ug = bk->field[st.base & 1] + slot;
    for (int i = threadIdx.x; i < n; i += kResThreads) {
        sR[i] = Rg[i];
        sT[i] = Tg[i];
        ux[i] = ug[i];
        uy[i] = ug[n + i];
    }
    __syncthreads();

    // gather geometry (as bil_geom): the cell's corner stays in [0, w-2] x [0, h-2]
    const float wm1 = (float)(w - 1), hm1 = (float)(h - 1);
    const float wm2 = (float)max(w - 2, 0), hm2 = (float)max(h - 2, 0), wf = (float)w;
    const int ddx = w > 1 ? 1 : 0, ddy = h > 1 ? w : 0;
    const double scale = (double)(1 << level);
    const int x = threadIdx.x & 63, y0 = threadIdx.x >> 6;
    const bool col = x < w;
    const int xm = max(x - 1, 0), xp = min(x + 1, w - 1);
    const float sx = (xp - xm == 2) ? 0.5f : 1.0f;
    int k = 0;
    bool conv = false;
    while (k < cap) {
        // the column index passes through an empty asm once per iteration, so that the compiler
        // recomputes the rows' LDS addresses in each iteration instead of keeping them all live
        int xi = x;
        asm volatile("" : "+v"(xi));
        res_force(sR, sT, ux, uy, vx, vy, h, w, xi, y0, col, xm, xp, sx, wm1, hm1, wm2, hm2, wf, ddx, ddy);
        __syncthreads();
        res_taps_h<RAD>(vx, vy, hx, hy, tp, h, w, xi, y0, col);
        __syncthreads();
        float ss = res_taps_v<RAD>(hx, hy, ux, uy, tp, h, w, xi, y0, col);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ss;
        __syncthreads();
        float tot = 0.0f;
#pragma unroll
        for (int i = 0; i < kResThreads / 64; i++) tot += red[i];
        k++;
        // the same value in every thread: a uniform decision
        if (tol > 0.0f && sqrt((double)tot / ((double)h * (double)w)) * scale < (double)tol) conv = true;
        __syncthreads();  // red is rewritten by the next iteration
        if (conv) break;
    }
    float* __restrict__ out = bk->field[(st.base + k) & 1] + slot;
    for (int i = threadIdx.x; i < n; i += kResThreads) {
        out[i] = ux[i];
        out[n + i] = uy[i];
    }
    if (threadIdx.x == 0) {
        bk->iters[(int64_t)b * bk->L + level] = k;
        st.cur = (st.base + k) & 1;
        st.stop = -1;
        if (conv) st.convmask |= 1u << level;
        bk->state[b] = st;
    }
}

template <int RAD>
hipError_t launch_rad(const Bucket* d_bk, int nb, int level, const Taps& tp, float tol, int cap, hipStream_t s)
{
    static std::atomic<uint64_t> attr_done{0};
    const hipError_t e = ensure_dynamic_lds((const void*)k_demons_resident<RAD>, (int)kResLdsBytes, attr_done);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_demons_resident<RAD>, dim3((unsigned)nb), dim3(kResThreads), kResLdsBytes, s, d_bk, level,
                       tp, tol, cap);
    return hipGetLastError();
}

}  // namespace

bool demons_resident_ok(int h, int w) { return h >= 1 && w >= 1 && h <= 64 && w <= 64; }

hipError_t launch_demons_resident(const Bucket* d_bk, const Bucket& hb, int level, const float* taps, int radius,
                                  float tol, int cap, hipStream_t s)
{
    if (!demons_resident_ok(hb.lh[level], hb.lw[level]) || hb.nb <= 0) return hipErrorInvalidValue;
    Taps tp;
    for (int i = 0; i < 2 * kMaxRadius + 1; i++) tp.w[i] = i <= 2 * radius ? taps[i] : 0.0f;
    switch (radius) {
    case 0: return launch_rad<0>(d_bk, hb.nb, level, tp, tol, cap, s);
    case 1: return launch_rad<1>(d_bk, hb.nb, level, tp, tol, cap, s);
    case 2: return launch_rad<2>(d_bk, hb.nb, level, tp, tol, cap, s);
    case 3: return launch_rad<3>(d_bk, hb.nb, level, tp, tol, cap, s);
    case 4: return launch_rad<4>(d_bk, hb.nb, level, tp, tol, cap, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ebsd
