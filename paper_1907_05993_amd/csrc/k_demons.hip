// Fused demons iteration for gfx950 (multi-resolution demons registration,
// arXiv:1907.05993 section 1, Eq. (1)).
//
// One launch performs one iteration at one pyramid level for every pair that is
// still active.  Each 256-thread workgroup owns a 64 x 16 output tile of one
// pair and:
//   1. computes v = u + du on the tile plus a halo of r = radius pixels:
//        warped = T(x + u) (bilinear, clamped),  a = R - warped,
//        g = grad R (central differences, one-sided at the border),
//        du = a g / (|g|^2 + a^2)  (0 when the denominator is <= 1e-9);
//   2. smooths v with the separable Gaussian (horizontal pass, then vertical
//      pass, border replicated) through LDS;
//   3. writes u_new and the block's sum of |u_new - u|^2.
// With a tolerance, each workgroup first reduces the pair's per-tile sums of
// the previous iteration in a fixed order (the same value in every workgroup)
// and skips the pair when 2^l RMS < tol; tile 0 records the stop.  No fences
// or atomics: a device-scope release fence per workgroup would write the whole
// L2 back to memory on this chip.
//
// Traffic per pixel and iteration: read u (8 B) + R (4 B) + T (4 B, gather),
// write u (8 B) = 24 B; the halo re-reads come from L2.  Consecutive tiles of a
// pair are placed on the same XCD so that halo and gather reuse stays inside one
// L2.
#include "dev_util.h"

namespace ebsd {

namespace {

constexpr int TX = kDemonsTX;
constexpr int TY = kDemonsTY;
constexpr int NT = kDemonsThreads;

// Wave64 + block reduction of one float per thread, fixed order; result valid
// in thread 0.
__device__ inline float block_sum_f(float v, float* red)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = v;
    __syncthreads();
    float r = 0.0f;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NT / 64; i++) r += red[i];
    }
    return r;
}

// One demons iteration on one tile.  Returns (in thread 0) the tile's sum of
// squared updates over in-image pixels.
template <int RAD>
__device__ float demons_tile(const float* __restrict__ Rg, const float* __restrict__ Tg,
                             const float* __restrict__ ug, float* __restrict__ ung, int h, int w,
                             int x0, int y0, const Taps& tp)
{
    const EBSD_GLOBAL float* __restrict__ R = gptr(Rg);
    const EBSD_GLOBAL float* __restrict__ T = gptr(Tg);
    const EBSD_GLOBAL float* __restrict__ u = gptr(ug);
    EBSD_GLOBAL float* __restrict__ un = gptr(ung);
    constexpr int RY = TY + 2 * RAD;
    constexpr int RX = TX + 2 * RAD;
    __shared__ float vx[RY][RX];
    __shared__ float vy[RY][RX];
    __shared__ float hx[RY][TX];
    __shared__ float hy[RY][TX];
    __shared__ float red[NT / 64];

    const int tid = threadIdx.x;
    const int64_t hw = (int64_t)h * w;
    const EBSD_GLOBAL float* __restrict__ uy_src = u + hw;

    // 1. v = u + du on the tile and its halo (clamped coordinates replicate
    //    the border, which is what the smoothing's clamped taps need).
    for (int c = tid; c < RY * RX; c += NT) {
        const int gy = c / RX, gx = c - gy * RX;
        const int yy = clampi(y0 + gy - RAD, 0, h - 1);
        const int xx = clampi(x0 + gx - RAD, 0, w - 1);
        const int64_t i = (int64_t)yy * w + xx;
        const float ux = u[i], uy = uy_src[i];
        const float r = R[i];
        // central difference inside, one-sided on the border (no branches)
        const int xm = max(xx - 1, 0), xp = min(xx + 1, w - 1);
        const int ym = max(yy - 1, 0), yp = min(yy + 1, h - 1);
        const float sx = (xp - xm == 2) ? 0.5f : 1.0f;
        const float sy = (yp - ym == 2) ? 0.5f : 1.0f;
        const int64_t row = (int64_t)yy * w;
        const float gxr = (R[row + xp] - R[row + xm]) * sx;
        const float gyr = (R[(int64_t)yp * w + xx] - R[(int64_t)ym * w + xx]) * sy;
        const float wv = bilinear_lerp(T, h, w, (float)xx + ux, (float)yy + uy);
        const float a = r - wv;
        const float den = fmaf(gxr, gxr, fmaf(gyr, gyr, a * a));
        float vxx = ux, vyy = uy;
        if (den > 1e-9f) {
            const float s = a * __builtin_amdgcn_rcpf(den);
            vxx = fmaf(s, gxr, ux);
            vyy = fmaf(s, gyr, uy);
        }
        vx[gy][gx] = vxx;
        vy[gy][gx] = vyy;
    }
    __syncthreads();

    // 2. horizontal Gaussian pass over all RY rows.
    for (int c = tid; c < RY * TX; c += NT) {
        const int gy = c / TX, x = c - gy * TX;
        float ax = 0.0f, ay = 0.0f;
#pragma unroll
        for (int j = 0; j <= 2 * RAD; j++) {
            ax = fmaf(tp.w[j], vx[gy][x + j], ax);
            ay = fmaf(tp.w[j], vy[gy][x + j], ay);
        }
        hx[gy][x] = ax;
        hy[gy][x] = ay;
    }
    __syncthreads();

    // 3. vertical pass, write u_new, accumulate |u_new - u|^2.
    float ss = 0.0f;
    for (int c = tid; c < TY * TX; c += NT) {
        const int y = c / TX, x = c - y * TX;
        float ax = 0.0f, ay = 0.0f;
#pragma unroll
        for (int j = 0; j <= 2 * RAD; j++) {
            ax = fmaf(tp.w[j], hx[y + j][x], ax);
            ay = fmaf(tp.w[j], hy[y + j][x], ay);
        }
        const int gy = y0 + y, gx = x0 + x;
        if (gy < h && gx < w) {
            const int64_t i = (int64_t)gy * w + gx;
            const float dx = ax - u[i], dy = ay - uy_src[i];
            ss = fmaf(dx, dx, fmaf(dy, dy, ss));
            un[i] = ax;
            un[hw + i] = ay;
        }
    }
    return block_sum_f(ss, red);
}

template <int RAD>
__global__ void __launch_bounds__(NT)
    k_demons_iter(const Bucket* __restrict__ bk, int level, int k, Taps tp, float tol, int tiles_x,
                  int ntiles)
{
    __shared__ double sh_sum;
    const int G = gridDim.x;
    const int lb = xcd_logical_block(blockIdx.x, G);
    const int b = lb / ntiles;
    const int tile = lb - b * ntiles;
    const PairState st = bk->state[b];
    if (st.stop >= 0) return;  // uniform over the block
    const int h = bk->lh[level], w = bk->lw[level];
    const int64_t npart = (int64_t)bk->nb * bk->max_tiles;
    if (tol > 0.0f && k > 0) {
        const float* prev = bk->partial + ((k - 1) & 1) * npart + (int64_t)b * bk->max_tiles;
        const double ss = pair_sum(prev, ntiles, &sh_sum);
        const double delta = sqrt(ss / ((double)h * (double)w)) * (double)(1 << level);
        if (delta < (double)tol) {
            if (tile == 0 && threadIdx.x == 0) {
                bk->state[b].stop = k;
                bk->state[b].convmask = st.convmask | (1u << level);
            }
            return;
        }
    }
    const int64_t slot = (int64_t)b * 2 * bk->H * bk->W;
    const float* R = bk->ref_pyr + (int64_t)bk->ref_slot[b] * bk->pyr_elems + bk->lvl_off[level];
    const float* T = bk->test_pyr + (int64_t)b * bk->pyr_elems + bk->lvl_off[level];
    const float* u = bk->field[(st.base + k) & 1] + slot;
    float* un = bk->field[(st.base + k + 1) & 1] + slot;
    const int ty = tile / tiles_x, tx = tile - ty * tiles_x;

    const float ss = demons_tile<RAD>(R, T, u, un, h, w, tx * TX, ty * TY, tp);
    if (tol > 0.0f && threadIdx.x == 0)
        bk->partial[(k & 1) * npart + (int64_t)b * bk->max_tiles + tile] = ss;
}

// End of level l, one thread per pair: iteration count, convergence on the
// last iteration (the in-loop check sees iteration k - 1 only), final buffer.
// fused != 0: the level ran two iterations per launch (partial slot i & 3,
// final field after n iterations in buffer (base + ceil(n / 2)) & 1).
__global__ void k_level_end(const Bucket* __restrict__ bk, int level, int cap, float tol, int ntiles, int fused)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= bk->nb) return;
    PairState st = bk->state[b];
    int n = st.stop >= 0 ? st.stop : cap;
    if (st.stop < 0 && tol > 0.0f && cap > 0) {
        const int64_t npart = (int64_t)bk->nb * bk->max_tiles;
        const int slot = fused ? ((cap - 1) & 3) : ((cap - 1) & 1);
        const float* last = bk->partial + slot * npart + (int64_t)b * bk->max_tiles;
        // same fixed order as pair_sum: 64 strided lanes, then the xor tree
        double lane[64];
        for (int l = 0; l < 64; l++) {
            lane[l] = 0.0;
            for (int i = l; i < ntiles; i += 64) lane[l] += (double)last[i];
        }
        for (int off = 32; off > 0; off >>= 1)
            for (int l = 0; l < 64; l++)
                if ((l & off) == 0) {
                    const double a = lane[l], c = lane[l | off];
                    lane[l] = a + c;
                    lane[l | off] = c + a;
                }
        const int h = bk->lh[level], w = bk->lw[level];
        const double delta = sqrt(lane[0] / ((double)h * (double)w)) * (double)(1 << level);
        if (delta < (double)tol) st.convmask |= 1u << level;
    }
    bk->iters[(int64_t)b * bk->L + level] = n;
    st.cur = fused ? (st.base + (n + 1) / 2) & 1 : (st.base + n) & 1;
    st.stop = -1;
    bk->state[b] = st;
}

// Stand-alone variant for the single-stage entry point: one block per pair
// walks all of its tiles in order, so the RMS of the update is reduced in a
// fixed order without scratch memory.
template <int RAD>
__global__ void __launch_bounds__(NT)
    k_demons_stage(const float* __restrict__ R, const float* __restrict__ T, int h, int w,
                   const float* __restrict__ u, Taps tp, float* __restrict__ un,
                   double* __restrict__ rms, int tiles_x, int ntiles)
{
    const int b = blockIdx.x;
    const int64_t hw = (int64_t)h * w;
    double acc = 0.0;
    for (int tile = 0; tile < ntiles; tile++) {
        const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
        const float ss = demons_tile<RAD>(R + b * hw, T + b * hw, u + 2 * b * hw, un + 2 * b * hw,
                                          h, w, tx * TX, ty * TY, tp);
        acc += (double)ss;  // meaningful in thread 0 only
        __syncthreads();
    }
    if (rms && threadIdx.x == 0) rms[b] = sqrt(acc / (double)hw);
}

Taps make_taps(const float* taps, int radius)
{
    Taps t;
    for (int i = 0; i < 2 * kMaxRadius + 1; i++) t.w[i] = i <= 2 * radius ? taps[i] : 0.0f;
    return t;
}

template <int RAD>
void launch_iter_rad(const Bucket* d_bk, const Bucket& hb, int level, int k, const Taps& tp,
                     float tol, hipStream_t s)
{
    const int h = hb.lh[level], w = hb.lw[level];
    const int tiles_x = (w + TX - 1) / TX;
    const int ntiles = demons_tiles(h, w);
    const int G = hb.nb * ntiles;
    hipLaunchKernelGGL(k_demons_iter<RAD>, dim3(G), dim3(NT), 0, s, d_bk, level, k, tp, tol,
                       tiles_x, ntiles);
}

}  // namespace

hipError_t launch_demons_iter2(const Bucket* d_bk, const Bucket& hb, int level, int L, const float* taps,
                               int radius, float tol, int cap, int ty, hipStream_t s)
{
    const Taps tp = make_taps(taps, radius);
    if (!launch_demons_rows2(d_bk, hb, level, L, tp, radius, tol, cap, ty, s)) return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_demons_iter(const Bucket* d_bk, const Bucket& hb, int level, int k,
                              const float* taps, int radius, float tol, int ty, hipStream_t s)
{
    const Taps tp = make_taps(taps, radius);
    if (launch_demons_rows(d_bk, hb, level, k, tp, radius, tol, ty, s)) return hipGetLastError();
    switch (radius) {
    case 0: launch_iter_rad<0>(d_bk, hb, level, k, tp, tol, s); break;
    case 1: launch_iter_rad<1>(d_bk, hb, level, k, tp, tol, s); break;
    case 2: launch_iter_rad<2>(d_bk, hb, level, k, tp, tol, s); break;
    case 3: launch_iter_rad<3>(d_bk, hb, level, k, tp, tol, s); break;
    case 4: launch_iter_rad<4>(d_bk, hb, level, k, tp, tol, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// One workgroup: the pairs that have not recorded a stop (fixed-order sum).
__global__ void __launch_bounds__(256) k_count_active(const Bucket* __restrict__ bk, int32_t* out)
{
    __shared__ int part[4];
    int c = 0;
    for (int b = threadIdx.x; b < bk->nb; b += 256) c += bk->state[b].stop < 0 ? 1 : 0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) *out = part[0] + part[1] + part[2] + part[3];
}

hipError_t launch_count_active(const Bucket* d_bk, int32_t* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_count_active, dim3(1), dim3(256), 0, s, d_bk, out);
    return hipGetLastError();
}

hipError_t launch_level_end(const Bucket* d_bk, const Bucket& hb, int level, int cap, float tol,
                            int ty, bool fused, hipStream_t s)
{
    const int ntiles = demons_units(hb.lh[level], hb.lw[level], ty);
    hipLaunchKernelGGL(k_level_end, dim3((hb.nb + 63) / 64), dim3(64), 0, s, d_bk, level, cap, tol,
                       ntiles, fused ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_stage_demons_iter(const float* R, const float* T, int n, int H, int W,
                                    const float* u_in, const float* taps, int radius,
                                    float* u_out, double* rms, hipStream_t s)
{
    const Taps tp = make_taps(taps, radius);
    if (launch_demons_rows_stage(R, T, n, H, W, u_in, tp, radius, u_out, rms, s))
        return hipGetLastError();
    const int tiles_x = (W + TX - 1) / TX;
    const int ntiles = demons_tiles(H, W);
    dim3 grid(n);
    switch (radius) {
    case 0: hipLaunchKernelGGL(k_demons_stage<0>, grid, dim3(NT), 0, s, R, T, H, W, u_in, tp, u_out, rms, tiles_x, ntiles); break;
    case 1: hipLaunchKernelGGL(k_demons_stage<1>, grid, dim3(NT), 0, s, R, T, H, W, u_in, tp, u_out, rms, tiles_x, ntiles); break;
    case 2: hipLaunchKernelGGL(k_demons_stage<2>, grid, dim3(NT), 0, s, R, T, H, W, u_in, tp, u_out, rms, tiles_x, ntiles); break;
    case 3: hipLaunchKernelGGL(k_demons_stage<3>, grid, dim3(NT), 0, s, R, T, H, W, u_in, tp, u_out, rms, tiles_x, ntiles); break;
    case 4: hipLaunchKernelGGL(k_demons_stage<4>, grid, dim3(NT), 0, s, R, T, H, W, u_in, tp, u_out, rms, tiles_x, ntiles); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace ebsd
