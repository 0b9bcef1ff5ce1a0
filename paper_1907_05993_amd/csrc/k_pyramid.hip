// Normalisation, pyramid restriction / prolongation and field bookkeeping
// kernels (multi-resolution demons, section 1 of arXiv:1907.05993).
//
// All of these are HBM-streaming passes that touch each pattern a few times per
// batch; they are far from the hot loop and are written for coalesced access
// rather than for peak bandwidth.
#include <cmath>

#include "dev_util.h"

#include "../../include/ebsd.h"

namespace ebsd {

namespace {

constexpr int kStatThreads = 256;

// Deterministic block sum of one double per thread (fixed tree order).
__device__ double block_sum(double v, double* sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = kStatThreads / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// Sum over one pattern of f(v) for every value v, per thread in a fixed order:
// 16-byte loads, four in flight per thread (one workgroup per pattern leaves
// few waves per CU, so the loads' latency has to be covered by the thread's
// own outstanding loads), and a scalar tail.  Requires 16-byte alignment for
// the vector part (else all scalar).
template <class F>
__device__ double pattern_sum(const float* __restrict__ p, int64_t n, F f)
{
    constexpr int T = kStatThreads;
    double acc = 0.0;
    const int64_t nv = ((uintptr_t)p & 15) == 0 ? n / 4 : 0;
    const float4* __restrict__ p4 = reinterpret_cast<const float4*>(p);
    int64_t i = threadIdx.x;
    for (; i + 3 * T < nv; i += 4 * T) {
        const float4 a = p4[i], b = p4[i + T], c = p4[i + 2 * T], d = p4[i + 3 * T];
        acc += f(a.x) + f(a.y) + f(a.z) + f(a.w);
        acc += f(b.x) + f(b.y) + f(b.z) + f(b.w);
        acc += f(c.x) + f(c.y) + f(c.z) + f(c.w);
        acc += f(d.x) + f(d.y) + f(d.z) + f(d.w);
    }
    for (; i < nv; i += T) {
        const float4 a = p4[i];
        acc += f(a.x) + f(a.y) + f(a.z) + f(a.w);
    }
    for (int64_t j = 4 * nv + threadIdx.x; j < n; j += T) acc += f(p[j]);
    return acc;
}

// Mean and 1/std of one pattern in FP64 (two passes: mean, then centred sum
// of squares).  Non-finite values or zero contrast are flagged.
__device__ void pattern_stats(const float* __restrict__ p, int64_t n, PatStat* out, double* sh)
{
    // the FP64 sum of finite floats cannot overflow (n < 2^40), so it is finite exactly
    // when every value is
    double tot = block_sum(pattern_sum(p, n, [](float v) { return (double)v; }), sh);
    const bool bad = !isfinite(tot);
    double mean = tot / (double)n;
    double ss = bad ? 0.0 : pattern_sum(p, n, [mean](float v) {
        const double d = (double)v - mean;
        return d * d;
    });
    double var = block_sum(ss, sh) / (double)n;
    if (threadIdx.x == 0) {
        PatStat st;
        st.pad = 0;
        if (bad) {
            st.mean = 0.0;
            st.inv_std = 0.0;
            st.flags = EBSD_NONFINITE_INPUT;
        } else {
            double sd = sqrt(var);
            if (!(sd > 1e-12 * (fabs(mean) + 1.0))) {
                st.mean = 0.0;
                st.inv_std = 0.0;
                st.flags = EBSD_DEGENERATE_INPUT;
            } else {
                st.mean = mean;
                st.inv_std = 1.0 / sd;
                st.flags = 0;
            }
        }
        *out = st;
    }
}

// Statistics of each raw pattern, or of its pre-filtered copy in level 0.
__global__ void __launch_bounds__(kStatThreads) k_stats(const Bucket* __restrict__ bk)
{
    __shared__ double sh[kStatThreads];
    const int i = blockIdx.x;
    const int64_t n = (int64_t)bk->H * bk->W;
    if (i < bk->nb)
        pattern_stats(bk->prefilter ? bk->test_pyr + (int64_t)i * bk->pyr_elems : bk->test_in[i], n,
                      &bk->test_stat[i], sh);
    else
        pattern_stats(bk->prefilter ? bk->ref_pyr + (int64_t)(i - bk->nb) * bk->pyr_elems : bk->ref_in[i - bk->nb],
                      n, &bk->ref_stat[i - bk->nb], sh);
}

// Level 0 of every pyramid: (p - mean) / std, zeros for flagged patterns.
__global__ void k_normalize_l0(const Bucket* __restrict__ bk)
{
    const int pat = blockIdx.y;
    const int64_t n = (int64_t)bk->H * bk->W;
    const float* src;
    float* dst;
    PatStat st;
    if (pat < bk->nb) {
        dst = bk->test_pyr + (int64_t)pat * bk->pyr_elems;
        src = bk->prefilter ? dst : bk->test_in[pat];  // in place over the pre-filtered copy
        st = bk->test_stat[pat];
    } else {
        int r = pat - bk->nb;
        dst = bk->ref_pyr + (int64_t)r * bk->pyr_elems;
        src = bk->prefilter ? dst : bk->ref_in[r];
        st = bk->ref_stat[r];
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        float v = 0.0f;
        if (st.flags == 0) v = (float)(((double)src[i] - st.mean) * st.inv_std);
        dst[i] = v;
    }
}

// Factor-2 restriction, separable [1,3,3,1]/8 with clamped borders:
// coarse pixel i is centred on fine 2i + 0.5; an odd size N gives ceil(N/2)
// coarse pixels, the last reading the border through the clamp.  Horizontal
// pass first.
__device__ inline float restrict_at(const float* __restrict__ in, int H, int W, int j, int i)
{
    float h[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const float* row = in + (int64_t)clampi(2 * j - 1 + k, 0, H - 1) * W;
        float a = row[clampi(2 * i - 1, 0, W - 1)];
        float b = row[clampi(2 * i, 0, W - 1)];
        float c = row[clampi(2 * i + 1, 0, W - 1)];
        float d = row[clampi(2 * i + 2, 0, W - 1)];
        h[k] = (a + 3.0f * b + 3.0f * c + d) / 8.0f;
    }
    return (h[0] + 3.0f * h[1] + 3.0f * h[2] + h[3]) / 8.0f;
}

__global__ void k_restrict_level(const Bucket* __restrict__ bk, int level)
{
    const int pat = blockIdx.y;
    float* base = pat < bk->nb ? bk->test_pyr + (int64_t)pat * bk->pyr_elems
                               : bk->ref_pyr + (int64_t)(pat - bk->nb) * bk->pyr_elems;
    const int Hi = bk->lh[level - 1], Wi = bk->lw[level - 1];
    const int h = bk->lh[level], w = bk->lw[level];
    const float* in = base + bk->lvl_off[level - 1];
    float* out = base + bk->lvl_off[level];
    // per-pattern indices fit in 32 bits (sides of at most 16384 px)
    const int n = h * w;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
        const int j = t / w, i = t - j * w;
        out[t] = restrict_at(in, Hi, Wi, j, i);
    }
}

__global__ void k_restrict_plain(const float* __restrict__ in, int H, int W,
                                 float* __restrict__ out)
{
    const int pat = blockIdx.y;
    const int h = (H + 1) / 2, w = (W + 1) / 2;
    const float* src = in + (int64_t)pat * H * W;
    float* dst = out + (int64_t)pat * h * w;
    const int n = h * w;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
        const int j = t / w, i = t - j * w;
        dst[t] = restrict_at(src, H, W, j, i);
    }
}

// Prolongation u_{l-1}(x) = 2 bilinear(u_l, (x - 0.5)/2): half-pixel centres;
// the finer level is H2 x W2 (2h x 2w, or one less where it was odd).
// Output t of the two channels (t < 2 H2 W2, which fits in 32 bits for sides
// of at most 16384 px).
__device__ inline void prolong_one(const float* __restrict__ src, int h, int w, int H2, int W2,
                                   float* __restrict__ dst, int t)
{
    const int hw2 = H2 * W2;
    const int c = t >= hw2 ? 1 : 0;
    const int r = t - c * hw2;
    const int y = r / W2, x = r - y * W2;
    float sx = ((float)x - 0.5f) * 0.5f, sy = ((float)y - 0.5f) * 0.5f;
    dst[t] = 2.0f * bilinear_clamped(src + c * h * w, h, w, sx, sy);
}

__global__ void k_prolong_level(const Bucket* __restrict__ bk, int level)
{
    const int b = blockIdx.y;
    const int h = bk->lh[level], w = bk->lw[level];
    const int H2 = bk->lh[level - 1], W2 = bk->lw[level - 1];
    const int cur = bk->state[b].cur;
    const int64_t slot = (int64_t)b * 2 * bk->H * bk->W;
    const float* src = bk->field[cur] + slot;
    float* dst = bk->field[cur ^ 1] + slot;
    const int n = 2 * H2 * W2;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x)
        prolong_one(src, h, w, H2, W2, dst, t);
}

__global__ void k_rearm(const Bucket* __restrict__ bk)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= bk->nb) return;
    PairState st = bk->state[b];
    st.base = st.cur ^ 1;  // the prolonged field was written to the other buffer
    st.stop = -1;
    bk->state[b] = st;
}

__global__ void k_prolong_plain(const float* __restrict__ u, int h, int w, float* __restrict__ out)
{
    const int b = blockIdx.y;
    const float* src = u + (int64_t)b * 2 * h * w;
    float* dst = out + (int64_t)b * 2 * 4 * h * w;
    const int n = 2 * 4 * h * w;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x)
        prolong_one(src, h, w, 2 * h, 2 * w, dst, t);
}

// Reset demons state; coarsest-level field = u_init / 2^(L-1) or zero.
__global__ void k_demons_init(const Bucket* __restrict__ bk)
{
    const float* __restrict__ u_init = bk->u_init;
    const int b = blockIdx.y;
    const int L = bk->L;
    const int h = bk->lh[L - 1], w = bk->lw[L - 1];
    const int64_t n = (int64_t)2 * h * w;
    float* dst = bk->field[0] + (int64_t)b * 2 * bk->H * bk->W;
    const float scale = 1.0f / (float)(1 << (L - 1));
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        dst[t] = u_init ? u_init[(int64_t)b * n + t] * scale : 0.0f;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        PairState st;
        st.base = 0;
        st.stop = -1;
        st.cur = 0;
        st.convmask = 0;
        bk->state[b] = st;
        for (int l = 0; l < L; l++) bk->iters[(int64_t)b * L + l] = 0;
    }
}

__global__ void k_sample_q1(const Bucket* __restrict__ bk)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= bk->nb * bk->n_roi) return;
    int b = t / bk->n_roi, j = t % bk->n_roi;
    const int H = bk->H, W = bk->W;
    const float* f = bk->field[bk->state[b].cur] + (int64_t)b * 2 * H * W;
    float cx = (float)bk->roi_c[2 * j], cy = (float)bk->roi_c[2 * j + 1];
    bk->q1[2 * t] = bilinear_clamped(f, H, W, cx, cy);
    bk->q1[2 * t + 1] = bilinear_clamped(f + (int64_t)H * W, H, W, cx, cy);
}

// ---- pre-filter -------------------------------------------------------------------
// Gaussian low-pass minus Gaussian background estimate, separable, replicated
// border.  Horizontal pass: one workgroup per (row, pattern), the row in LDS,
// both filters' row sums to tmp; vertical pass: one thread per pixel, the
// column sums combined into the destination.
__device__ inline const float* band_src(const BandIO& io, int p)
{
    if (io.src) return io.src + (int64_t)p * io.src_stride;
    if (io.src_a) return p < io.na ? io.src_a[p] : io.src_b[p - io.na];
    return p < io.na ? io.srcb_a + (int64_t)p * io.srcb_stride : io.srcb_b + (int64_t)(p - io.na) * io.srcb_stride;
}

__device__ inline float* band_dst(const BandIO& io, int p)
{
    return p < io.na ? io.dst_a + (int64_t)p * io.dst_stride : io.dst_b + (int64_t)(p - io.na) * io.dst_stride;
}

// static background: pixelwise mean of the nb patterns (double sums in order)
__global__ void k_mean_pattern(const float* const* __restrict__ src, int nb, int64_t hw, float* __restrict__ bg)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hw; i += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int k = 0; k < nb; k++) s += (double)src[k][i];
        bg[i] = (float)(s / (double)nb);
    }
}

__global__ void k_bg_static(BandIO io, const float* __restrict__ bg)
{
    const int p = blockIdx.y;
    const int64_t hw = (int64_t)io.H * io.W;
    const float* __restrict__ src = band_src(io, p);
    float* dst = band_dst(io, p);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hw; i += (int64_t)gridDim.x * blockDim.x) {
        float v = src[i];
        if (bg) {
            const float d = bg[i];
            v = d > 0.0f ? v / d : 0.0f;
        }
        dst[i] = v;
    }
}

__global__ void k_bg_dynamic(BandIO io, const float* __restrict__ blur)
{
    const int p = blockIdx.y;
    const int64_t hw = (int64_t)io.H * io.W;
    float* dst = band_dst(io, p);
    const float* __restrict__ b = blur + (int64_t)p * hw;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hw; i += (int64_t)gridDim.x * blockDim.x) {
        const float d = b[i];
        dst[i] = d > 0.0f ? dst[i] / d : 0.0f;
    }
}

__global__ void __launch_bounds__(256) k_band_rows(BandIO io, BandTaps tp)
{
    extern __shared__ float row[];
    const int y = blockIdx.x, p = blockIdx.y, W = io.W;
    const float* __restrict__ src = band_src(io, p) + (int64_t)y * W;
    for (int x = threadIdx.x; x < W; x += 256) row[x] = src[x];
    __syncthreads();
    const int64_t HW = (int64_t)io.H * W;
    float* tlo = io.tmp + (2 * (int64_t)p) * HW + (int64_t)y * W;
    float* thi = tlo + HW;
    for (int x = threadIdx.x; x < W; x += 256) {
        if (tp.rlo >= 0) {
            float acc = 0.0f;
            for (int j = -tp.rlo; j <= tp.rlo; j++) acc += tp.lo[j + tp.rlo] * row[clampi(x + j, 0, W - 1)];
            tlo[x] = acc;
        }
        if (tp.rhi >= 0) {
            float acc = 0.0f;
            for (int j = -tp.rhi; j <= tp.rhi; j++) acc += tp.hi[j + tp.rhi] * row[clampi(x + j, 0, W - 1)];
            thi[x] = acc;
        }
    }
}

__global__ void __launch_bounds__(256) k_band_cols(BandIO io, BandTaps tp)
{
    const int p = blockIdx.y, H = io.H, W = io.W;
    const int64_t HW = (int64_t)H * W;
    const float* __restrict__ tlo = io.tmp + (2 * (int64_t)p) * HW;
    const float* __restrict__ thi = tlo + HW;
    const float* src = band_src(io, p);  // may be dst (in place): read before the write of each element
    float* dst = band_dst(io, p);
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < HW; t += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(t / W), x = (int)(t - (int64_t)W * (t / W));
        float v;
        if (tp.rlo >= 0) {
            v = 0.0f;
            for (int j = -tp.rlo; j <= tp.rlo; j++) v += tp.lo[j + tp.rlo] * tlo[(int64_t)clampi(y + j, 0, H - 1) * W + x];
        } else {
            v = src[t];
        }
        if (tp.rhi >= 0) {
            float b = 0.0f;
            for (int j = -tp.rhi; j <= tp.rhi; j++) b += tp.hi[j + tp.rhi] * thi[(int64_t)clampi(y + j, 0, H - 1) * W + x];
            v -= b;
        }
        dst[t] = v;
    }
}

// ---- structural similarity of the registration -----------------------------------
// Tiles of 32 x 32 output pixels over the pixels whose 11 x 11 window fits
// (x, y in [5, W - 5) x [5, H - 5)); the (32 + 10)^2 patch of the reference
// and of the warped test, T(x + u(x)) (bilinear, clamped), sits in LDS; a
// horizontal pass leaves the five windowed sums (a, b, a^2, b^2, ab) of 42
// rows x 32 columns in LDS, the vertical pass forms SSIM per pixel; the tile's
// sum (double) goes to ssim_part, and k_ssim_finish adds the tiles of a pair
// in order.
constexpr int kSsimT = 32, kSsimR = 5, kSsimP = kSsimT + 2 * kSsimR;

__device__ inline void ssim_taps(float (&w)[2 * kSsimR + 1])
{
    double ws = 0.0, t[2 * kSsimR + 1];
    for (int j = -kSsimR; j <= kSsimR; j++) ws += (t[j + kSsimR] = exp(-(double)(j * j) / (2.0 * 1.5 * 1.5)));
    for (int j = 0; j <= 2 * kSsimR; j++) w[j] = (float)(t[j] / ws);
}

__global__ void __launch_bounds__(256) k_ssim_tiles(const Bucket* __restrict__ bk, int tiles_x)
{
    __shared__ float sa[kSsimP][kSsimP + 1], sb[kSsimP][kSsimP + 1];
    __shared__ float hsum[5][kSsimP][kSsimT + 1];
    __shared__ double red[256];
    const int b = blockIdx.y, tile = blockIdx.x;
    const int H = bk->H, W = bk->W;
    const int tyi = tile / tiles_x, txi = tile - tyi * tiles_x;
    const int ox = kSsimR + txi * kSsimT, oy = kSsimR + tyi * kSsimT;
    const float* __restrict__ R = bk->ref_pyr + (int64_t)bk->ref_slot[b] * bk->pyr_elems;
    const float* __restrict__ T = bk->test_pyr + (int64_t)b * bk->pyr_elems;
    const int64_t HW = (int64_t)H * W;
    const float* __restrict__ u = bk->field[bk->state[b].cur] + (int64_t)b * 2 * HW;
    float w[2 * kSsimR + 1];
    ssim_taps(w);
    for (int i = threadIdx.x; i < kSsimP * kSsimP; i += 256) {
        const int py = i / kSsimP, px = i - kSsimP * (i / kSsimP);
        // rows / columns past the pattern only feed outputs that are skipped
        const int y = min(oy - kSsimR + py, H - 1), x = min(ox - kSsimR + px, W - 1);
        const int64_t o = (int64_t)y * W + x;
        sa[py][px] = R[o];
        sb[py][px] = bilinear_clamped(T, H, W, (float)x + u[o], (float)y + u[HW + o]);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kSsimP * kSsimT; i += 256) {
        const int py = i / kSsimT, c = i - kSsimT * (i / kSsimT);
        float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f, s4 = 0.0f;
#pragma unroll
        for (int j = 0; j <= 2 * kSsimR; j++) {
            const float a = sa[py][c + j], bv = sb[py][c + j], ww = w[j];
            s0 += ww * a;
            s1 += ww * bv;
            s2 += ww * (a * a);
            s3 += ww * (bv * bv);
            s4 += ww * (a * bv);
        }
        hsum[0][py][c] = s0;
        hsum[1][py][c] = s1;
        hsum[2][py][c] = s2;
        hsum[3][py][c] = s3;
        hsum[4][py][c] = s4;
    }
    __syncthreads();
    const float L = 6.0f, C1 = (0.01f * L) * (0.01f * L), C2 = (0.03f * L) * (0.03f * L);
    double acc = 0.0;
    for (int i = threadIdx.x; i < kSsimT * kSsimT; i += 256) {
        const int r = i / kSsimT, c = i - kSsimT * (i / kSsimT);
        if (oy + r >= H - kSsimR || ox + c >= W - kSsimR) continue;
        float m[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int j = 0; j <= 2 * kSsimR; j++)
#pragma unroll
            for (int k = 0; k < 5; k++) m[k] += w[j] * hsum[k][r + j][c];
        const float va = m[2] - m[0] * m[0], vb = m[3] - m[1] * m[1], cv = m[4] - m[0] * m[1];
        acc += (double)((2.0f * m[0] * m[1] + C1) * (2.0f * cv + C2) /
                        ((m[0] * m[0] + m[1] * m[1] + C1) * (va + vb + C2)));
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) bk->ssim_part[(int64_t)b * gridDim.x + tile] = red[0];
}

__global__ void k_ssim_finish(const Bucket* __restrict__ bk, int tiles)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= bk->nb) return;
    double s = 0.0;
    for (int t = 0; t < tiles; t++) s += bk->ssim_part[(int64_t)b * tiles + t];
    bk->ssim[b] = s / ((double)(bk->H - 2 * kSsimR) * (double)(bk->W - 2 * kSsimR));
}

__global__ void k_zero_iters(const Bucket* __restrict__ bk)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < (int64_t)bk->nb * bk->L) bk->iters[t] = 0;
}

__global__ void k_copy_field(const Bucket* __restrict__ bk)
{
    const int b = blockIdx.y;
    if (!bk->field_dst) return;
    float* dst = bk->field_dst[b];
    if (!dst) return;
    const int64_t n = (int64_t)2 * bk->H * bk->W;
    const float4* src = reinterpret_cast<const float4*>(bk->field[bk->state[b].cur] + (int64_t)b * n);
    if ((reinterpret_cast<uintptr_t>(dst) & 15) == 0 && (n & 3) == 0) {
        float4* d4 = reinterpret_cast<float4*>(dst);
        for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n / 4;
             t += (int64_t)gridDim.x * blockDim.x)
            d4[t] = src[t];
    } else {
        const float* s1 = reinterpret_cast<const float*>(src);
        for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
             t += (int64_t)gridDim.x * blockDim.x)
            dst[t] = s1[t];
    }
}

// Stand-alone normalisation: one block per pattern computes the statistics
// and writes the normalised pattern.
__global__ void __launch_bounds__(kStatThreads)
    k_stage_norm(const float* __restrict__ in, int64_t elems, float* __restrict__ out,
                 uint32_t* __restrict__ flags)
{
    __shared__ double sh[kStatThreads];
    __shared__ PatStat st;
    const int p = blockIdx.x;
    const float* src = in + (int64_t)p * elems;
    float* dst = out + (int64_t)p * elems;
    pattern_stats(src, elems, &st, sh);
    __syncthreads();
    const PatStat s = st;
    const int64_t nv = (((uintptr_t)src | (uintptr_t)dst) & 15) == 0 ? elems / 4 : 0;
    const float4* __restrict__ s4 = reinterpret_cast<const float4*>(src);
    float4* __restrict__ d4 = reinterpret_cast<float4*>(dst);
    auto nz = [&s](float v) { return s.flags ? 0.0f : (float)(((double)v - s.mean) * s.inv_std); };
    int64_t i = threadIdx.x;
    for (; i + kStatThreads < nv; i += 2 * kStatThreads) {
        const float4 a = s4[i], b = s4[i + kStatThreads];
        d4[i] = make_float4(nz(a.x), nz(a.y), nz(a.z), nz(a.w));
        d4[i + kStatThreads] = make_float4(nz(b.x), nz(b.y), nz(b.z), nz(b.w));
    }
    for (; i < nv; i += kStatThreads) {
        const float4 a = s4[i];
        d4[i] = make_float4(nz(a.x), nz(a.y), nz(a.z), nz(a.w));
    }
    for (int64_t j = 4 * nv + threadIdx.x; j < elems; j += kStatThreads) dst[j] = nz(src[j]);
    if (flags && threadIdx.x == 0) flags[p] = s.flags;
}

inline unsigned grid_for(int64_t n, int per_pattern_max = 1024)
{
    int64_t g = (n + 255) / 256;
    if (g > per_pattern_max) g = per_pattern_max;
    if (g < 1) g = 1;
    return (unsigned)g;
}

}  // namespace

hipError_t launch_stats(const Bucket* d_bk, int nb, int nref, hipStream_t s)
{
    hipLaunchKernelGGL(k_stats, dim3(nb + nref), dim3(kStatThreads), 0, s, d_bk);
    return hipGetLastError();
}

hipError_t launch_pyramids(const Bucket* d_bk, const Bucket& hb, hipStream_t s)
{
    const int npat = hb.nb + hb.nref;
    int64_t n0 = (int64_t)hb.H * hb.W;
    hipLaunchKernelGGL(k_normalize_l0, dim3(grid_for(n0, 64), npat), dim3(256), 0, s, d_bk);
    for (int l = 1; l < hb.L; l++) {
        int64_t n = (int64_t)hb.lh[l] * hb.lw[l];
        hipLaunchKernelGGL(k_restrict_level, dim3(grid_for(n, 64), npat), dim3(256), 0, s, d_bk, l);
    }
    return hipGetLastError();
}

hipError_t launch_demons_init(const Bucket* d_bk, const Bucket& hb, hipStream_t s)
{
    int64_t n = (int64_t)2 * hb.lh[hb.L - 1] * hb.lw[hb.L - 1];
    hipLaunchKernelGGL(k_demons_init, dim3(grid_for(n, 64), hb.nb), dim3(256), 0, s, d_bk);
    return hipGetLastError();
}

hipError_t launch_prolong_level(const Bucket* d_bk, const Bucket& hb, int level, hipStream_t s)
{
    int64_t n = (int64_t)2 * hb.lh[level - 1] * hb.lw[level - 1];
    hipLaunchKernelGGL(k_prolong_level, dim3(grid_for(n, 128), hb.nb), dim3(256), 0, s, d_bk, level);
    hipLaunchKernelGGL(k_rearm, dim3((hb.nb + 255) / 256), dim3(256), 0, s, d_bk);
    return hipGetLastError();
}

hipError_t launch_sample_q1(const Bucket* d_bk, const Bucket& hb, hipStream_t s)
{
    int n = hb.nb * hb.n_roi;
    hipLaunchKernelGGL(k_sample_q1, dim3((n + 255) / 256), dim3(256), 0, s, d_bk);
    return hipGetLastError();
}

BandTaps make_band_taps(double lo, double hi)
{
    BandTaps tp;
    auto fill = [](double sigma, float* w) -> int {
        if (!(sigma > 0.0)) return -1;
        const int r = (int)std::floor(3.0 * sigma + 0.5);
        double t[2 * kBandMaxR + 1], sum = 0.0;
        for (int j = -r; j <= r; j++) sum += (t[j + r] = std::exp(-(double)(j * j) / (2.0 * sigma * sigma)));
        for (int j = 0; j <= 2 * r; j++) w[j] = (float)(t[j] / sum);
        return r;
    };
    for (int j = 0; j <= 2 * kBandMaxR; j++) tp.lo[j] = tp.hi[j] = 0.0f;
    tp.rlo = fill(lo, tp.lo);
    tp.rhi = fill(hi, tp.hi);
    return tp;
}

hipError_t launch_bandpass(const BandIO& io, const BandTaps& tp, hipStream_t s)
{
    if (io.npat <= 0) return hipSuccess;
    if (io.W > 16384 || io.H > 65535 || io.npat > 65535 || tp.rlo > kBandMaxR || tp.rhi > kBandMaxR)
        return hipErrorInvalidValue;
    const size_t lds = sizeof(float) * (size_t)io.W;  // <= 64 KiB
    hipLaunchKernelGGL(k_band_rows, dim3((unsigned)io.H, (unsigned)io.npat), dim3(256), lds, s, io, tp);
    hipLaunchKernelGGL(k_band_cols, dim3(grid_for((int64_t)io.H * io.W, 256), (unsigned)io.npat), dim3(256), 0, s,
                       io, tp);
    return hipGetLastError();
}

hipError_t launch_mean_pattern(const float* const* src, int nb, int64_t hw, float* bg, hipStream_t s)
{
    if (nb <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mean_pattern, dim3(grid_for(hw, 4096)), dim3(256), 0, s, src, nb, hw, bg);
    return hipGetLastError();
}

hipError_t launch_bg_static(const BandIO& io, const float* bg, hipStream_t s)
{
    if (io.npat <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bg_static, dim3(grid_for((int64_t)io.H * io.W, 256), (unsigned)io.npat), dim3(256), 0, s,
                       io, bg);
    return hipGetLastError();
}

hipError_t launch_bg_dynamic(const BandIO& io, const float* blur, hipStream_t s)
{
    if (io.npat <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bg_dynamic, dim3(grid_for((int64_t)io.H * io.W, 256), (unsigned)io.npat), dim3(256), 0, s,
                       io, blur);
    return hipGetLastError();
}

int ssim_tiles(int H, int W)
{
    if (H <= 2 * kSsimR || W <= 2 * kSsimR) return 0;
    return ((W - 2 * kSsimR + kSsimT - 1) / kSsimT) * ((H - 2 * kSsimR + kSsimT - 1) / kSsimT);
}

hipError_t launch_ssim(const Bucket* d_bk, const Bucket& hb, hipStream_t s)
{
    const int tiles = ssim_tiles(hb.H, hb.W);
    if (!hb.ssim || !hb.ssim_part || tiles == 0 || hb.nb > 65535) return hipErrorInvalidValue;
    const int tiles_x = (hb.W - 2 * kSsimR + kSsimT - 1) / kSsimT;
    hipLaunchKernelGGL(k_ssim_tiles, dim3((unsigned)tiles, (unsigned)hb.nb), dim3(256), 0, s, d_bk, tiles_x);
    hipLaunchKernelGGL(k_ssim_finish, dim3((hb.nb + 63) / 64), dim3(64), 0, s, d_bk, tiles);
    return hipGetLastError();
}

hipError_t launch_zero_iters(const Bucket* d_bk, const Bucket& hb, hipStream_t s)
{
    const int64_t n = (int64_t)hb.nb * hb.L;
    hipLaunchKernelGGL(k_zero_iters, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d_bk);
    return hipGetLastError();
}

hipError_t launch_copy_field(const Bucket* d_bk, const Bucket& hb, hipStream_t s)
{
    int64_t n = (int64_t)2 * hb.H * hb.W / 4;
    hipLaunchKernelGGL(k_copy_field, dim3(grid_for(n, 64), hb.nb), dim3(256), 0, s, d_bk);
    return hipGetLastError();
}

hipError_t launch_stage_normalize(const float* in, int n, int64_t elems, float* out,
                                  uint32_t* flags, hipStream_t s)
{
    hipLaunchKernelGGL(k_stage_norm, dim3(n), dim3(kStatThreads), 0, s, in, elems, out, flags);
    return hipGetLastError();
}

hipError_t launch_stage_restrict(const float* in, int n, int H, int W, float* out, hipStream_t s)
{
    int64_t m = (int64_t)((H + 1) / 2) * ((W + 1) / 2);
    hipLaunchKernelGGL(k_restrict_plain, dim3(grid_for(m, 64), n), dim3(256), 0, s, in, H, W, out);
    return hipGetLastError();
}

hipError_t launch_stage_prolong(const float* u, int n, int h, int w, float* out, hipStream_t s)
{
    int64_t m = (int64_t)2 * 4 * h * w;
    hipLaunchKernelGGL(k_prolong_plain, dim3(grid_for(m, 128), n), dim3(256), 0, s, u, h, w, out);
    return hipGetLastError();
}

}  // namespace ebsd
