// ROI cross-correlation of the second pass for gfx950 (arXiv:1907.05993,
// section 2: zero-mean ROIs, Hann window, FFT, test spectrum times the
// conjugate reference spectrum, inverse FFT, interpolated peak; the reference
// is first remapped by R_finite, the step before Eq. (12)).
//
// One 256-thread workgroup per (pair, ROI), N in {32, 64, 128}:
//   gather   reference ROI remapped on the fly, Rm(x') = R0(pi(R_finite^T r(x'))),
//            interpolated by the cubic B-spline (the paper's cubic scheme,
//            coefficients from k_bspline_rows / k_bspline_cols) or bilinearly, and test ROI,
//            packed as z = a + i b (one complex FFT serves both);
//   window   per-ROI mean removed, symmetric Hann window h (x) h;
//   FFT      2-D radix-2 in LDS, three stages per pass in registers:
//            decimation-in-frequency forward (natural in, bit-reversed out),
//            so no explicit permutation is needed;
//   product  P(k) = B(k) conj A(k) with A = (Z(k) + conj Z(-k))/2 and
//            B = (Z(k) - conj Z(-k))/(2i), computed in the bit-reversed domain;
//   inverse  decimation-in-time (bit-reversed in, natural out), scaled 1/N^2;
//   peak     argmax of Re C (ties: lowest row-major index), wrap k >= N/2 to
//            k - N, 2-D quadratic fit on the 3 x 3 circular neighbourhood,
//            peak height C0 / sqrt(sum (a)^2 sum (b)^2).
// The N x N complex tile (padded rows) is LDS resident: 132 KiB at N = 128.
// Twiddles and the window are evaluated per block in FP64 and rounded.
#include <algorithm>

#include "ebsd_internal.h"

namespace ebsd {

namespace {

constexpr int NT = 256;

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

template <int N>
struct Log2;
template <>
struct Log2<32> { static constexpr int v = 5; };
template <>
struct Log2<64> { static constexpr int v = 6; };
template <>
struct Log2<128> { static constexpr int v = 7; };

template <int N>
__device__ inline int brev(int i)
{
    return (int)(__brev((unsigned)i) >> (32 - Log2<N>::v));
}

__device__ inline float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline float2 cmulc(float2 a, float2 b)  // a * conj(b)
{
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

// Bilinear sample at double-precision coordinates, clamped to the image.
__device__ inline float bilinear_d(const float* __restrict__ img, int h, int w, double x, double y)
{
    double xc = fmin(fmax(x, 0.0), (double)(w - 1));
    double yc = fmin(fmax(y, 0.0), (double)(h - 1));
    int x0 = clampi((int)floor(xc), 0, w - 1), y0 = clampi((int)floor(yc), 0, h - 1);
    float fx = (float)(xc - (double)x0), fy = (float)(yc - (double)y0);
    int x1 = min(x0 + 1, w - 1), y1 = min(y0 + 1, h - 1);
    const float* r0 = img + (int64_t)y0 * w;
    const float* r1 = img + (int64_t)y1 * w;
    float top = (1.0f - fx) * r0[x0] + fx * r0[x1];
    float bot = (1.0f - fx) * r1[x0] + fx * r1[x1];
    return (1.0f - fy) * top + fy * bot;
}

// Whole-sample mirror of an index at most n - 1 outside [0, n - 1] (n >= 2).
__device__ inline int mirror1(int i, int n)
{
    i = i < 0 ? -i : i;
    return i > n - 1 ? 2 * n - 2 - i : i;
}

// Cubic B-spline interpolant with coefficients c (h x w, whole-sample mirror
// extension) at double-precision coordinates clamped to the image: weights
// beta3(t + 1), beta3(t), beta3(t - 1), beta3(t - 2) on the four nodes
// floor(x) - 1 .. floor(x) + 2 per axis.  Needs w, h >= 3.
__device__ inline float bspline_d(const float* __restrict__ c, int h, int w, double x, double y)
{
    const double xc = fmin(fmax(x, 0.0), (double)(w - 1));
    const double yc = fmin(fmax(y, 0.0), (double)(h - 1));
    const int ix = clampi((int)floor(xc), 0, w - 1), iy = clampi((int)floor(yc), 0, h - 1);
    const float tx = (float)(xc - (double)ix), ty = (float)(yc - (double)iy);
    float wx[4], wy[4];
    {
        const float t = tx, t2 = t * t, t3 = t2 * t, u = 1.0f - t;
        wx[0] = u * u * u * (1.0f / 6.0f);
        wx[1] = (3.0f * t3 - 6.0f * t2 + 4.0f) * (1.0f / 6.0f);
        wx[2] = (-3.0f * t3 + 3.0f * t2 + 3.0f * t + 1.0f) * (1.0f / 6.0f);
        wx[3] = t3 * (1.0f / 6.0f);
    }
    {
        const float t = ty, t2 = t * t, t3 = t2 * t, u = 1.0f - t;
        wy[0] = u * u * u * (1.0f / 6.0f);
        wy[1] = (3.0f * t3 - 6.0f * t2 + 4.0f) * (1.0f / 6.0f);
        wy[2] = (-3.0f * t3 + 3.0f * t2 + 3.0f * t + 1.0f) * (1.0f / 6.0f);
        wy[3] = t3 * (1.0f / 6.0f);
    }
    int cx[4];
#pragma unroll
    for (int k = 0; k < 4; k++) cx[k] = mirror1(ix - 1 + k, w);
    float acc = 0.0f;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const float* row = c + (int64_t)mirror1(iy - 1 + j, h) * w;
        float r = 0.0f;
#pragma unroll
        for (int k = 0; k < 4; k++) r += wx[k] * row[cx[k]];
        acc += wy[j] * r;
    }
    return acc;
}

// Cubic B-spline coefficients of images (whole-sample mirror extension).
// Along one line the coefficients are the samples filtered by the inverse of
// (1, 4, 1)/6: a causal recursion c+[k] = s[k] + z c+[k-1] followed by an
// anti-causal one c-[k] = z (c-[k+1] - c+[k]), c = 6 c-, pole z = sqrt(3) - 2.
// Each thread produces 32 consecutive outputs of one line: it starts the
// causal recursion 16 samples before its block and the anti-causal one 16
// after it, both from zero, on the mirror-extended line; the starting values
// it drops weigh |z|^16 < 7.1e-10 (times at most 1.4 max|s|), so the result
// equals the exact filtering of the mirror extension to FP32 rounding.  Rows
// first (image -> tmp), then columns (tmp -> dst); consecutive lanes take
// consecutive rows (row pass) or columns (column pass).
constexpr int kCoefB = 32, kCoefWarm = 16;

// Whole-sample mirror of any index into [0, n - 1].
__device__ inline int mirror_any(int i, int n)
{
    if (n == 1) return 0;
    const int P = 2 * n - 2;
    int m = i % P;
    m = m < 0 ? m + P : m;
    return m < n ? m : P - m;
}

// One line of n samples at stride `st` (elements) from `in` into `out`,
// outputs a .. a + kCoefB - 1 (those inside the line).
__device__ inline void bspline_line_block(const float* __restrict__ in, float* __restrict__ out, int n, int64_t st,
                                          int a)
{
    const float z = -0.267949192431122706f;  // sqrt(3) - 2
    float cp = 0.0f, buf[kCoefB + kCoefWarm];
    if (n > kCoefWarm + kCoefB) {
        // one reflection covers indices a - 16 .. a + 47 (a <= n - 1)
#pragma unroll
        for (int j = 0; j < kCoefB + 3 * kCoefWarm; j++) {
            int k = a - kCoefWarm + j;
            k = k < 0 ? -k : (k > n - 1 ? 2 * n - 2 - k : k);
            cp = in[(int64_t)k * st] + z * cp;
            if (j >= kCoefWarm) buf[j - kCoefWarm] = cp;
        }
    } else {
#pragma unroll
        for (int j = 0; j < kCoefB + 3 * kCoefWarm; j++) {
            cp = in[(int64_t)mirror_any(a - kCoefWarm + j, n) * st] + z * cp;
            if (j >= kCoefWarm) buf[j - kCoefWarm] = cp;
        }
    }
    float cm = 0.0f;
#pragma unroll
    for (int j = kCoefB + kCoefWarm - 1; j >= 0; j--) {
        cm = z * (cm - buf[j]);
        if (j < kCoefB && a + j < n) out[(int64_t)(a + j) * st] = 6.0f * cm;
    }
}

// Row pass: a workgroup stages nr rows of one image in LDS with coalesced
// loads (row pitch W + 1 words: the lanes of a wavefront, which walk
// different rows, hit different banks), runs the recursions of every
// (row, 32-column block) from LDS into a second LDS copy, and stores it
// coalesced.  grid (ceil(H / nr), images); dynamic LDS 2 nr (W + 1) words.
constexpr int kCoefRows = 32;
constexpr int kCoefLdsWords = 40960;  // 160 KiB

__global__ void __launch_bounds__(256)
    k_bspline_rows(const float* __restrict__ src_all, int64_t src_stride, float* __restrict__ tmp_all, int H, int W,
                   int nr)
{
    extern __shared__ float lds[];
    const int P = W + 1;
    float* sin = lds;
    float* sout = lds + nr * P;
    const int y0 = blockIdx.x * nr, img = blockIdx.y;
    const int rows = min(nr, H - y0);
    const float* src = src_all + img * src_stride + (int64_t)y0 * W;
    float* dst = tmp_all + ((int64_t)img * H + y0) * W;
    for (int r = 0; r < rows; r++)
        for (int x = threadIdx.x; x < W; x += blockDim.x) sin[r * P + x] = src[(int64_t)r * W + x];
    __syncthreads();
    const int nblk = (W + kCoefB - 1) / kCoefB;
    for (int t = threadIdx.x; t < rows * nblk; t += blockDim.x) {
        const int r = t % rows, blk = t / rows;
        bspline_line_block(sin + r * P, sout + r * P, W, 1, blk * kCoefB);
    }
    __syncthreads();
    for (int r = 0; r < rows; r++)
        for (int x = threadIdx.x; x < W; x += blockDim.x) dst[(int64_t)r * W + x] = sout[r * P + x];
}

// thread = (image, row block, column), columns fastest
__global__ void __launch_bounds__(256)
    k_bspline_cols(const float* __restrict__ tmp_all, float* __restrict__ dst_all, int nimg, int H, int W)
{
    const int nblk = (H + kCoefB - 1) / kCoefB;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nimg * nblk * W) return;
    const int x = (int)(t % W);
    const int64_t r = t / W;
    const int blk = (int)(r % nblk), img = (int)(r / nblk);
    const int64_t o = (int64_t)img * H * W + x;
    bspline_line_block(tmp_all + o, dst_all + o, H, W, blk * kCoefB);
}

// Coefficients of n images (image i at src + i src_stride, H x W) into dst
// [n][H][W]; tmp [n][H][W] holds the row pass.
hipError_t launch_coef_images(const float* src, int64_t src_stride, int n, int H, int W, float* dst, float* tmp,
                              hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t tc = (int64_t)n * W * ((H + kCoefB - 1) / kCoefB);
    const int nr = std::max(1, std::min(kCoefRows, kCoefLdsWords / (2 * (W + 1))));
    if (2 * nr * (W + 1) > kCoefLdsWords) return hipErrorInvalidValue;  // rows longer than 20479 samples
    const size_t lds = sizeof(float) * 2 * nr * (size_t)(W + 1);
    static std::atomic<uint64_t> attr_done{0};
    const hipError_t e =
        ensure_dynamic_lds((const void*)k_bspline_rows, (int)(sizeof(float) * kCoefLdsWords), attr_done);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bspline_rows, dim3((unsigned)((H + nr - 1) / nr), (unsigned)n), dim3(256), lds, s, src,
                       src_stride, tmp, H, W, nr);
    hipLaunchKernelGGL(k_bspline_cols, dim3((unsigned)((tc + 255) / 256)), dim3(256), 0, s, tmp, dst, n, H, W);
    return hipGetLastError();
}

// Whole-image remap Rm(x') = I(pi(R^T r(x'))) of n images (stage entry):
// INTERP 3 samples the cubic B-spline with coefficients `img`, 1 samples
// `img` bilinearly.  grid (ceil(W / 64), H, n), 64 threads per row segment.
template <int INTERP>
__global__ void __launch_bounds__(64)
    k_remap_stage(const float* __restrict__ img_all, int n, int H, int W, const double* __restrict__ Rall,
                  double xs, double ys, double zs, float* __restrict__ out)
{
    const int x = blockIdx.x * 64 + threadIdx.x, y = blockIdx.y, i = blockIdx.z;
    if (x >= W || i >= n) return;
    const double* Rf = Rall + 9 * (int64_t)i;
    const float* img = img_all + (int64_t)i * H * W;
    const double p0 = (double)x - xs, p1 = (double)y - ys, p2 = zs;
    const double v0 = Rf[0] * p0 + Rf[3] * p1 + Rf[6] * p2;
    const double v1 = Rf[1] * p0 + Rf[4] * p1 + Rf[7] * p2;
    const double v2 = Rf[2] * p0 + Rf[5] * p1 + Rf[8] * p2;
    const double sx = xs + zs * v0 / v2, sy = ys + zs * v1 / v2;
    out[((int64_t)i * H + y) * W + x] = INTERP == 3 ? bspline_d(img, H, W, sx, sy) : bilinear_d(img, H, W, sx, sy);
}

template <int N>
struct XcfShared {
    float2 z[N][N + 1];
    float2 tw[N / 2];
    float win[N];
    float red[4][NT / 64];
    float bv[NT / 64];
    int bi[NT / 64];
};

// Block sum of up to four floats per thread (fixed order), broadcast to all.
__device__ inline void block_sum4(float v[4], float (*red)[NT / 64], int k)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int q = 0; q < k; q++) {
        float s = v[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if (lane == 0) red[q][wv] = s;
    }
    __syncthreads();
    for (int q = 0; q < k; q++) {
        float s = 0.0f;
#pragma unroll
        for (int i = 0; i < NT / 64; i++) s += red[q][i];
        v[q] = s;
    }
    __syncthreads();
}

// Radix-2 butterflies, up to three stages per pass held in registers: a pass
// takes the stages of half-size s, 2s, .., s 2^(R-1) (s = 2^SL); each task owns
// the 2^R elements base + m s of one row (ROWS) or column, base = g 2^R s + t,
// t < s.  Every butterfly is the one the stage-by-stage transform computes
// (same operands, same twiddle tw[(i0 mod h) N / 2h]), so the values are
// those of one LDS pass per stage, with a third of the LDS traffic and
// barriers.  Forward: decimation in frequency (stages from N/2 down to 1);
// inverse: decimation in time with conjugate twiddles (from 1 up to N/2).
// Consecutive threads take consecutive lines, so a wavefront's accesses of
// one element fall in distinct banks (row pitch N + 1) or are contiguous.
struct NoHook {
    __device__ void operator()(int, int, float2&) const {}
};

// pre(line, index, v) runs on each element after it is loaded, post(line,
// index, v) on each result before it is stored (index along the line).
template <int N, bool DIF, bool ROWS, int SL, int R, class Pre = NoHook, class Post = NoHook>
__device__ void fft_pass(XcfShared<N>& S, Pre pre = Pre(), Post post = Post())
{
    constexpr int s = 1 << SL, M = 1 << R, span = M * s;
    constexpr int per_line = N / M;
    for (int c = threadIdx.x; c < N * per_line; c += NT) {
        const int line = c % N, k = c / N;
        const int t = k % s, g = k / s;
        const int base = g * span + t;
        float2 v[M];
#pragma unroll
        for (int m = 0; m < M; m++) {
            v[m] = ROWS ? S.z[line][base + m * s] : S.z[base + m * s][line];
            pre(line, base + m * s, v[m]);
        }
        // every loop below is unrolled: stage sizes and element indices are constants
#pragma unroll
        for (int r = 0; r < R; r++) {
            const int e = DIF ? R - 1 - r : r;
            const int hs = 1 << e;  // h / s
            const int h = hs * s;
            const int step = N / (2 * h);
#pragma unroll
            for (int m = 0; m < M; m++) {
                if (m & hs) continue;
                const float2 w = S.tw[(t + (m * s) % h) * step];
                const float2 a = v[m];
                if (DIF) {
                    const float2 b = v[m + hs];
                    v[m] = make_float2(a.x + b.x, a.y + b.y);
                    v[m + hs] = cmul(make_float2(a.x - b.x, a.y - b.y), w);
                } else {
                    const float2 b = cmulc(v[m + hs], w);
                    v[m] = make_float2(a.x + b.x, a.y + b.y);
                    v[m + hs] = make_float2(a.x - b.x, a.y - b.y);
                }
            }
        }
#pragma unroll
        for (int m = 0; m < M; m++) {
            post(line, base + m * s, v[m]);
            if (ROWS) S.z[line][base + m * s] = v[m];
            else S.z[base + m * s][line] = v[m];
        }
    }
    __syncthreads();
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// Forward stages E .. 0 (half-size 2^E down to 1), three per pass; `pre`
// runs in the first pass only.
template <int N, bool ROWS, int E, class Pre = NoHook>
__device__ void fft_dif_from(XcfShared<N>& S, Pre pre = Pre())
{
    constexpr int R = E + 1 < 3 ? E + 1 : 3;
    fft_pass<N, true, ROWS, E - R + 1, R>(S, pre);
    if constexpr (E - R >= 0) fft_dif_from<N, ROWS, E - R>(S);
}

// Inverse stages E .. log2(N) - 1 (half-size 2^E up to N / 2), three per pass;
// `post` runs in the last pass only.
template <int N, bool ROWS, int E, class Post = NoHook>
__device__ void fft_dit_from(XcfShared<N>& S, Post post = Post())
{
    constexpr int LOGN = ilog2(N);
    constexpr int R = LOGN - E < 3 ? LOGN - E : 3;
    if constexpr (E + R < LOGN) {
        fft_pass<N, false, ROWS, E, R>(S);
        fft_dit_from<N, ROWS, E + R>(S, post);
    } else {
        fft_pass<N, false, ROWS, E, R, NoHook, Post>(S, NoHook(), post);
    }
}

// The whole correlation for one ROI.  `load(x, y)` returns (reference, test)
// at ROI pixel (x, y).  Writes q (x, y) and ph from thread 0.
// 2-D quadratic fit of the correlation peak from its circular 3 x 3
// neighbourhood, C(dy, dx) around the integer maximum (ky, kx); q = wrapped
// integer shift plus the fit, ph = C0 / sqrt(ea eb).
template <int N, class At>
__device__ void peak_fit(At C, int ky, int kx, float ea, float eb, float* q, float* ph)
{
    const double c0 = C(0, 0);
    const double gx = 0.5 * (C(0, 1) - C(0, -1));
    const double gy = 0.5 * (C(1, 0) - C(-1, 0));
    const double hxx = C(0, 1) - 2.0 * c0 + C(0, -1);
    const double hyy = C(1, 0) - 2.0 * c0 + C(-1, 0);
    const double hxy = 0.25 * (C(1, 1) - C(1, -1) - C(-1, 1) + C(-1, -1));
    const double det = hxx * hyy - hxy * hxy;
    double dx = 0.0, dy = 0.0;
    if (hxx < 0.0 && det > 0.0) {
        dx = fmin(fmax(-(hyy * gx - hxy * gy) / det, -1.0), 1.0);
        dy = fmin(fmax(-(hxx * gy - hxy * gx) / det, -1.0), 1.0);
    }
    const int sx = kx < N / 2 ? kx : kx - N;
    const int sy = ky < N / 2 ? ky : ky - N;
    q[0] = (float)((double)sx + dx);
    q[1] = (float)((double)sy + dy);
    if (ph) {
        const double nrm = sqrt((double)ea * (double)eb);
        *ph = nrm > 0.0 ? (float)(c0 / nrm) : 0.0f;
    }
}

template <int N, class Loader>
__device__ void xcf_core(XcfShared<N>& S, Loader load, int window, float* q, float* ph)
{
    const int tid = threadIdx.x;
    for (int k = tid; k < N / 2; k += NT) {
        double s, c;
        sincospi(-2.0 * (double)k / (double)N, &s, &c);
        S.tw[k] = make_float2((float)c, (float)s);
    }
    for (int n = tid; n < N; n += NT)
        S.win[n] = window ? (float)(0.5 - 0.5 * cospi(2.0 * (double)n / (double)(N - 1))) : 1.0f;

    // gather + means
    float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int p = tid; p < N * N; p += NT) {
        const int y = p / N, x = p - y * N;
        float2 ab = load(x, y);
        S.z[y][x] = ab;
        acc[0] += ab.x;
        acc[1] += ab.y;
    }
    block_sum4(acc, S.red, 2);
    const float ma = acc[0] / (float)(N * N), mb = acc[1] / (float)(N * N);

    // forward transform; its first pass removes the means, applies the window
    // and sums the energies of the windowed ROIs
    float en0 = 0.0f, en1 = 0.0f;
    fft_dif_from<N, true, ilog2(N) - 1>(S, [&](int y, int x, float2& ab) {
        const float wgt = S.win[y] * S.win[x];
        const float a = (ab.x - ma) * wgt, b = (ab.y - mb) * wgt;
        ab = make_float2(a, b);
        en0 += a * a;
        en1 += b * b;
    });
    fft_dif_from<N, false, ilog2(N) - 1>(S);

    // cross-power spectrum in the bit-reversed domain
    const float scale = 1.0f / (float)(N * N);
    for (int p = tid; p < N * N; p += NT) {
        const int py = p / N, px = p - py * N;
        const int ky = brev<N>(py), kx = brev<N>(px);
        const int qy = brev<N>((N - ky) & (N - 1)), qx = brev<N>((N - kx) & (N - 1));
        const int qi = qy * N + qx;
        if (qi < p) continue;
        float2 z1 = S.z[py][px], z2 = S.z[qy][qx];
        // A = (z1 + conj z2)/2, B = (z1 - conj z2)/(2i)
        float2 A = make_float2(0.5f * (z1.x + z2.x), 0.5f * (z1.y - z2.y));
        float2 B = make_float2(0.5f * (z1.y + z2.y), -0.5f * (z1.x - z2.x));
        float2 P = cmulc(B, A);
        P.x *= scale;
        P.y *= scale;
        if (qi == p) {
            S.z[py][px] = make_float2(P.x, 0.0f);
        } else {
            S.z[py][px] = P;
            S.z[qy][qx] = make_float2(P.x, -P.y);
        }
    }
    __syncthreads();

    // inverse transform; its last pass also takes each thread's argmax of Re C
    // (ties to the lowest row-major index; NaNs never win)
    float bv = -INFINITY;
    int bi = 0x7fffffff;
    fft_dit_from<N, false, 0>(S);
    fft_dit_from<N, true, 0>(S, [&](int y, int x, float2& c) {
        const int p = y * N + x;
        if (c.x > bv || (c.x == bv && p < bi)) {
            bv = c.x;
            bi = p;
        }
    });
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        float ov = __shfl_xor(bv, off, 64);
        int oi = __shfl_xor(bi, off, 64);
        if (ov > bv || (ov == bv && oi < bi)) {
            bv = ov;
            bi = oi;
        }
        en0 += __shfl_xor(en0, off, 64);
        en1 += __shfl_xor(en1, off, 64);
    }
    const int lane = tid & 63, wv = tid >> 6;
    if (lane == 0) {
        S.bv[wv] = bv;
        S.bi[wv] = bi;
        S.red[0][wv] = en0;
        S.red[1][wv] = en1;
    }
    __syncthreads();
    if (tid == 0) {
        float ea = 0.0f, eb = 0.0f;
#pragma unroll
        for (int i = 0; i < NT / 64; i++) {
            ea += S.red[0][i];
            eb += S.red[1][i];
        }
        bv = S.bv[0];
        bi = S.bi[0];
        for (int i = 1; i < NT / 64; i++)
            if (S.bv[i] > bv || (S.bv[i] == bv && S.bi[i] < bi)) {
                bv = S.bv[i];
                bi = S.bi[i];
            }
        if (bi < 0 || bi >= N * N) bi = 0;  // all-NaN correlation
        const int ky = bi / N, kx = bi - ky * N;
        auto C = [&](int dy, int dx) -> double {
            return (double)S.z[(ky + dy + N) & (N - 1)][(kx + dx + N) & (N - 1)].x;
        };
        peak_fit<N>(C, ky, kx, ea, eb, q, ph);
    }
}

// ---- ROIs of 256 x 256 (the paper's ROI size) ----------------------------------
// The 256 x 256 complex tile (512 KiB) does not fit in LDS, so one workgroup
// per ROI keeps it in a slot of global scratch (L2 / MALL resident while the
// workgroup works on it) and moves 32 lines at a time through an LDS tile:
//   gather   z = a + i b of the ROI (remapped reference, test) into the slot,
//            natural order, and the two means;
//   rows     per 32 rows: mean removed, Hann window, energies, forward
//            transform along x (decimation in frequency: bit-reversed out),
//            written back in that order;
//   columns  per 32 physical columns: forward transform along y, the cross
//            power spectrum P(k) = B(k) conj A(k) (A, B separated from Z(k)
//            and Z(-k) as for the smaller ROIs), inverse transform along y;
//            the physical columns of a chunk are two blocks of 16 chosen so
//            that the partner -k of every element lies in the same chunk (bit
//            reversal of 8 bits maps the block of physical columns 16 j .. 16 j + 15 of
//            logical kx = 16 rev4(i) + rev4(j) onto the block rev4((16 -
//            rev4(j)) mod 16) of the partners -kx; blocks 0 and 1 are their own
//            partners, the others pair up);
//   inverse  per 32 rows: inverse transform along x (bit-reversed in, natural
//            out), the real part into the slot's correlation plane, each
//            thread's argmax (ties to the lowest row-major index);
// then the block's argmax and the 2-D quadratic fit of its neighbourhood.
// Every butterfly is the one the LDS-resident kernels compute for N = 256.
constexpr int kX2 = 256, kX2Lines = 32, kX2Pitch = kX2 + 1;
constexpr int64_t kX2SlotFloats = (int64_t)2 * kX2 * kX2 + (int64_t)kX2 * kX2;  // complex tile + real plane
constexpr int kX2Slots = 512;  // workgroups (two per compute unit at 68 KiB of LDS each)

struct Xcf256Shared {
    float2 t[kX2Lines][kX2Pitch];
    float2 tw[kX2 / 2];
    float win[kX2];
    float red[4][NT / 64];
    float bv[NT / 64];
    int bi[NT / 64];
};

__device__ inline int rev4(int v) { return (int)(__brev((unsigned)v) >> 28); }
__device__ inline int rev8(int v) { return (int)(__brev((unsigned)v) >> 24); }

// Radix-2 butterflies over the kX2Lines lines of the LDS tile (length 256),
// up to three stages per pass in registers; the same butterflies and twiddles
// as fft_pass.  Consecutive threads take consecutive lines.
template <bool DIF, int SL, int R>
__device__ void line_pass(Xcf256Shared& S)
{
    constexpr int N = kX2;
    constexpr int s = 1 << SL, M = 1 << R, span = M * s;
    constexpr int per_line = N / M;
    for (int c = threadIdx.x; c < kX2Lines * per_line; c += NT) {
        const int line = c % kX2Lines, k = c / kX2Lines;
        const int t = k % s, g = k / s;
        const int base = g * span + t;
        float2 v[M];
#pragma unroll
        for (int m = 0; m < M; m++) v[m] = S.t[line][base + m * s];
#pragma unroll
        for (int r = 0; r < R; r++) {
            const int e = DIF ? R - 1 - r : r;
            const int hs = 1 << e;
            const int h = hs * s;
            const int step = N / (2 * h);
#pragma unroll
            for (int m = 0; m < M; m++) {
                if (m & hs) continue;
                const float2 w = S.tw[(t + (m * s) % h) * step];
                const float2 a = v[m];
                if (DIF) {
                    const float2 b = v[m + hs];
                    v[m] = make_float2(a.x + b.x, a.y + b.y);
                    v[m + hs] = cmul(make_float2(a.x - b.x, a.y - b.y), w);
                } else {
                    const float2 b = cmulc(v[m + hs], w);
                    v[m] = make_float2(a.x + b.x, a.y + b.y);
                    v[m + hs] = make_float2(a.x - b.x, a.y - b.y);
                }
            }
        }
#pragma unroll
        for (int m = 0; m < M; m++) S.t[line][base + m * s] = v[m];
    }
    __syncthreads();
}

// forward: stages 7 .. 0 (half-sizes 128 down to 1) in passes of 3, 3, 2
__device__ inline void lines_dif(Xcf256Shared& S)
{
    line_pass<true, 5, 3>(S);
    line_pass<true, 2, 3>(S);
    line_pass<true, 0, 2>(S);
}
// inverse: stages 0 .. 7 in passes of 3, 3, 2
__device__ inline void lines_dit(Xcf256Shared& S)
{
    line_pass<false, 0, 3>(S);
    line_pass<false, 3, 3>(S);
    line_pass<false, 6, 2>(S);
}

// The physical column blocks of column chunk c (0..7): (0, 1), then the pairs
// (j, partner(j)) with j < partner(j) in increasing j.
__device__ inline void x2_chunk_blocks(int c, int& ba, int& bb)
{
    if (c == 0) {
        ba = 0;
        bb = 1;
        return;
    }
    int seen = 0;
    for (int j = 2; j < 16; j++) {
        const int pj = rev4((16 - rev4(j)) & 15);
        if (j < pj && ++seen == c) {
            ba = j;
            bb = pj;
            return;
        }
    }
    ba = bb = 0;  // not reached for c < 8
}

template <class Loader>
__device__ void xcf256_core(Xcf256Shared& S, float2* __restrict__ Z, float* __restrict__ Cr, Loader load,
                            int window, float* q, float* ph)
{
    constexpr int N = kX2, L = kX2Lines;
    const int tid = threadIdx.x;
    for (int k = tid; k < N / 2; k += NT) {
        double sn, cs;
        sincospi(-2.0 * (double)k / (double)N, &sn, &cs);
        S.tw[k] = make_float2((float)cs, (float)sn);
    }
    for (int n = tid; n < N; n += NT)
        S.win[n] = window ? (float)(0.5 - 0.5 * cospi(2.0 * (double)n / (double)(N - 1))) : 1.0f;

    // gather + means
    float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int p = tid; p < N * N; p += NT) {
        const float2 ab = load(p & (N - 1), p >> 8);
        Z[p] = ab;
        acc[0] += ab.x;
        acc[1] += ab.y;
    }
    block_sum4(acc, S.red, 2);  // its barriers also order the slot's writes before the reads below
    const float ma = acc[0] / (float)(N * N), mb = acc[1] / (float)(N * N);

    // rows: window, energies, forward transform
    float en0 = 0.0f, en1 = 0.0f;
    for (int r0 = 0; r0 < N; r0 += L) {
        for (int i = tid; i < L * N; i += NT) {
            const int line = i >> 8, x = i & (N - 1);
            const float2 ab = Z[(r0 + line) * N + x];
            const float wgt = S.win[r0 + line] * S.win[x];
            const float a = (ab.x - ma) * wgt, b = (ab.y - mb) * wgt;
            en0 += a * a;
            en1 += b * b;
            S.t[line][x] = make_float2(a, b);
        }
        __syncthreads();
        lines_dif(S);
        for (int i = tid; i < L * N; i += NT) {
            const int line = i >> 8, x = i & (N - 1);
            Z[(r0 + line) * N + x] = S.t[line][x];
        }
        __syncthreads();
    }

    // columns: forward transform, cross power spectrum, inverse transform
    const float scale = 1.0f / (float)(N * N);
    for (int c = 0; c < 8; c++) {
        int ba, bb;
        x2_chunk_blocks(c, ba, bb);
        for (int i = tid; i < L * N; i += NT) {
            const int y = i >> 5, l = i & (L - 1);
            const int px = (l < 16 ? ba : bb) * 16 + (l & 15);
            S.t[l][y] = Z[y * N + px];
        }
        __syncthreads();
        lines_dif(S);
        for (int i = tid; i < L * N; i += NT) {
            const int l = i >> 8, py = i & (N - 1);
            const int px = (l < 16 ? ba : bb) * 16 + (l & 15);
            const int ky = rev8(py), kx = rev8(px);
            const int qy = rev8((N - ky) & (N - 1)), qx = rev8((N - kx) & (N - 1));
            const int ql = ((qx >> 4) == ba ? 0 : 16) + (qx & 15);
            if (ql * N + qy < i) continue;  // each pair once
            const float2 z1 = S.t[l][py], z2 = S.t[ql][qy];
            const float2 A = make_float2(0.5f * (z1.x + z2.x), 0.5f * (z1.y - z2.y));
            const float2 B = make_float2(0.5f * (z1.y + z2.y), -0.5f * (z1.x - z2.x));
            float2 P = cmulc(B, A);
            P.x *= scale;
            P.y *= scale;
            if (ql * N + qy == i) {
                S.t[l][py] = make_float2(P.x, 0.0f);
            } else {
                S.t[l][py] = P;
                S.t[ql][qy] = make_float2(P.x, -P.y);
            }
        }
        __syncthreads();
        lines_dit(S);
        for (int i = tid; i < L * N; i += NT) {
            const int y = i >> 5, l = i & (L - 1);
            const int px = (l < 16 ? ba : bb) * 16 + (l & 15);
            Z[y * N + px] = S.t[l][y];
        }
        __syncthreads();
    }

    // rows: inverse transform, real part, argmax (NaNs never win)
    float bv = -INFINITY;
    int bi = 0x7fffffff;
    for (int r0 = 0; r0 < N; r0 += L) {
        for (int i = tid; i < L * N; i += NT) {
            const int line = i >> 8, x = i & (N - 1);
            S.t[line][x] = Z[(r0 + line) * N + x];
        }
        __syncthreads();
        lines_dit(S);
        for (int i = tid; i < L * N; i += NT) {
            const int line = i >> 8, x = i & (N - 1);
            const int p = (r0 + line) * N + x;
            const float v = S.t[line][x].x;
            Cr[p] = v;
            if (v > bv || (v == bv && p < bi)) {
                bv = v;
                bi = p;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const float ov = __shfl_xor(bv, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ov > bv || (ov == bv && oi < bi)) {
            bv = ov;
            bi = oi;
        }
        en0 += __shfl_xor(en0, off, 64);
        en1 += __shfl_xor(en1, off, 64);
    }
    const int lane = tid & 63, wv = tid >> 6;
    if (lane == 0) {
        S.bv[wv] = bv;
        S.bi[wv] = bi;
        S.red[0][wv] = en0;
        S.red[1][wv] = en1;
    }
    __syncthreads();
    if (tid == 0) {
        float ea = 0.0f, eb = 0.0f;
#pragma unroll
        for (int i = 0; i < NT / 64; i++) {
            ea += S.red[0][i];
            eb += S.red[1][i];
        }
        bv = S.bv[0];
        bi = S.bi[0];
        for (int i = 1; i < NT / 64; i++)
            if (S.bv[i] > bv || (S.bv[i] == bv && S.bi[i] < bi)) {
                bv = S.bv[i];
                bi = S.bi[i];
            }
        if (bi < 0 || bi >= N * N) bi = 0;  // all-NaN correlation
        const int ky = bi >> 8, kx = bi & (N - 1);
        auto C = [&](int dy, int dx) -> double { return (double)Cr[((ky + dy) & (N - 1)) * N + ((kx + dx) & (N - 1))]; };
        peak_fit<N>(C, ky, kx, ea, eb, q, ph);
    }
    __syncthreads();  // the slot is reused by the workgroup's next ROI
}

// One workgroup per (pair, ROI).  INTERP 3 / 1: the second pass, the
// reference remapped (cubic B-spline / bilinear) -> q2; INTERP 0: the
// conventional first pass, the unremapped reference ROI -> q1.  Both write
// the peak height.
// The (reference, test) sample at pixel (x, y) of ROI j of pair b.  INTERP 3 /
// 1: the reference remapped (cubic B-spline / bilinear); pass 0 remaps by
// R_finite (source direction R^T r), a later pass by the previous pass's F
// (source direction F^-1 r: the same map with (F^-1)^T = cofactor(F) / det F
// in place of R).  INTERP 0: the unremapped reference.
template <int INTERP>
struct RoiLoader {
    const float* Rn;
    const float* Tn;
    const float* Cf;
    int H, W, x0, y0;
    double r00, r01, r02, r10, r11, r12, r20, r21, r22, xs, ys, zs;

    __device__ RoiLoader(const Bucket* __restrict__ bk, int b, int j, int pass)
    {
        H = bk->H;
        W = bk->W;
        Rn = bk->ref_pyr + (int64_t)bk->ref_slot[b] * bk->pyr_elems;
        Tn = bk->test_pyr + (int64_t)b * bk->pyr_elems;
        x0 = bk->roi_xy[2 * j];
        y0 = bk->roi_xy[2 * j + 1];
        Cf = INTERP == 3 ? bk->ref_coef + (int64_t)bk->ref_slot[b] * H * W : nullptr;
        double m[9];
        if (INTERP == 0) {
            for (int i = 0; i < 9; i++) m[i] = 0.0;  // unused
        } else if (pass == 0) {
            const double* Rf = bk->Rfin + 9 * (int64_t)b;
            for (int i = 0; i < 9; i++) m[i] = Rf[i];
        } else {
            const double* A = bk->F + 9 * (int64_t)b;
            m[0] = A[4] * A[8] - A[5] * A[7];
            m[1] = A[5] * A[6] - A[3] * A[8];
            m[2] = A[3] * A[7] - A[4] * A[6];
            m[3] = A[2] * A[7] - A[1] * A[8];
            m[4] = A[0] * A[8] - A[2] * A[6];
            m[5] = A[1] * A[6] - A[0] * A[7];
            m[6] = A[1] * A[5] - A[2] * A[4];
            m[7] = A[2] * A[3] - A[0] * A[5];
            m[8] = A[0] * A[4] - A[1] * A[3];
            const double det = A[0] * m[0] + A[1] * m[1] + A[2] * m[2];
            for (int i = 0; i < 9; i++) m[i] /= det;
        }
        r00 = m[0]; r01 = m[1]; r02 = m[2];
        r10 = m[3]; r11 = m[4]; r12 = m[5];
        r20 = m[6]; r21 = m[7]; r22 = m[8];
        xs = bk->xs;
        ys = bk->ys;
        zs = bk->zs;
    }

    __device__ float2 operator()(int x, int y) const
    {
        const int X = x0 + x, Y = y0 + y;
        if (INTERP == 0) return make_float2(Rn[(int64_t)Y * W + X], Tn[(int64_t)Y * W + X]);
        const double p0 = (double)X - xs, p1 = (double)Y - ys, p2 = zs;
        // v = R_finite^T r
        const double v0 = r00 * p0 + r10 * p1 + r20 * p2;
        const double v1 = r01 * p0 + r11 * p1 + r21 * p2;
        const double v2 = r02 * p0 + r12 * p1 + r22 * p2;
        const double sx = xs + zs * v0 / v2, sy = ys + zs * v1 / v2;
        const float a = INTERP == 3 ? bspline_d(Cf, H, W, sx, sy) : bilinear_d(Rn, H, W, sx, sy);
        return make_float2(a, Tn[(int64_t)Y * W + X]);
    }
};

// One workgroup per (pair, ROI).  INTERP 3 / 1: the second pass -> q2;
// INTERP 0: the conventional first pass -> q1.  Both write the peak height.
template <int N, int INTERP>
__global__ void __launch_bounds__(NT) k_xcf_pairs(const Bucket* __restrict__ bk, int window, int pass)
{
    extern __shared__ __align__(16) unsigned char smem[];
    XcfShared<N>& S = *reinterpret_cast<XcfShared<N>*>(smem);
    const int b = blockIdx.x / bk->n_roi;
    const int j = blockIdx.x - b * bk->n_roi;
    const RoiLoader<INTERP> load(bk, b, j, pass);
    const int64_t o = (int64_t)b * bk->n_roi + j;
    xcf_core<N>(S, load, window, (INTERP == 0 ? bk->q1 : bk->q2) + 2 * o, bk->ph + o);
}

// ROIs of 256: a grid of at most kX2Slots workgroups walks the (pair, ROI)
// list; workgroup g works in scratch slot g.
template <int INTERP>
__global__ void __launch_bounds__(NT) k_xcf256_pairs(const Bucket* __restrict__ bk, int window, int pass,
                                                     float* __restrict__ scratch)
{
    extern __shared__ __align__(16) unsigned char smem[];
    Xcf256Shared& S = *reinterpret_cast<Xcf256Shared*>(smem);
    float* slot = scratch + (int64_t)blockIdx.x * kX2SlotFloats;
    const int total = bk->nb * bk->n_roi;
    for (int r = blockIdx.x; r < total; r += gridDim.x) {
        const int b = r / bk->n_roi, j = r - (r / bk->n_roi) * bk->n_roi;
        const RoiLoader<INTERP> load(bk, b, j, pass);
        xcf256_core(S, reinterpret_cast<float2*>(slot), slot + 2 * kX2 * kX2, load, window,
                    (INTERP == 0 ? bk->q1 : bk->q2) + 2 * (int64_t)r, bk->ph + r);
    }
}

__global__ void __launch_bounds__(NT)
    k_xcf256_stage(const float* __restrict__ A, const float* __restrict__ B, int n, int window,
                   float* __restrict__ q, float* __restrict__ ph, float* __restrict__ scratch)
{
    extern __shared__ __align__(16) unsigned char smem[];
    Xcf256Shared& S = *reinterpret_cast<Xcf256Shared*>(smem);
    float* slot = scratch + (int64_t)blockIdx.x * kX2SlotFloats;
    for (int r = blockIdx.x; r < n; r += gridDim.x) {
        const float* a = A + (int64_t)r * kX2 * kX2;
        const float* bb = B + (int64_t)r * kX2 * kX2;
        auto load = [&](int x, int y) -> float2 { return make_float2(a[y * kX2 + x], bb[y * kX2 + x]); };
        xcf256_core(S, reinterpret_cast<float2*>(slot), slot + 2 * kX2 * kX2, load, window, q + 2 * (int64_t)r,
                    ph ? ph + r : nullptr);
    }
}

template <int N>
__global__ void __launch_bounds__(NT)
    k_xcf_stage(const float* __restrict__ A, const float* __restrict__ B, int window,
                float* __restrict__ q, float* __restrict__ ph)
{
    extern __shared__ __align__(16) unsigned char smem[];
    XcfShared<N>& S = *reinterpret_cast<XcfShared<N>*>(smem);
    const int64_t r = blockIdx.x;
    const float* a = A + r * N * N;
    const float* bb = B + r * N * N;
    auto load = [&](int x, int y) -> float2 { return make_float2(a[y * N + x], bb[y * N + x]); };
    xcf_core<N>(S, load, window, q + 2 * r, ph ? ph + r : nullptr);
}

template <int N, int INTERP>
hipError_t launch_pairs_n(const Bucket* d_bk, int blocks, int window, int pass, hipStream_t s)
{
    const size_t sm = sizeof(XcfShared<N>);
    static std::atomic<uint64_t> attr_done{0};
    const hipError_t e = ensure_dynamic_lds((const void*)k_xcf_pairs<N, INTERP>, (int)sm, attr_done);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_xcf_pairs<N, INTERP>), dim3(blocks), dim3(NT), sm, s, d_bk, window, pass);
    return hipGetLastError();
}

template <int INTERP>
hipError_t launch_pairs256(const Bucket* d_bk, const Bucket& hb, int window, int pass, hipStream_t s)
{
    const int total = hb.nb * hb.n_roi;
    if (!hb.xcf_scratch || total <= 0) return hipErrorInvalidValue;
    const size_t sm = sizeof(Xcf256Shared);
    static std::atomic<uint64_t> attr_done{0};
    const hipError_t e = ensure_dynamic_lds((const void*)k_xcf256_pairs<INTERP>, (int)sm, attr_done);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_xcf256_pairs<INTERP>), dim3(std::min(total, kX2Slots)), dim3(NT), sm, s, d_bk, window,
                       pass, hb.xcf_scratch);
    return hipGetLastError();
}

template <int INTERP>
hipError_t launch_pairs_i(const Bucket* d_bk, const Bucket& hb, int window, int pass, hipStream_t s)
{
    const int blocks = hb.nb * hb.n_roi;
    switch (hb.roi_N) {
    case 32: return launch_pairs_n<32, INTERP>(d_bk, blocks, window, pass, s);
    case 64: return launch_pairs_n<64, INTERP>(d_bk, blocks, window, pass, s);
    case 128: return launch_pairs_n<128, INTERP>(d_bk, blocks, window, pass, s);
    case 256: return launch_pairs256<INTERP>(d_bk, hb, window, pass, s);
    default: return hipErrorInvalidValue;
    }
}

template <int N>
hipError_t launch_stage_n(const float* A, const float* B, int n, int window, float* q, float* ph,
                          hipStream_t s)
{
    const size_t sm = sizeof(XcfShared<N>);
    static std::atomic<uint64_t> attr_done{0};
    const hipError_t e = ensure_dynamic_lds((const void*)k_xcf_stage<N>, (int)sm, attr_done);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_xcf_stage<N>, dim3(n), dim3(NT), sm, s, A, B, window, q, ph);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_xcf_pairs(const Bucket* d_bk, const Bucket& hb, int window, int interp, int pass,
                            hipStream_t s)
{
    if (interp == 3) {
        if (!hb.ref_coef || hb.H < 3 || hb.W < 3) return hipErrorInvalidValue;
        return launch_pairs_i<3>(d_bk, hb, window, pass, s);
    }
    return launch_pairs_i<1>(d_bk, hb, window, pass, s);
}

hipError_t launch_xcf_first(const Bucket* d_bk, const Bucket& hb, int window, hipStream_t s)
{
    return launch_pairs_i<0>(d_bk, hb, window, 0, s);
}

hipError_t launch_bspline_coef(const Bucket* d_bk, const Bucket& hb, hipStream_t s)
{
    (void)d_bk;
    if (!hb.ref_coef || !hb.coef_tmp || hb.nref == 0) return hipSuccess;
    // level 0 of each (normalised) reference pyramid
    return launch_coef_images(hb.ref_pyr, hb.pyr_elems, hb.nref, hb.H, hb.W, hb.ref_coef, hb.coef_tmp, s);
}

hipError_t launch_stage_remap(const float* ref, int n, int H, int W, const double* R, double xs, double ys,
                              double zs, int interp, float* coef, float* out, hipStream_t s)
{
    if (interp == 3) {
        // the output buffer holds the row pass until the remap overwrites it
        hipError_t e = launch_coef_images(ref, (int64_t)H * W, n, H, W, coef, out, s);
        if (e != hipSuccess) return e;
    }
    const dim3 grid((W + 63) / 64, H, n);
    if (interp == 3)
        hipLaunchKernelGGL((k_remap_stage<3>), grid, dim3(64), 0, s, coef, n, H, W, R, xs, ys, zs, out);
    else
        hipLaunchKernelGGL((k_remap_stage<1>), grid, dim3(64), 0, s, ref, n, H, W, R, xs, ys, zs, out);
    return hipGetLastError();
}

hipError_t launch_stage_xcf(const float* A, const float* B, int n, int N, int window, float* q,
                            float* ph, float* scratch, hipStream_t s)
{
    switch (N) {
    case 32: return launch_stage_n<32>(A, B, n, window, q, ph, s);
    case 64: return launch_stage_n<64>(A, B, n, window, q, ph, s);
    case 128: return launch_stage_n<128>(A, B, n, window, q, ph, s);
    case 256: {
        if (!scratch) return hipErrorInvalidValue;
        const size_t sm = sizeof(Xcf256Shared);
        static std::atomic<uint64_t> attr_done{0};
        const hipError_t e = ensure_dynamic_lds((const void*)k_xcf256_stage, (int)sm, attr_done);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_xcf256_stage, dim3(std::min(n, kX2Slots)), dim3(NT), sm, s, A, B, n, window, q, ph,
                           scratch);
        return hipGetLastError();
    }
    default: return hipErrorInvalidValue;
    }
}

int64_t xcf_scratch_floats(int N, int64_t rois)
{
    if (N != kX2 || rois <= 0) return 0;
    return std::min<int64_t>(rois, kX2Slots) * kX2SlotFloats;
}

}  // namespace ebsd
