// ROI cross-correlation of the second pass for gfx950 (arXiv:1907.05993,
// section 2: zero-mean ROIs, Hann window, FFT, test spectrum times the
// conjugate reference spectrum, inverse FFT, interpolated peak; the reference
// is first remapped by R_finite, the step before Eq. (12)).
//
// One 256-thread workgroup per (pair, ROI), N in {32, 64, 128}:
//   gather   reference ROI remapped on the fly, Rm(x') = R0(pi(R_finite^T r(x'))),
//            and test ROI, packed as z = a + i b (one complex FFT serves both);
//   window   per-ROI mean removed, symmetric Hann window h (x) h;
//   FFT      2-D radix-2 in LDS: decimation-in-frequency forward (natural in,
//            bit-reversed out), so no explicit permutation is needed;
//   product  P(k) = B(k) conj A(k) with A = (Z(k) + conj Z(-k))/2 and
//            B = (Z(k) - conj Z(-k))/(2i), computed in the bit-reversed domain;
//   inverse  decimation-in-time (bit-reversed in, natural out), scaled 1/N^2;
//   peak     argmax of Re C (ties: lowest row-major index), wrap k >= N/2 to
//            k - N, 2-D quadratic fit on the 3 x 3 circular neighbourhood,
//            peak height C0 / sqrt(sum (a)^2 sum (b)^2).
// The N x N complex tile (padded rows) is LDS resident: 132 KiB at N = 128.
// Twiddles and the window are evaluated per block in FP64 and rounded.
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

template <int N>
__device__ void fft_rows_dif(XcfShared<N>& S)
{
    for (int h = N / 2; h >= 1; h >>= 1) {
        const int step = N / (2 * h);
        for (int c = threadIdx.x; c < N * N / 2; c += NT) {
            const int row = c / (N / 2), j = c - row * (N / 2);
            const int t = j & (h - 1), g = j / h;
            const int i0 = g * 2 * h + t, i1 = i0 + h;
            float2 a = S.z[row][i0], b = S.z[row][i1];
            S.z[row][i0] = make_float2(a.x + b.x, a.y + b.y);
            S.z[row][i1] = cmul(make_float2(a.x - b.x, a.y - b.y), S.tw[t * step]);
        }
        __syncthreads();
    }
}

template <int N>
__device__ void fft_cols_dif(XcfShared<N>& S)
{
    for (int h = N / 2; h >= 1; h >>= 1) {
        const int step = N / (2 * h);
        for (int c = threadIdx.x; c < N * N / 2; c += NT) {
            const int col = c % N, j = c / N;
            const int t = j & (h - 1), g = j / h;
            const int i0 = g * 2 * h + t, i1 = i0 + h;
            float2 a = S.z[i0][col], b = S.z[i1][col];
            S.z[i0][col] = make_float2(a.x + b.x, a.y + b.y);
            S.z[i1][col] = cmul(make_float2(a.x - b.x, a.y - b.y), S.tw[t * step]);
        }
        __syncthreads();
    }
}

template <int N>
__device__ void ifft_cols_dit(XcfShared<N>& S)
{
    for (int h = 1; h <= N / 2; h <<= 1) {
        const int step = N / (2 * h);
        for (int c = threadIdx.x; c < N * N / 2; c += NT) {
            const int col = c % N, j = c / N;
            const int t = j & (h - 1), g = j / h;
            const int i0 = g * 2 * h + t, i1 = i0 + h;
            float2 a = S.z[i0][col];
            float2 b = cmulc(S.z[i1][col], S.tw[t * step]);
            S.z[i0][col] = make_float2(a.x + b.x, a.y + b.y);
            S.z[i1][col] = make_float2(a.x - b.x, a.y - b.y);
        }
        __syncthreads();
    }
}

template <int N>
__device__ void ifft_rows_dit(XcfShared<N>& S)
{
    for (int h = 1; h <= N / 2; h <<= 1) {
        const int step = N / (2 * h);
        for (int c = threadIdx.x; c < N * N / 2; c += NT) {
            const int row = c / (N / 2), j = c - row * (N / 2);
            const int t = j & (h - 1), g = j / h;
            const int i0 = g * 2 * h + t, i1 = i0 + h;
            float2 a = S.z[row][i0];
            float2 b = cmulc(S.z[row][i1], S.tw[t * step]);
            S.z[row][i0] = make_float2(a.x + b.x, a.y + b.y);
            S.z[row][i1] = make_float2(a.x - b.x, a.y - b.y);
        }
        __syncthreads();
    }
}

// The whole correlation for one ROI.  `load(x, y)` returns (reference, test)
// at ROI pixel (x, y).  Writes q (x, y) and ph from thread 0.
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

    // zero mean, window, energies
    float en[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int p = tid; p < N * N; p += NT) {
        const int y = p / N, x = p - y * N;
        const float wgt = S.win[y] * S.win[x];
        float2 ab = S.z[y][x];
        float a = (ab.x - ma) * wgt, b = (ab.y - mb) * wgt;
        S.z[y][x] = make_float2(a, b);
        en[0] += a * a;
        en[1] += b * b;
    }
    block_sum4(en, S.red, 2);
    const float ea = en[0], eb = en[1];

    fft_rows_dif<N>(S);
    fft_cols_dif<N>(S);

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

    ifft_cols_dit<N>(S);
    ifft_rows_dit<N>(S);

    // argmax, ties to the lowest row-major index
    float bv = -INFINITY;
    int bi = 0x7fffffff;
    for (int p = tid; p < N * N; p += NT) {
        const int y = p / N, x = p - y * N;
        float v = S.z[y][x].x;
        if (v > bv) {
            bv = v;
            bi = p;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        float ov = __shfl_xor(bv, off, 64);
        int oi = __shfl_xor(bi, off, 64);
        if (ov > bv || (ov == bv && oi < bi)) {
            bv = ov;
            bi = oi;
        }
    }
    const int lane = tid & 63, wv = tid >> 6;
    if (lane == 0) {
        S.bv[wv] = bv;
        S.bi[wv] = bi;
    }
    __syncthreads();
    if (tid == 0) {
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
}

template <int N>
__global__ void __launch_bounds__(NT) k_xcf_pairs(const Bucket* __restrict__ bk, int window)
{
    extern __shared__ __align__(16) unsigned char smem[];
    XcfShared<N>& S = *reinterpret_cast<XcfShared<N>*>(smem);
    const int b = blockIdx.x / bk->n_roi;
    const int j = blockIdx.x - b * bk->n_roi;
    const int H = bk->H, W = bk->W;
    const float* Rn = bk->ref_pyr + (int64_t)bk->ref_slot[b] * bk->pyr_elems;
    const float* Tn = bk->test_pyr + (int64_t)b * bk->pyr_elems;
    const int x0 = bk->roi_xy[2 * j], y0 = bk->roi_xy[2 * j + 1];
    const double* Rf = bk->Rfin + 9 * (int64_t)b;
    const double r00 = Rf[0], r01 = Rf[1], r02 = Rf[2], r10 = Rf[3], r11 = Rf[4], r12 = Rf[5],
                 r20 = Rf[6], r21 = Rf[7], r22 = Rf[8];
    const double xs = bk->xs, ys = bk->ys, zs = bk->zs;
    auto load = [&](int x, int y) -> float2 {
        const int X = x0 + x, Y = y0 + y;
        const double p0 = (double)X - xs, p1 = (double)Y - ys, p2 = zs;
        // v = R_finite^T r
        const double v0 = r00 * p0 + r10 * p1 + r20 * p2;
        const double v1 = r01 * p0 + r11 * p1 + r21 * p2;
        const double v2 = r02 * p0 + r12 * p1 + r22 * p2;
        const double sx = xs + zs * v0 / v2, sy = ys + zs * v1 / v2;
        const float a = bilinear_d(Rn, H, W, sx, sy);
        const float t = Tn[(int64_t)Y * W + X];
        return make_float2(a, t);
    };
    const int64_t o = (int64_t)b * bk->n_roi + j;
    xcf_core<N>(S, load, window, bk->q2 + 2 * o, bk->ph + o);
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

template <int N>
hipError_t launch_pairs_n(const Bucket* d_bk, int blocks, int window, hipStream_t s)
{
    const size_t sm = sizeof(XcfShared<N>);
    static bool attr_set = false;  // a host attribute, set once (not a stream operation)
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)k_xcf_pairs<N>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(k_xcf_pairs<N>, dim3(blocks), dim3(NT), sm, s, d_bk, window);
    return hipGetLastError();
}

template <int N>
hipError_t launch_stage_n(const float* A, const float* B, int n, int window, float* q, float* ph,
                          hipStream_t s)
{
    const size_t sm = sizeof(XcfShared<N>);
    hipError_t e = hipFuncSetAttribute((const void*)k_xcf_stage<N>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_xcf_stage<N>, dim3(n), dim3(NT), sm, s, A, B, window, q, ph);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_xcf_pairs(const Bucket* d_bk, const Bucket& hb, int window, hipStream_t s)
{
    const int blocks = hb.nb * hb.n_roi;
    switch (hb.roi_N) {
    case 32: return launch_pairs_n<32>(d_bk, blocks, window, s);
    case 64: return launch_pairs_n<64>(d_bk, blocks, window, s);
    case 128: return launch_pairs_n<128>(d_bk, blocks, window, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_stage_xcf(const float* A, const float* B, int n, int N, int window, float* q,
                            float* ph, hipStream_t s)
{
    switch (N) {
    case 32: return launch_stage_n<32>(A, B, n, window, q, ph, s);
    case 64: return launch_stage_n<64>(A, B, n, window, q, ph, s);
    case 128: return launch_stage_n<128>(A, B, n, window, q, ph, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ebsd
