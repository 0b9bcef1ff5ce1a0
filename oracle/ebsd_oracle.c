/*
 * ebsd_oracle.c -- plain, slow, FP64 CPU oracle for demons-based HR-EBSD
 * remapping (Zhu, Kaufmann & Vecchio, "Novel Remapping Approach for HR-EBSD
 * based on Demons Registration", arXiv:1907.05993).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
 * Python binding) may include, link, load or call this file.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark use it.
 * It shares no code, header, table or constant generator with the GPU path.
 *
 * Everything is computed in double precision with plain loops, in the order
 * the method states it, so that it can be checked against the paper by eye:
 *
 *   normalise        z-score per pattern (zero mean as in section 2)
 *   pyramid          factor-2 restriction, [1,3,3,1]/8 separable filter
 *   demons           Eq. (1) force, iterated per level, coarse to fine
 *                    (multi-resolution demons, section 1)
 *   shifts           field sampled at the ROI centres (section 2)
 *   F solve          Eq. (2)/(3) projective model, DLT + Gauss-Newton
 *   polar            Eq. (4)/(5): F = P D Q^T, R = P Q^T
 *   remap            reference remapped by R_finite (section 2, before Eq. 12),
 *                    cubic B-spline interpolation (the paper's cubic scheme)
 *                    or bilinear
 *   XCF              zero mean, Hann window, FFT, F_test . conj(F_ref), IFFT,
 *                    interpolated peak (section 2)
 *   compose          Eq. (12): F = F_inf R_finite; optional further passes
 *                    remap by the previous pass's F and compose with it
 *   rotation vector  axis-angle of R (the passage after Eq. 5, Eq. 6)
 *
 * Readings where the paper is silent or ambiguous (sign of the force, which
 * gradient, smoothing, ROI layout, sub-pixel estimator, determinant
 * normalisation in place of the traction-free condition) are listed in the
 * design notes and restated at each function below.
 *
 * Pins: every function here is checked by tests that do not use this file's
 * arithmetic (numpy/scipy routines, brute-force DFT, closed forms and
 * invariants).  The whole demons loop beyond those invariants is
 * "parity unpinned" except through the identical-pair and known-shift cases.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_CONVERGED 1u
#define ORC_HIT_CAP 2u
#define ORC_SOLVE_ILLCOND 16u
#define ORC_NONFINITE_INPUT 32u
#define ORC_DEGENERATE_INPUT 64u

#define ORC_MAX_LEVELS 8

/* Parameters of one registration (mirrored by a ctypes Structure). */
typedef struct {
    int32_t levels;
    int32_t max_iters[ORC_MAX_LEVELS]; /* [0] = finest level */
    double sigma;                      /* Gaussian smoothing of the field, px; 0 = none */
    double tol;                        /* RMS field update in full-res px; 0 = fixed count */
    double pc_x, pc_y, pc_z;           /* pattern centre as fractions (x*, y* of W, H; Z* of W) */
    int32_t n_roi;                     /* 1 at the pattern centre + (n_roi-1) on a ring */
    int32_t roi_size;                  /* power of two */
    double roi_radius_frac;            /* ring radius / W */
    int32_t window;                    /* 1 = Hann window, 0 = none */
    int32_t second_pass;               /* 1 = remap + XCF second pass */
    int32_t remap_interp;              /* 3 = cubic B-spline, 1 = bilinear */
    int32_t xcf_passes;                /* remap + XCF passes (>= 1) */
    int32_t first_pass;                /* 0 = demons (the paper's method), 1 = ROI
                                          cross-correlation of the unremapped
                                          patterns (the conventional first pass) */
    double bandpass_lo;                /* pre-filter: sigma (px) of the low-pass, 0 = off */
    double bandpass_hi;                /* pre-filter: sigma (px) of the background
                                          Gaussian subtracted (high-pass), 0 = off */
    int32_t background_static;         /* 1 = divide by the static background */
    double background_dynamic;         /* sigma (px) of the dynamic background, 0 = off */
    const double* background;          /* static background [H][W]; orc_register_batch
                                          sets it to the mean of its test patterns */
    int32_t peak_fit;                  /* sub-pixel peak of each XCF: 0 = 2-D quadratic
                                          through the 3 x 3 neighbourhood, 1 = maximum of
                                          the band-limited interpolant of C */
} orc_params;

/* ------------------------------------------------------------------------ */
/* small helpers                                                             */

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }
static double clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* ------------------------------------------------------------------------ */
/* Normalisation.  The paper zero-means the pattern before cross-correlation
 * (section 2); the oracle z-scores each pattern (population std) before
 * every stage.  Returns ORC_DEGENERATE_INPUT (and writes zeros) when the
 * pattern has no contrast, ORC_NONFINITE_INPUT when it holds NaN/Inf.      */
uint32_t orc_normalize_d(const double* in, int64_t n, double* out);

uint32_t orc_normalize(const float* in, int64_t n, double* out)
{
    double* d = (double*)malloc(sizeof(double) * (size_t)n);
    for (int64_t i = 0; i < n; i++) d[i] = (double)in[i];
    uint32_t st = orc_normalize_d(d, n, out);
    free(d);
    return st;
}

uint32_t orc_normalize_d(const double* in, int64_t n, double* out)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; i++) {
        double v = in[i];
        if (!isfinite(v)) {
            for (int64_t j = 0; j < n; j++) out[j] = 0.0;
            return ORC_NONFINITE_INPUT;
        }
        s += v;
    }
    double mean = s / (double)n;
    double ss = 0.0;
    for (int64_t i = 0; i < n; i++) {
        double d = in[i] - mean;
        ss += d * d;
    }
    double sd = sqrt(ss / (double)n);
    if (!(sd > 1e-12 * (fabs(mean) + 1.0))) {
        for (int64_t i = 0; i < n; i++) out[i] = 0.0;
        return ORC_DEGENERATE_INPUT;
    }
    for (int64_t i = 0; i < n; i++) out[i] = (in[i] - mean) / sd;
    return 0u;
}

/* ------------------------------------------------------------------------ */
/* Pyramid restriction (multi-resolution demons, section 1; the paper gives
 * neither factor nor filter).  Factor 2, separable [1,3,3,1]/8 filter with
 * clamped borders, so that coarse pixel i is centred on fine 2i + 0.5:
 *   out[i] = (in[c(2i-1)] + 3 in[c(2i)] + 3 in[c(2i+1)] + in[c(2i+2)]) / 8,
 * c clamping to [0, N-1].  N fine pixels give ceil(N/2) coarse ones (an odd
 * N: the last coarse pixel sees the last fine pixel through the clamp).    */
void orc_restrict(const double* in, int H, int W, double* out)
{
    int h = (H + 1) / 2, w = (W + 1) / 2;
    double* tmp = (double*)malloc(sizeof(double) * (size_t)H * (size_t)w);
    for (int y = 0; y < H; y++) {
        const double* row = in + (size_t)y * W;
        for (int i = 0; i < w; i++) {
            double a = row[clampi(2 * i - 1, 0, W - 1)];
            double b = row[clampi(2 * i, 0, W - 1)];
            double c = row[clampi(2 * i + 1, 0, W - 1)];
            double d = row[clampi(2 * i + 2, 0, W - 1)];
            tmp[(size_t)y * w + i] = (a + 3.0 * b + 3.0 * c + d) / 8.0;
        }
    }
    for (int j = 0; j < h; j++) {
        for (int x = 0; x < w; x++) {
            double a = tmp[(size_t)clampi(2 * j - 1, 0, H - 1) * w + x];
            double b = tmp[(size_t)clampi(2 * j, 0, H - 1) * w + x];
            double c = tmp[(size_t)clampi(2 * j + 1, 0, H - 1) * w + x];
            double d = tmp[(size_t)clampi(2 * j + 2, 0, H - 1) * w + x];
            out[(size_t)j * w + x] = (a + 3.0 * b + 3.0 * c + d) / 8.0;
        }
    }
    free(tmp);
}

/* ------------------------------------------------------------------------ */
/* Image gradient used by the demons force of Eq. (1): central differences in
 * the interior, one-sided differences on the border rows/columns.          */
void orc_gradient(const double* f, int H, int W, double* gx, double* gy)
{
    for (int y = 0; y < H; y++) {
        for (int x = 0; x < W; x++) {
            size_t i = (size_t)y * W + x;
            double dx, dy;
            if (W == 1) dx = 0.0;
            else if (x == 0) dx = f[i + 1] - f[i];
            else if (x == W - 1) dx = f[i] - f[i - 1];
            else dx = (f[i + 1] - f[i - 1]) / 2.0;
            if (H == 1) dy = 0.0;
            else if (y == 0) dy = f[i + W] - f[i];
            else if (y == H - 1) dy = f[i] - f[i - W];
            else dy = (f[i + W] - f[i - W]) / 2.0;
            gx[i] = dx;
            gy[i] = dy;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Bilinear sample of img (H x W, pixel centres at integers, x = column) at
 * (x, y).  Coordinates are clamped to [0, W-1] x [0, H-1] before the floor,
 * i.e. the image is extended by replicating its border.                    */
double orc_bilinear(const double* img, int H, int W, double x, double y)
{
    double xc = clampd(x, 0.0, (double)(W - 1));
    double yc = clampd(y, 0.0, (double)(H - 1));
    int x0 = (int)floor(xc), y0 = (int)floor(yc);
    double fx = xc - (double)x0, fy = yc - (double)y0;
    int x1 = x0 + 1 < W ? x0 + 1 : W - 1;
    int y1 = y0 + 1 < H ? y0 + 1 : H - 1;
    double v00 = img[(size_t)y0 * W + x0], v01 = img[(size_t)y0 * W + x1];
    double v10 = img[(size_t)y1 * W + x0], v11 = img[(size_t)y1 * W + x1];
    double top = (1.0 - fx) * v00 + fx * v01;
    double bot = (1.0 - fx) * v10 + fx * v11;
    return (1.0 - fy) * top + fy * bot;
}

void orc_bilinear_points(const double* img, int H, int W, const double* xs,
                         const double* ys, int64_t n, double* out)
{
    for (int64_t i = 0; i < n; i++) out[i] = orc_bilinear(img, H, W, xs[i], ys[i]);
}

/* Warp: out(x) = img(x + u(x)), u = [2][H][W] (channel 0 along columns). */
void orc_warp(const double* img, int H, int W, const double* u, double* out)
{
    size_t HW = (size_t)H * W;
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            size_t i = (size_t)y * W + x;
            out[i] = orc_bilinear(img, H, W, (double)x + u[i], (double)y + u[HW + i]);
        }
}

/* ------------------------------------------------------------------------ */
/* Structural similarity of the registration (the SSIM section 3 reports for
 * demons; its window and constants are not given, the standard choices are
 * taken): between the normalised reference R and the test warped by the
 * final field, Tw(x) = T(x + u(x)).  For each pixel whose 11 x 11 window lies
 * inside the pattern, with the Gaussian window w (sigma 1.5 px, radius 5,
 * unit sum): mu_a = sum w a, var_a = sum w a^2 - mu_a^2, cov = sum w R Tw -
 * mu_R mu_T, and
 *   SSIM = (2 mu_R mu_T + C1)(2 cov + C2) / ((mu_R^2 + mu_T^2 + C1)(var_R + var_T + C2))
 * with C1 = (0.01 L)^2, C2 = (0.03 L)^2 and L = 6 (the patterns are z-scored:
 * +-3 standard deviations).  Returns the mean over those pixels (NaN when
 * the pattern is 10 px or less in either direction: no window fits).      */
double orc_ssim(const double* R, const double* Tw, int H, int W)
{
    const int rad = 5;
    double w[11], ws = 0.0;
    for (int j = -rad; j <= rad; j++) ws += (w[j + rad] = exp(-(double)(j * j) / (2.0 * 1.5 * 1.5)));
    for (int j = 0; j < 11; j++) w[j] /= ws;
    const double L = 6.0, C1 = (0.01 * L) * (0.01 * L), C2 = (0.03 * L) * (0.03 * L);
    double sum = 0.0;
    long count = 0;
    for (int y = rad; y < H - rad; y++)
        for (int x = rad; x < W - rad; x++) {
            double ma = 0, mb = 0, saa = 0, sbb = 0, sab = 0;
            for (int j = -rad; j <= rad; j++)
                for (int i = -rad; i <= rad; i++) {
                    double ww = w[j + rad] * w[i + rad];
                    double a = R[(size_t)(y + j) * W + x + i], b = Tw[(size_t)(y + j) * W + x + i];
                    ma += ww * a;
                    mb += ww * b;
                    saa += ww * a * a;
                    sbb += ww * b * b;
                    sab += ww * a * b;
                }
            double va = saa - ma * ma, vb = sbb - mb * mb, cv = sab - ma * mb;
            sum += (2.0 * ma * mb + C1) * (2.0 * cv + C2) / ((ma * ma + mb * mb + C1) * (va + vb + C2));
            count++;
        }
    return count > 0 ? sum / (double)count : NAN; /* no window fits: undefined */
}

/* ------------------------------------------------------------------------ */
/* Gaussian smoothing of one field channel: separable taps
 * w_j = exp(-j^2 / (2 sigma^2)), j = -r..r, r = floor(3 sigma + 0.5),
 * normalised to unit sum; the border is replicated.  sigma <= 0 copies.    */
void orc_smooth(const double* v, int H, int W, double sigma, double* out)
{
    size_t HW = (size_t)H * W;
    if (!(sigma > 0.0)) {
        memcpy(out, v, sizeof(double) * HW);
        return;
    }
    int r = (int)floor(3.0 * sigma + 0.5);
    double* w = (double*)malloc(sizeof(double) * (size_t)(2 * r + 1));
    double sum = 0.0;
    for (int j = -r; j <= r; j++) {
        w[j + r] = exp(-(double)(j * j) / (2.0 * sigma * sigma));
        sum += w[j + r];
    }
    for (int j = 0; j <= 2 * r; j++) w[j] /= sum;
    double* tmp = (double*)malloc(sizeof(double) * HW);
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            double acc = 0.0;
            for (int j = -r; j <= r; j++)
                acc += w[j + r] * v[(size_t)y * W + clampi(x + j, 0, W - 1)];
            tmp[(size_t)y * W + x] = acc;
        }
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            double acc = 0.0;
            for (int j = -r; j <= r; j++)
                acc += w[j + r] * tmp[(size_t)clampi(y + j, 0, H - 1) * W + x];
            out[(size_t)y * W + x] = acc;
        }
    free(tmp);
    free(w);
}

/* Pre-filter of a raw pattern (section 3.3: a low-pass filter against
 * high-frequency noise and a high-pass filter against low-frequency
 * background gradients, applied before registration; their kernels are not
 * given).  Reading: Gaussian filters, out = G_lo * p - G_hi * p, where G_lo
 * is orc_smooth with sigma lo (identity when lo <= 0) and G_hi * p the
 * background estimate with sigma hi (nothing subtracted when hi <= 0).      */
void orc_bandpass_d(const double* p, int H, int W, double lo, double hi, double* out)
{
    size_t HW = (size_t)H * W;
    double* t = (double*)malloc(sizeof(double) * HW);
    if (lo > 0.0) orc_smooth(p, H, W, lo, out);
    else memcpy(out, p, sizeof(double) * HW);
    if (hi > 0.0) {
        orc_smooth(p, H, W, hi, t);
        for (size_t i = 0; i < HW; i++) out[i] -= t[i];
    }
    free(t);
}

void orc_bandpass(const float* in, int H, int W, double lo, double hi, double* out)
{
    size_t HW = (size_t)H * W;
    double* p = (double*)malloc(sizeof(double) * HW);
    for (size_t i = 0; i < HW; i++) p[i] = (double)in[i];
    orc_bandpass_d(p, H, W, lo, hi, out);
    free(p);
}

/* Background correction (section 3.3 applies a dynamic and a static
 * background correction to the experimental patterns; their forms are not
 * given).  Reading: static, divide by the scan's mean pattern bg (the
 * pixelwise mean of the call's test patterns); dynamic, then divide by the
 * pattern's own Gaussian blur of sigma dyn (orc_smooth).  A non-positive
 * divisor gives 0.  bg may be NULL, dyn <= 0 turns the dynamic step off.   */
void orc_background(const float* in, int H, int W, const double* bg, double dyn, double* out)
{
    size_t HW = (size_t)H * W;
    for (size_t i = 0; i < HW; i++) {
        double v = (double)in[i];
        if (bg) v = bg[i] > 0.0 ? v / bg[i] : 0.0;
        out[i] = v;
    }
    if (dyn > 0.0) {
        double* b = (double*)malloc(sizeof(double) * HW);
        orc_smooth(out, H, W, dyn, b);
        for (size_t i = 0; i < HW; i++) out[i] = b[i] > 0.0 ? out[i] / b[i] : 0.0;
        free(b);
    }
}

/* Pixelwise mean of n patterns [n][H][W] (the static background). */
void orc_mean_pattern(const float* p, int n, int H, int W, double* out)
{
    size_t HW = (size_t)H * W;
    for (size_t i = 0; i < HW; i++) {
        double s = 0.0;
        for (int k = 0; k < n; k++) s += (double)p[(size_t)k * HW + i];
        out[i] = s / (double)n;
    }
}

/* ------------------------------------------------------------------------ */
/* One demons iteration at one pyramid level (Eq. (1), Thirion's force).
 *
 * Field convention: u lives on the reference grid and T(x + u(x)) ~ R(x),
 * so that u at a ROI centre is the shift q of Eq. (2).  With a = R - T(x+u)
 * the update is du = a grad(R) / (|grad R|^2 + a^2), the Eq. (1) force with
 * the intensity difference taken reference-minus-warped-test (the opposite
 * order to the printed Eq. (1), which belongs to the opposite field
 * direction), and the gradient taken on the fixed reference image as
 * Eq. (1)'s symbol says.  0/0 (den <= 1e-9) gives du = 0.
 *
 * The accumulated field is then smoothed (the paper applies none; sigma = 0
 * reproduces that).  Returns RMS over pixels of |u_new - u| in level px.  */
double orc_demons_iter(const double* R, const double* T, const double* gx,
                       const double* gy, int H, int W, const double* u,
                       double sigma, double* u_new)
{
    size_t HW = (size_t)H * W;
    double* v = (double*)malloc(sizeof(double) * 2 * HW);
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            size_t i = (size_t)y * W + x;
            double wv = orc_bilinear(T, H, W, (double)x + u[i], (double)y + u[HW + i]);
            double a = R[i] - wv;
            double den = gx[i] * gx[i] + gy[i] * gy[i] + a * a;
            double dux = 0.0, duy = 0.0;
            if (den > 1e-9) {
                dux = a * gx[i] / den;
                duy = a * gy[i] / den;
            }
            v[i] = u[i] + dux;
            v[HW + i] = u[HW + i] + duy;
        }
    orc_smooth(v, H, W, sigma, u_new);
    orc_smooth(v + HW, H, W, sigma, u_new + HW);
    double ss = 0.0;
    for (size_t i = 0; i < HW; i++) {
        double dx = u_new[i] - u[i], dy = u_new[HW + i] - u[HW + i];
        ss += dx * dx + dy * dy;
    }
    free(v);
    return sqrt(ss / (double)HW);
}

/* Prolongation of the field to the next finer level (H x W, 2h x 2w or one
 * less where the finer level was odd): bilinear with the half-pixel-centre
 * map (fine i -> coarse (i - 0.5)/2), values doubled because the field is
 * measured in the pixels of its level.                                    */
void orc_prolong(const double* u, int h, int w, int H, int W, double* out)
{
    size_t hw = (size_t)h * w, HW = (size_t)H * W;
    for (int c = 0; c < 2; c++)
        for (int y = 0; y < H; y++)
            for (int x = 0; x < W; x++)
                out[(size_t)c * HW + (size_t)y * W + x] =
                    2.0 * orc_bilinear(u + (size_t)c * hw, h, w, ((double)x - 0.5) / 2.0,
                                       ((double)y - 0.5) / 2.0);
}

/* ------------------------------------------------------------------------ */
/* Multi-resolution demons (section 1): the field found on the coarser level
 * initialises the next finer level.  Rn/Tn are the normalised full-res
 * images.  u_init, if not NULL, is the initial field on the coarsest level
 * (in that level's px).  Writes the finest field [2][H][W] and per-level
 * iteration counts.  Returns ORC_CONVERGED when every level stopped on the
 * tolerance, ORC_HIT_CAP when a level ran to its cap with tol > 0.       */
uint32_t orc_demons(const double* Rn, const double* Tn, int H, int W, const orc_params* p,
                    const double* u_init, double* field, int32_t* iters)
{
    int L = p->levels;
    const double* Rl[ORC_MAX_LEVELS];
    const double* Tl[ORC_MAX_LEVELS];
    double* own[2 * ORC_MAX_LEVELS];
    int nown = 0;
    int Hs[ORC_MAX_LEVELS], Ws[ORC_MAX_LEVELS];
    Rl[0] = Rn;
    Tl[0] = Tn;
    Hs[0] = H;
    Ws[0] = W;
    for (int l = 1; l < L; l++) {
        Hs[l] = (Hs[l - 1] + 1) / 2;
        Ws[l] = (Ws[l - 1] + 1) / 2;
        double* r = (double*)malloc(sizeof(double) * (size_t)Hs[l] * Ws[l]);
        double* t = (double*)malloc(sizeof(double) * (size_t)Hs[l] * Ws[l]);
        orc_restrict(Rl[l - 1], Hs[l - 1], Ws[l - 1], r);
        orc_restrict(Tl[l - 1], Hs[l - 1], Ws[l - 1], t);
        Rl[l] = r;
        Tl[l] = t;
        own[nown++] = r;
        own[nown++] = t;
    }
    size_t HW0 = (size_t)H * W;
    double* ua = (double*)calloc(2 * HW0, sizeof(double));
    double* ub = (double*)calloc(2 * HW0, sizeof(double));
    double* gx = (double*)malloc(sizeof(double) * HW0);
    double* gy = (double*)malloc(sizeof(double) * HW0);
    {
        size_t n = 2 * (size_t)Hs[L - 1] * Ws[L - 1];
        if (u_init)
            memcpy(ua, u_init, sizeof(double) * n);
    }
    uint32_t status = 0;
    int all_conv = 1, any_cap = 0;
    for (int l = L - 1; l >= 0; l--) {
        int h = Hs[l], w = Ws[l];
        orc_gradient(Rl[l], h, w, gx, gy);
        double scale = (double)(1 << l);
        int k = 0, conv = 0;
        while (k < p->max_iters[l]) {
            double rms = orc_demons_iter(Rl[l], Tl[l], gx, gy, h, w, ua, p->sigma, ub);
            double* t = ua;
            ua = ub;
            ub = t;
            k++;
            if (p->tol > 0.0 && scale * rms < p->tol) {
                conv = 1;
                break;
            }
        }
        iters[l] = k;
        if (!conv) all_conv = 0;
        if (!conv && p->tol > 0.0) any_cap = 1;
        if (l > 0) {
            orc_prolong(ua, h, w, Hs[l - 1], Ws[l - 1], ub);
            double* t = ua;
            ua = ub;
            ub = t;
        }
    }
    memcpy(field, ua, sizeof(double) * 2 * HW0);
    if (p->tol > 0.0 && all_conv) status |= ORC_CONVERGED;
    if (any_cap) status |= ORC_HIT_CAP;
    free(ua);
    free(ub);
    free(gx);
    free(gy);
    for (int i = 0; i < nown; i++) free(own[i]);
    return status;
}

/* ------------------------------------------------------------------------ */
/* ROI layout (section 2: ROIs evenly spaced around the pattern centre plus
 * one at the centre).  ROI 0 sits at the pattern centre, ROIs 1..n-1 on a
 * ring of radius frac*W at angles 2 pi j/(n-1), measured from +x toward +y.
 * Top-left corner x0 = floor(cx - (N-1)/2 + 0.5); the actual centre used in
 * Eq. (2) is x0 + (N-1)/2.  Returns 0 if all ROIs are inside the pattern. */
int orc_roi_layout(int H, int W, const orc_params* p, double* cx, double* cy,
                   int32_t* x0, int32_t* y0)
{
    const double pi = 3.14159265358979323846;
    double xs = p->pc_x * W - 0.5, ys = p->pc_y * H - 0.5;
    double rho = p->roi_radius_frac * W;
    int N = p->roi_size;
    int bad = 0;
    for (int j = 0; j < p->n_roi; j++) {
        double px = xs, py = ys;
        if (j > 0) {
            double ang = 2.0 * pi * (double)(j - 1) / (double)(p->n_roi - 1);
            px = xs + rho * cos(ang);
            py = ys + rho * sin(ang);
        }
        int ix = (int)floor(px - (N - 1) / 2.0 + 0.5);
        int iy = (int)floor(py - (N - 1) / 2.0 + 0.5);
        x0[j] = ix;
        y0[j] = iy;
        cx[j] = ix + (N - 1) / 2.0;
        cy[j] = iy + (N - 1) / 2.0;
        if (ix < 0 || iy < 0 || ix + N > W || iy + N > H) bad = 1;
    }
    return bad;
}

/* ------------------------------------------------------------------------ */
/* Dense linear algebra for the small solves (textbook methods).            */

/* Cyclic Jacobi eigen-decomposition of a symmetric n x n matrix A (row-major,
 * destroyed).  On exit evals[i] are the eigenvalues and column i of V
 * (row-major n x n) the matching unit eigenvector.  Golub & Van Loan,
 * "Matrix Computations", symmetric Schur rotations.                         */
void orc_jacobi_eig(double* A, int n, double* evals, double* V)
{
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) V[i * n + j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; sweep++) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; i++)
            for (int j = 0; j < n; j++) {
                tot += A[i * n + j] * A[i * n + j];
                if (i != j) off += A[i * n + j] * A[i * n + j];
            }
        if (off <= 1e-30 * tot || off == 0.0) break;
        for (int p = 0; p < n - 1; p++)
            for (int q = p + 1; q < n; q++) {
                double apq = A[p * n + q];
                if (apq == 0.0) continue;
                double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
                double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                /* A <- J^T A J with J the (p,q) rotation [c s; -s c] */
                for (int k = 0; k < n; k++) {
                    double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; k++) {
                    double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; k++) {
                    double vkp = V[k * n + p], vkq = V[k * n + q];
                    V[k * n + p] = c * vkp - s * vkq;
                    V[k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    for (int i = 0; i < n; i++) evals[i] = A[i * n + i];
}

/* Solve A x = b (n x n, row-major, both destroyed) by Gaussian elimination
 * with partial pivoting.  Returns 0 on success, 1 if a pivot is zero.     */
static int orc_gauss_solve(double* A, double* b, int n, double* x)
{
    for (int k = 0; k < n; k++) {
        int piv = k;
        for (int i = k + 1; i < n; i++)
            if (fabs(A[i * n + k]) > fabs(A[piv * n + k])) piv = i;
        if (A[piv * n + k] == 0.0) return 1;
        if (piv != k) {
            for (int j = 0; j < n; j++) {
                double t = A[k * n + j];
                A[k * n + j] = A[piv * n + j];
                A[piv * n + j] = t;
            }
            double t = b[k];
            b[k] = b[piv];
            b[piv] = t;
        }
        for (int i = k + 1; i < n; i++) {
            double m = A[i * n + k] / A[k * n + k];
            for (int j = k; j < n; j++) A[i * n + j] -= m * A[k * n + j];
            b[i] -= m * b[k];
        }
    }
    for (int i = n - 1; i >= 0; i--) {
        double s = b[i];
        for (int j = i + 1; j < n; j++) s -= A[i * n + j] * x[j];
        x[i] = s / A[i * n + i];
    }
    return 0;
}

static double det3(const double* F)
{
    return F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) +
           F[2] * (F[3] * F[7] - F[4] * F[6]);
}

/* (A^-1)^T = cofactor matrix / det A (row-major); A must be invertible. */
static void inv3_transposed(const double* A, double* out)
{
    double c[9];
    c[0] = A[4] * A[8] - A[5] * A[7];
    c[1] = A[5] * A[6] - A[3] * A[8];
    c[2] = A[3] * A[7] - A[4] * A[6];
    c[3] = A[2] * A[7] - A[1] * A[8];
    c[4] = A[0] * A[8] - A[2] * A[6];
    c[5] = A[1] * A[6] - A[0] * A[7];
    c[6] = A[1] * A[5] - A[2] * A[4];
    c[7] = A[2] * A[3] - A[0] * A[5];
    c[8] = A[0] * A[4] - A[1] * A[3];
    double det = A[0] * c[0] + A[1] * c[1] + A[2] * c[2];
    for (int i = 0; i < 9; i++) out[i] = c[i] / det;
}

static void matmul3(const double* A, const double* B, double* C)
{
    double t[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0.0;
            for (int k = 0; k < 3; k++) s += A[i * 3 + k] * B[k * 3 + j];
            t[i * 3 + j] = s;
        }
    memcpy(C, t, sizeof t);
}

/* F <- F / cbrt(det F): the isochoric normalisation that stands in for the
 * traction-free condition (the shifts fix F only up to scale).             */
void orc_det_normalize(double* F)
{
    double d = det3(F);
    double s = cbrt(d);
    for (int i = 0; i < 9; i++) F[i] /= s;
}

/* ------------------------------------------------------------------------ */
/* Deformation gradient from ROI shifts: the minimiser of Eq. (3) for the
 * projective model of Eq. (2),  r' = r + q = Z* F r / ((F r) . k).
 * r_i = (cx_i - x*, cy_i - y*, Z*), k = (0,0,1); positions in units of Z*.
 *   1. DLT start: smallest right singular vector of the 2n x 9 system
 *      F1.r - p_x F3.r = 0, F2.r - p_y F3.r = 0 (via eigen of A^T A),
 *      scaled to F33 = 1;
 *   2. Gauss-Newton on the 8 free entries (F33 = 1) with Eq. (3)'s
 *      residuals, stop when |step| < 1e-14 or after 100 steps;
 *   3. det F = 1.
 * Returns ORC_SOLVE_ILLCOND when cond(J^T J) > 1e12 or a step fails.       */
uint32_t orc_solve_F(const double* q, const double* cx, const double* cy, int n,
                     double xs, double ys, double zs, double* F)
{
    uint32_t st = 0;
    double* rx = (double*)malloc(sizeof(double) * n);
    double* ry = (double*)malloc(sizeof(double) * n);
    double* px = (double*)malloc(sizeof(double) * n);
    double* py = (double*)malloc(sizeof(double) * n);
    for (int i = 0; i < n; i++) {
        rx[i] = (cx[i] - xs) / zs;
        ry[i] = (cy[i] - ys) / zs;
        px[i] = (cx[i] - xs + q[2 * i]) / zs;
        py[i] = (cy[i] - ys + q[2 * i + 1]) / zs;
    }
    /* 1. DLT */
    double AtA[81];
    memset(AtA, 0, sizeof AtA);
    for (int i = 0; i < n; i++) {
        double r[3] = {rx[i], ry[i], 1.0};
        double row1[9] = {r[0], r[1], r[2], 0, 0, 0, -px[i] * r[0], -px[i] * r[1], -px[i] * r[2]};
        double row2[9] = {0, 0, 0, r[0], r[1], r[2], -py[i] * r[0], -py[i] * r[1], -py[i] * r[2]};
        for (int a = 0; a < 9; a++)
            for (int b = 0; b < 9; b++) AtA[a * 9 + b] += row1[a] * row1[b] + row2[a] * row2[b];
    }
    double ev[9], V[81];
    orc_jacobi_eig(AtA, 9, ev, V);
    int imin = 0;
    for (int i = 1; i < 9; i++)
        if (ev[i] < ev[imin]) imin = i;
    double f[9];
    for (int i = 0; i < 9; i++) f[i] = V[i * 9 + imin];
    double s33 = f[8];
    if (s33 == 0.0) {
        st |= ORC_SOLVE_ILLCOND;
        s33 = 1.0;
    }
    for (int i = 0; i < 9; i++) f[i] /= s33;

    /* 2. Gauss-Newton on theta = (F11,F12,F13,F21,F22,F23,F31,F32), F33 = 1 */
    double JtJ[64], Jte[8];
    for (int it = 0; it < 100; it++) {
        memset(JtJ, 0, sizeof JtJ);
        memset(Jte, 0, sizeof Jte);
        for (int i = 0; i < n; i++) {
            double r[3] = {rx[i], ry[i], 1.0};
            double n1 = f[0] * r[0] + f[1] * r[1] + f[2] * r[2];
            double n2 = f[3] * r[0] + f[4] * r[1] + f[5] * r[2];
            double d = f[6] * r[0] + f[7] * r[1] + f[8] * r[2];
            double ex = n1 / d - px[i], ey = n2 / d - py[i];
            double jx[8] = {r[0] / d, r[1] / d, r[2] / d, 0, 0, 0, -n1 * r[0] / (d * d), -n1 * r[1] / (d * d)};
            double jy[8] = {0, 0, 0, r[0] / d, r[1] / d, r[2] / d, -n2 * r[0] / (d * d), -n2 * r[1] / (d * d)};
            for (int a = 0; a < 8; a++) {
                Jte[a] += jx[a] * ex + jy[a] * ey;
                for (int b = 0; b < 8; b++) JtJ[a * 8 + b] += jx[a] * jx[b] + jy[a] * jy[b];
            }
        }
        double A[64], rhs[8], step[8];
        memcpy(A, JtJ, sizeof A);
        for (int a = 0; a < 8; a++) rhs[a] = -Jte[a];
        if (orc_gauss_solve(A, rhs, 8, step)) {
            st |= ORC_SOLVE_ILLCOND;
            break;
        }
        double nrm = 0.0;
        for (int a = 0; a < 8; a++) {
            f[a] += step[a];
            nrm += step[a] * step[a];
        }
        if (!isfinite(nrm)) {
            st |= ORC_SOLVE_ILLCOND;
            break;
        }
        if (sqrt(nrm) < 1e-14) break;
    }
    /* conditioning at the solution */
    {
        memset(JtJ, 0, sizeof JtJ);
        for (int i = 0; i < n; i++) {
            double r[3] = {rx[i], ry[i], 1.0};
            double n1 = f[0] * r[0] + f[1] * r[1] + f[2] * r[2];
            double n2 = f[3] * r[0] + f[4] * r[1] + f[5] * r[2];
            double d = f[6] * r[0] + f[7] * r[1] + f[8] * r[2];
            double jx[8] = {r[0] / d, r[1] / d, r[2] / d, 0, 0, 0, -n1 * r[0] / (d * d), -n1 * r[1] / (d * d)};
            double jy[8] = {0, 0, 0, r[0] / d, r[1] / d, r[2] / d, -n2 * r[0] / (d * d), -n2 * r[1] / (d * d)};
            for (int a = 0; a < 8; a++)
                for (int b = 0; b < 8; b++) JtJ[a * 8 + b] += jx[a] * jx[b] + jy[a] * jy[b];
        }
        double e8[8], V8[64];
        orc_jacobi_eig(JtJ, 8, e8, V8);
        double lo = e8[0], hi = e8[0];
        for (int a = 1; a < 8; a++) {
            if (e8[a] < lo) lo = e8[a];
            if (e8[a] > hi) hi = e8[a];
        }
        if (!(lo > 0.0) || hi / lo > 1e12) st |= ORC_SOLVE_ILLCOND;
    }
    memcpy(F, f, sizeof f);
    if (!(det3(F) > 0.0)) st |= ORC_SOLVE_ILLCOND;
    else orc_det_normalize(F);
    free(rx);
    free(ry);
    free(px);
    free(py);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Stress of a sample-frame strain (Eq. (16); supplementary Eq. (2.4)-(2.8)).
 * The strain goes to the crystal frame, eps_C = g eps_S g^T (g: the passive
 * orientation taking sample coordinates to crystal coordinates, Eq. (2.1)),
 * Hooke's law acts there with the cubic stiffness in Voigt form (C11 on the
 * normal strains, C12 between them, C44 on the engineering shears
 * 2 eps_ij), and the stress comes back, sigma_S = g^T sigma_C g.           */
void orc_stress(const double* eps_S, const double* g, double C11, double C12, double C44,
                double* sig_S)
{
    double t[9], e[9], sc[9];
    matmul3(g, eps_S, t);
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) e[3 * i + j] = t[3 * i] * g[3 * j] + t[3 * i + 1] * g[3 * j + 1] +
                                                   t[3 * i + 2] * g[3 * j + 2];
    sc[0] = C11 * e[0] + C12 * (e[4] + e[8]);
    sc[4] = C11 * e[4] + C12 * (e[0] + e[8]);
    sc[8] = C11 * e[8] + C12 * (e[0] + e[4]);
    sc[1] = sc[3] = C44 * (e[1] + e[3]);
    sc[2] = sc[6] = C44 * (e[2] + e[6]);
    sc[5] = sc[7] = C44 * (e[5] + e[7]);
    /* sigma_S = g^T sc g */
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double acc = 0.0;
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++) acc += g[3 * a + i] * sc[3 * a + b] * g[3 * b + j];
            sig_S[3 * i + j] = acc;
        }
}

/* Strain and stress of a detector-frame deformation gradient (Eq. (14)-(16)):
 * F_S = S F S^T with S the detector-to-sample rotation (Eq. (13)'s R_tilt
 * is one), eps_S = (F_S F_S^T - I)/2 (the first form of Eq. (15): the
 * rotation in F cancels), sigma_S from orc_stress.  Any output may be NULL. */
void orc_strain_stress(const double* F, const double* S, const double* g, double C11, double C12,
                       double C44, double* FS_out, double* eps_out, double* sig_out)
{
    double t[9], FS[9], eps[9], sig[9];
    matmul3(S, F, t);
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            FS[3 * i + j] = t[3 * i] * S[3 * j] + t[3 * i + 1] * S[3 * j + 1] + t[3 * i + 2] * S[3 * j + 2];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            eps[3 * i + j] = 0.5 * (FS[3 * i] * FS[3 * j] + FS[3 * i + 1] * FS[3 * j + 1] +
                                    FS[3 * i + 2] * FS[3 * j + 2] - (i == j ? 1.0 : 0.0));
    orc_stress(eps, g, C11, C12, C44, sig);
    if (FS_out) memcpy(FS_out, FS, sizeof FS);
    if (eps_out) memcpy(eps_out, eps, sizeof eps);
    if (sig_out) memcpy(sig_out, sig, sizeof sig);
}

/* The three surface tractions of the total F = X M, sigma_S33, sigma_S23,
 * sigma_S13, divided by C11, and (if A != NULL) their derivatives with
 * respect to the nine entries of X (A: 3 x 9, row-major): eps_S is
 * quadratic in X, d eps_S = (dF_S F_S^T + F_S dF_S^T)/2 with
 * dF_S = S E_ab M S^T, and the stress is linear in the strain.            */
static void traction_terms(const double* X, const double* M, const double* S, const double* g,
                           double C11, double C12, double C44, double* c, double* A)
{
    double F[9], FS[9], sig[9];
    matmul3(X, M, F);
    orc_strain_stress(F, S, g, C11, C12, C44, FS, NULL, sig);
    c[0] = sig[8] / C11;
    c[1] = sig[5] / C11;
    c[2] = sig[2] / C11;
    if (!A) return;
    double MS[9]; /* M S^T */
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) MS[3 * i + j] = M[3 * i] * S[3 * j] + M[3 * i + 1] * S[3 * j + 1] + M[3 * i + 2] * S[3 * j + 2];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double dFS[9], de[9], ds[9];
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) dFS[3 * i + j] = S[3 * i + a] * MS[3 * b + j];
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) {
                    double acc = 0.0;
                    for (int k = 0; k < 3; k++) acc += dFS[3 * i + k] * FS[3 * j + k] + FS[3 * i + k] * dFS[3 * j + k];
                    de[3 * i + j] = 0.5 * acc;
                }
            orc_stress(de, g, C11, C12, C44, ds);
            A[0 * 9 + 3 * a + b] = ds[8] / C11;
            A[1 * 9 + 3 * a + b] = ds[5] / C11;
            A[2 * 9 + 3 * a + b] = ds[2] / C11;
        }
}

/* Eq. (3) under the traction-free equality constraint (section 2; Eq. (16);
 * supplementary Part 2): minimise the Eq. (3) objective over F_inf subject
 * to sigma_S33 = sigma_S23 = sigma_S13 = 0 (no traction on the surface,
 * t = sigma_S z_S) for the total F = F_inf M (M: what a second-pass fit
 * composes with, Eq. (12); NULL = identity, a first-pass fit).  The
 * objective fixes F_inf only up to scale; the constraints fix the scale and
 * tie two more directions.
 *   1. F_inf up to scale: orc_solve_F.
 *   2. Starting scale from sigma_S33 = 0 alone: with B = F_S F_S^T at unit
 *      scale, sigma(s) = (s^2 sigma[B] - sigma[I]) / 2 (sigma[.] Hooke's law
 *      of a strain), so s^2 = sigma[I]_33 / sigma[B]_33.
 *   3. Lagrange-Newton steps over all nine entries (Gauss-Newton on the
 *      objective, Newton on the constraints): [J^T J  A^T; A  0] [d; l] =
 *      [-J^T e; -c], e the residuals in units of Z*, J their Jacobian, c the
 *      three stresses over C11 and A their Jacobian; stop when |d| < 1e-14
 *      or after 100 steps.
 * F receives the total F (detector frame), eps and sig (optional) the
 * sample-frame strain and stress (units of the stiffness constants).
 * Returns ORC_SOLVE_ILLCOND if a step fails or the steps do not converge. */
uint32_t orc_solve_F_traction_free(const double* q, const double* cx, const double* cy, int n,
                                   double xs, double ys, double zs, const double* M_in,
                                   const double* S, const double* g, double C11, double C12,
                                   double C44, double* F, double* eps, double* sig)
{
    const double I3[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    const double* M = M_in ? M_in : I3;
    double X[9];
    uint32_t st = orc_solve_F(q, cx, cy, n, xs, ys, zs, X);
    /* 2. starting scale */
    {
        double Ft[9], B[9], sB[9], sI[9];
        matmul3(X, M, Ft);
        orc_strain_stress(Ft, S, g, C11, C12, C44, NULL, B, NULL);
        for (int i = 0; i < 9; i++) B[i] = 2.0 * B[i] + I3[i]; /* F_S F_S^T */
        orc_stress(B, g, C11, C12, C44, sB);
        orc_stress(I3, g, C11, C12, C44, sI);
        double s2 = sI[8] / sB[8];
        if (!(s2 > 0.0) || !isfinite(s2)) {
            st |= ORC_SOLVE_ILLCOND;
            s2 = 1.0;
        }
        for (int i = 0; i < 9; i++) X[i] *= sqrt(s2);
    }
    /* 3. Lagrange-Newton */
    int done = 0;
    for (int it = 0; it < 100 && !done; it++) {
        double K[144], rhs[12], sol[12];
        memset(K, 0, sizeof K);
        memset(rhs, 0, sizeof rhs);
        for (int i = 0; i < n; i++) {
            double r[3] = {(cx[i] - xs) / zs, (cy[i] - ys) / zs, 1.0};
            double px = (cx[i] - xs + q[2 * i]) / zs, py = (cy[i] - ys + q[2 * i + 1]) / zs;
            double n1 = X[0] * r[0] + X[1] * r[1] + X[2] * r[2];
            double n2 = X[3] * r[0] + X[4] * r[1] + X[5] * r[2];
            double d = X[6] * r[0] + X[7] * r[1] + X[8] * r[2];
            double ex = n1 / d - px, ey = n2 / d - py;
            double jx[9] = {r[0] / d, r[1] / d, r[2] / d, 0, 0, 0,
                            -n1 * r[0] / (d * d), -n1 * r[1] / (d * d), -n1 * r[2] / (d * d)};
            double jy[9] = {0, 0, 0, r[0] / d, r[1] / d, r[2] / d,
                            -n2 * r[0] / (d * d), -n2 * r[1] / (d * d), -n2 * r[2] / (d * d)};
            for (int a = 0; a < 9; a++) {
                rhs[a] -= jx[a] * ex + jy[a] * ey;
                for (int b = 0; b < 9; b++) K[12 * a + b] += jx[a] * jx[b] + jy[a] * jy[b];
            }
        }
        double c[3], A[27];
        traction_terms(X, M, S, g, C11, C12, C44, c, A);
        for (int k = 0; k < 3; k++) {
            rhs[9 + k] = -c[k];
            for (int a = 0; a < 9; a++) {
                K[12 * (9 + k) + a] = A[9 * k + a];
                K[12 * a + 9 + k] = A[9 * k + a];
            }
        }
        if (orc_gauss_solve(K, rhs, 12, sol)) {
            st |= ORC_SOLVE_ILLCOND;
            break;
        }
        double nrm = 0.0;
        for (int a = 0; a < 9; a++) {
            X[a] += sol[a];
            nrm += sol[a] * sol[a];
        }
        if (!isfinite(nrm)) {
            st |= ORC_SOLVE_ILLCOND;
            break;
        }
        if (sqrt(nrm) < 1e-14) done = 1;
    }
    if (!done) st |= ORC_SOLVE_ILLCOND;
    matmul3(X, M, F);
    orc_strain_stress(F, S, g, C11, C12, C44, NULL, eps, sig);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Polar rotation, Eq. (4)-(5): F = P D Q^T (SVD), R = P Q^T.  With the
 * eigen-decomposition F^T F = Q D^2 Q^T, P = F Q D^-1 and so
 * R = F Q D^-1 Q^T.  If det R < 0 the last column of P is negated.        */
void orc_polar(const double* F, double* R)
{
    double C[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0.0;
            for (int k = 0; k < 3; k++) s += F[k * 3 + i] * F[k * 3 + j];
            C[i * 3 + j] = s;
        }
    double ev[3], Q[9];
    orc_jacobi_eig(C, 3, ev, Q);
    double P[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0.0;
            for (int k = 0; k < 3; k++) s += F[i * 3 + k] * Q[k * 3 + j];
            P[i * 3 + j] = s / sqrt(ev[j]);
        }
    /* R = P Q^T */
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0.0;
            for (int k = 0; k < 3; k++) s += P[i * 3 + k] * Q[j * 3 + k];
            R[i * 3 + j] = s;
        }
    if (det3(R) < 0.0) {
        /* pick the column of P belonging to the smallest singular value */
        int kmin = 0;
        for (int k = 1; k < 3; k++)
            if (ev[k] < ev[kmin]) kmin = k;
        for (int i = 0; i < 3; i++) P[i * 3 + kmin] = -P[i * 3 + kmin];
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) {
                double s = 0.0;
                for (int k = 0; k < 3; k++) s += P[i * 3 + k] * Q[j * 3 + k];
                R[i * 3 + j] = s;
            }
    }
}

/* Axis-angle of R (the passage after Eq. (5)), written with atan2 so small
 * angles keep their digits: w = (R32-R23, R13-R31, R21-R12)/2 = sin(theta) m,
 * theta = atan2(|w|, (tr R - 1)/2), rotation vector theta_k = theta m_k.   */
/* Eq. (6): the rotation tensor of a rotation vector theta (the axis times
 * the angle), omega_ij = -eps_ijk theta_k (eps the permutation symbol),
 * row-major 3 x 3.                                                         */
void orc_omega(const double* th, double* om)
{
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double v = 0.0;
            for (int k = 0; k < 3; k++) {
                /* eps_ijk = (i - j)(j - k)(k - i) / 2 for indices 0..2 */
                const int e = (i - j) * (j - k) * (k - i) / 2;
                v -= (double)e * th[k];
            }
            om[3 * i + j] = v;
        }
}

void orc_rotvec(const double* R, double* rv)
{
    double w0 = 0.5 * (R[7] - R[5]);
    double w1 = 0.5 * (R[2] - R[6]);
    double w2 = 0.5 * (R[3] - R[1]);
    double s = sqrt(w0 * w0 + w1 * w1 + w2 * w2);
    double c = 0.5 * (R[0] + R[4] + R[8] - 1.0);
    double th = atan2(s, c);
    if (s == 0.0) {
        rv[0] = rv[1] = rv[2] = 0.0;
        return;
    }
    rv[0] = th * w0 / s;
    rv[1] = th * w1 / s;
    rv[2] = th * w2 / s;
}

/* ------------------------------------------------------------------------ */
/* Cubic B-spline interpolation (the paper remaps with a cubic scheme; the
 * reading here is the interpolating cubic B-spline).  The image s is
 * extended by whole-sample mirroring (s[-k] = s[k], s[N-1+k] = s[N-1-k]);
 * the coefficients c solve sum_k c[k] beta3(x - k) = s[x] at every integer x,
 * separably along rows then columns.  Along one line that is the inverse of
 * the filter (1, 4, 1)/6, factored into a causal and an anti-causal
 * first-order recursion with pole z = sqrt(3) - 2 (Unser, Aldroubi & Eden,
 * IEEE Trans. Signal Process. 41 (1993) 821-833):
 *   c+[0] = sum_{k=0}^{2N-3} z^k s~[k] / (1 - z^(2N-2))   (s~ = the mirror
 *           extension, period 2N-2: the exact start for that extension)
 *   c+[k] = s[k] + z c+[k-1]
 *   c-[N-1] = z / (z^2 - 1) (c+[N-1] + z c+[N-2])
 *   c-[k] = z (c-[k+1] - c+[k])
 *   c[k] = 6 c-[k].
 * N == 1 gives c = s.                                                       */
static void bspline_line(double* v, int N, size_t stride)
{
    if (N < 2) return;
    const double z = sqrt(3.0) - 2.0;
    const int P = 2 * N - 2;
    double zk = 1.0, acc = 0.0;
    for (int k = 0; k < P; k++) {
        int m = k < N ? k : P - k;
        acc += zk * v[(size_t)m * stride];
        zk *= z;
    }
    double* cp = (double*)malloc(sizeof(double) * N);
    cp[0] = acc / (1.0 - zk);
    for (int k = 1; k < N; k++) cp[k] = v[(size_t)k * stride] + z * cp[k - 1];
    double cm = z / (z * z - 1.0) * (cp[N - 1] + z * cp[N - 2]);
    v[(size_t)(N - 1) * stride] = 6.0 * cm;
    for (int k = N - 2; k >= 0; k--) {
        cm = z * (cm - cp[k]);
        v[(size_t)k * stride] = 6.0 * cm;
    }
    free(cp);
}

void orc_bspline_coeffs(const double* img, int H, int W, double* c)
{
    memcpy(c, img, sizeof(double) * (size_t)H * W);
    for (int y = 0; y < H; y++) bspline_line(c + (size_t)y * W, W, 1);
    for (int x = 0; x < W; x++) bspline_line(c + x, H, (size_t)W);
}

/* Whole-sample mirror of index i into [0, N-1]. */
static int mirror_index(int i, int N)
{
    if (N == 1) return 0;
    const int P = 2 * N - 2;
    int m = i % P;
    if (m < 0) m += P;
    return m < N ? m : P - m;
}

/* Cubic B-spline  beta3(t) = (4 - 6t^2 + 3|t|^3)/6 for |t| <= 1,
 * (2 - |t|)^3/6 for 1 < |t| < 2, else 0. */
static double beta3(double t)
{
    t = fabs(t);
    if (t < 1.0) return (4.0 - 6.0 * t * t + 3.0 * t * t * t) / 6.0;
    if (t < 2.0) return (2.0 - t) * (2.0 - t) * (2.0 - t) / 6.0;
    return 0.0;
}

/* Interpolant sum_{j,k} c[j][k] beta3(y - j) beta3(x - k) at (x, y), with
 * the coordinates clamped to [0, W-1] x [0, H-1] as for the bilinear
 * sample, coefficients indexed through the mirror extension. */
double orc_bspline_at(const double* c, int H, int W, double x, double y)
{
    double xc = clampd(x, 0.0, (double)(W - 1));
    double yc = clampd(y, 0.0, (double)(H - 1));
    int ix = (int)floor(xc), iy = (int)floor(yc);
    double acc = 0.0;
    for (int j = iy - 1; j <= iy + 2; j++) {
        double wy = beta3(yc - (double)j);
        const double* row = c + (size_t)mirror_index(j, H) * W;
        for (int k = ix - 1; k <= ix + 2; k++)
            acc += wy * beta3(xc - (double)k) * row[mirror_index(k, W)];
    }
    return acc;
}

void orc_bspline_points(const double* c, int H, int W, const double* xs, const double* ys,
                        int64_t n, double* out)
{
    for (int64_t i = 0; i < n; i++) out[i] = orc_bspline_at(c, H, W, xs[i], ys[i]);
}

/* Remap of the reference by R_finite (section 2, before Eq. (12)), R
 * row-major:
 *   Rm(x') = ref(pi(R^T r(x'))),  r(x) = (x - x*, y - y*, Z*),
 *   pi(v) = (x* + Z* v_x/v_z, y* + Z* v_y/v_z);
 * interp 3: cubic B-spline interpolation (above), interp 1: bilinear; both
 * clamp the sample position to the pattern.  With R = (F^-1)^T for a
 * deformation gradient F the same map remaps by F (pi is scale-invariant). */
void orc_remap(const double* ref, int H, int W, const double* Rf, double xs, double ys,
               double zs, int interp, double* out)
{
    double* c = NULL;
    if (interp == 3) {
        c = (double*)malloc(sizeof(double) * (size_t)H * W);
        orc_bspline_coeffs(ref, H, W, c);
    }
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            double r0 = x - xs, r1 = y - ys, r2 = zs;
            double v0 = Rf[0] * r0 + Rf[3] * r1 + Rf[6] * r2;
            double v1 = Rf[1] * r0 + Rf[4] * r1 + Rf[7] * r2;
            double v2 = Rf[2] * r0 + Rf[5] * r1 + Rf[8] * r2;
            double sx = xs + zs * v0 / v2, sy = ys + zs * v1 / v2;
            out[(size_t)y * W + x] = c ? orc_bspline_at(c, H, W, sx, sy) : orc_bilinear(ref, H, W, sx, sy);
        }
    free(c);
}

/* ------------------------------------------------------------------------ */
/* Radix-2 Cooley-Tukey FFT (decimation in time, bit-reversed input order),
 * forward kernel exp(-2 pi i k n / N); the inverse uses exp(+...) and
 * divides by N.  N must be a power of two.                                 */
void orc_fft1(double* re, double* im, int N, int inverse)
{
    const double pi = 3.14159265358979323846;
    for (int i = 1, j = 0; i < N; i++) {
        int bit = N >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            double t = re[i];
            re[i] = re[j];
            re[j] = t;
            t = im[i];
            im[i] = im[j];
            im[j] = t;
        }
    }
    for (int len = 2; len <= N; len <<= 1) {
        double ang = (inverse ? 2.0 : -2.0) * pi / (double)len;
        for (int i = 0; i < N; i += len)
            for (int k = 0; k < len / 2; k++) {
                double wr = cos(ang * k), wi = sin(ang * k);
                int a = i + k, b = i + k + len / 2;
                double xr = re[b] * wr - im[b] * wi;
                double xi = re[b] * wi + im[b] * wr;
                re[b] = re[a] - xr;
                im[b] = im[a] - xi;
                re[a] += xr;
                im[a] += xi;
            }
    }
    if (inverse)
        for (int i = 0; i < N; i++) {
            re[i] /= (double)N;
            im[i] /= (double)N;
        }
}

/* 2-D FFT of an N x N row-major array: rows, then columns. */
void orc_fft2(double* re, double* im, int N, int inverse)
{
    double* cr = (double*)malloc(sizeof(double) * N);
    double* ci = (double*)malloc(sizeof(double) * N);
    for (int y = 0; y < N; y++) orc_fft1(re + (size_t)y * N, im + (size_t)y * N, N, inverse);
    for (int x = 0; x < N; x++) {
        for (int y = 0; y < N; y++) {
            cr[y] = re[(size_t)y * N + x];
            ci[y] = im[(size_t)y * N + x];
        }
        orc_fft1(cr, ci, N, inverse);
        for (int y = 0; y < N; y++) {
            re[(size_t)y * N + x] = cr[y];
            im[(size_t)y * N + x] = ci[y];
        }
    }
    free(cr);
    free(ci);
}

/* ------------------------------------------------------------------------ */
/* Sub-pixel offset of a correlation peak (section 2 interpolates the peak of
 * the cross-correlation): the quadratic surface through the 3 x 3
 * neighbourhood nb[(dy + 1) * 3 + (dx + 1)], dx, dy in {-1, 0, 1}, around the
 * integer maximum.  Central differences give its gradient g = (Cx, Cy) and
 * Hessian Hs = [[Cxx, Cxy], [Cxy, Cyy]] at the centre, exactly for a
 * quadratic; its stationary point d = -Hs^-1 g is the peak when Hs is
 * negative definite (Cxx < 0 and det Hs > 0).  Each component is clamped to
 * +-1; a surface that is not negative definite gives d = 0 (return 0).      */
int orc_peak_subpixel(const double* nb, double* d)
{
#define NB(dy, dx) nb[((dy) + 1) * 3 + ((dx) + 1)]
    const double c0 = NB(0, 0);
    const double gx = 0.5 * (NB(0, 1) - NB(0, -1));
    const double gy = 0.5 * (NB(1, 0) - NB(-1, 0));
    const double hxx = NB(0, 1) - 2.0 * c0 + NB(0, -1);
    const double hyy = NB(1, 0) - 2.0 * c0 + NB(-1, 0);
    const double hxy = 0.25 * (NB(1, 1) - NB(1, -1) - NB(-1, 1) + NB(-1, -1));
#undef NB
    const double det = hxx * hyy - hxy * hxy;
    d[0] = 0.0;
    d[1] = 0.0;
    if (!(hxx < 0.0 && det > 0.0)) return 0;
    d[0] = clampd(-(hyy * gx - hxy * gy) / det, -1.0, 1.0);
    d[1] = clampd(-(hxx * gy - hxy * gx) / det, -1.0, 1.0);
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Maximum of the band-limited interpolant of a correlation (a reading of
 * section 2's interpolated peak).  C is the inverse DFT of the cross-power
 * spectrum P (N x N, k = 0..N-1, row = k_y); between the samples C is
 * continued by its Fourier series,
 *   C(x, y) = Re (1/N^2) sum_k P(k) exp(2 pi i (k_x' x + k_y' y) / N),
 * with signed frequencies k' = k for k < N/2, k - N otherwise, which agrees
 * with C at every integer point.  Newton's method on grad C = 0 with the
 * exact gradient and Hessian of the series, from (x, y) (the quadratic
 * estimate in signed shift coordinates), until the step is below 1e-12 px
 * (at most 30 steps).  Returns 0 and leaves (x, y) when a Hessian is not
 * negative definite or the iterate leaves the unit square around the
 * starting integer peak (kx, ky), 1 on success.                            */
int orc_peak_fourier(const double* Pre, const double* Pim, int N, int sx, int sy, double* x, double* y)
{
    const double pi = 3.14159265358979323846;
    double cx = *x, cy = *y;
    double* ex_re = (double*)malloc(sizeof(double) * N);
    double* ex_im = (double*)malloc(sizeof(double) * N);
    double* ey_re = (double*)malloc(sizeof(double) * N);
    double* ey_im = (double*)malloc(sizeof(double) * N);
    int ok = 0;
    for (int it = 0; it < 30; it++) {
        for (int k = 0; k < N; k++) {
            const int ks = k < N / 2 ? k : k - N;
            ex_re[k] = cos(2.0 * pi * ks * cx / N);
            ex_im[k] = sin(2.0 * pi * ks * cx / N);
            ey_re[k] = cos(2.0 * pi * ks * cy / N);
            ey_im[k] = sin(2.0 * pi * ks * cy / N);
        }
        double gx = 0.0, gy = 0.0, hxx = 0.0, hxy = 0.0, hyy = 0.0;
        for (int ky = 0; ky < N; ky++) {
            const double fy = 2.0 * pi * (ky < N / 2 ? ky : ky - N) / N;
            for (int kx = 0; kx < N; kx++) {
                const double fx = 2.0 * pi * (kx < N / 2 ? kx : kx - N) / N;
                const size_t i = (size_t)ky * N + kx;
                /* e = exp(i (fx x + fy y)) */
                const double er = ex_re[kx] * ey_re[ky] - ex_im[kx] * ey_im[ky];
                const double ei = ex_re[kx] * ey_im[ky] + ex_im[kx] * ey_re[ky];
                const double tr = Pre[i] * er - Pim[i] * ei; /* Re(P e) */
                const double ti = Pre[i] * ei + Pim[i] * er; /* Im(P e) */
                gx -= fx * ti;
                gy -= fy * ti;
                hxx -= fx * fx * tr;
                hxy -= fx * fy * tr;
                hyy -= fy * fy * tr;
            }
        }
        const double det = hxx * hyy - hxy * hxy;
        if (!(hxx < 0.0 && det > 0.0)) break;
        const double dx = -(hyy * gx - hxy * gy) / det;
        const double dy = -(hxx * gy - hxy * gx) / det;
        cx += dx;
        cy += dy;
        if (fabs(cx - sx) > 1.0 || fabs(cy - sy) > 1.0) break;
        if (sqrt(dx * dx + dy * dy) < 1e-12) {
            ok = 1;
            break;
        }
    }
    free(ex_re);
    free(ex_im);
    free(ey_re);
    free(ey_im);
    if (ok) {
        *x = cx;
        *y = cy;
    }
    return ok;
}

/* ------------------------------------------------------------------------ */
/* ROI cross-correlation and its peak (section 2).
 *   A = reference ROI, B = test ROI (N x N); each loses its own mean, is
 *   multiplied by the symmetric Hann window h (x) h, h[n] = 0.5 - 0.5
 *   cos(2 pi n/(N-1)) (window = 0: no window);
 *   C = Re IFFT2( FFT2(B w) . conj(FFT2(A w)) ), so B(x) = A(x - s) puts the
 *   peak at +s;
 *   integer peak = argmax C, ties to the lowest row-major index; index
 *   k >= N/2 means k - N;
 *   sub-pixel (the paper interpolates the peak): the 2-D quadratic through the
 *   3 x 3 circular neighbourhood of the integer peak, with central
 *   differences g = (dC/dx, dC/dy) and Hessian Hs = [[Cxx, Cxy], [Cxy, Cyy]];
 *   d = -Hs^-1 g when Hs is negative definite (Cxx < 0, det > 0), each
 *   component clamped to +-1, else d = 0.  Band-pattern correlation peaks
 *   are tilted ridges, which per-axis fits mislocate;
 *   peak height PH = C_max / sqrt(sum (A w)^2 sum (B w)^2).
 * C (optional) receives the N x N correlation.  q = (x shift, y shift).   */
void orc_xcf_fit(const double* A, const double* B, int N, int window, int peak_fit, double* C, double* q,
                 double* ph);

void orc_xcf(const double* A, const double* B, int N, int window, double* C, double* q, double* ph)
{
    orc_xcf_fit(A, B, N, window, 0, C, q, ph);
}

/* peak_fit 0: the 2-D quadratic fit of the 3 x 3 neighbourhood; 1: then the
 * maximum of the band-limited interpolant (orc_peak_fourier) from there. */
void orc_xcf_fit(const double* A, const double* B, int N, int window, int peak_fit, double* C, double* q,
                 double* ph)
{
    const double pi = 3.14159265358979323846;
    size_t NN = (size_t)N * N;
    double* ar = (double*)malloc(sizeof(double) * NN);
    double* ai = (double*)calloc(NN, sizeof(double));
    double* br = (double*)malloc(sizeof(double) * NN);
    double* bi = (double*)calloc(NN, sizeof(double));
    double* h = (double*)malloc(sizeof(double) * N);
    for (int n = 0; n < N; n++) h[n] = window ? 0.5 - 0.5 * cos(2.0 * pi * n / (double)(N - 1)) : 1.0;
    double ma = 0.0, mb = 0.0;
    for (size_t i = 0; i < NN; i++) {
        ma += A[i];
        mb += B[i];
    }
    ma /= (double)NN;
    mb /= (double)NN;
    double ea = 0.0, eb = 0.0;
    for (int y = 0; y < N; y++)
        for (int x = 0; x < N; x++) {
            size_t i = (size_t)y * N + x;
            double w = h[y] * h[x];
            ar[i] = (A[i] - ma) * w;
            br[i] = (B[i] - mb) * w;
            ea += ar[i] * ar[i];
            eb += br[i] * br[i];
        }
    orc_fft2(ar, ai, N, 0);
    orc_fft2(br, bi, N, 0);
    /* P = FB . conj(FA) */
    for (size_t i = 0; i < NN; i++) {
        double pr = br[i] * ar[i] + bi[i] * ai[i];
        double pi_ = bi[i] * ar[i] - br[i] * ai[i];
        br[i] = pr;
        bi[i] = pi_;
    }
    /* the spectrum, kept for the interpolant (ar, ai are free from here) */
    memcpy(ar, br, sizeof(double) * NN);
    memcpy(ai, bi, sizeof(double) * NN);
    orc_fft2(br, bi, N, 1);
    size_t best = 0;
    for (size_t i = 1; i < NN; i++)
        if (br[i] > br[best]) best = i;
    int ky = (int)(best / N), kx = (int)(best % N);
    double c0 = br[best];
    double nb[9], d[2];
    for (int dy = -1; dy <= 1; dy++)
        for (int dx = -1; dx <= 1; dx++)
            nb[(dy + 1) * 3 + (dx + 1)] = br[(size_t)((ky + dy + N) % N) * N + (size_t)((kx + dx + N) % N)];
    orc_peak_subpixel(nb, d);
    int sx = kx < N / 2 ? kx : kx - N;
    int sy = ky < N / 2 ? ky : ky - N;
    q[0] = sx + d[0];
    q[1] = sy + d[1];
    if (peak_fit == 1) {
        /* C = IFFT(P) carries the 1/N^2 of the inverse transform */
        for (size_t i = 0; i < NN; i++) {
            ar[i] /= (double)NN;
            ai[i] /= (double)NN;
        }
        orc_peak_fourier(ar, ai, N, sx, sy, &q[0], &q[1]);
    }
    double nrm = sqrt(ea * eb);
    *ph = nrm > 0.0 ? c0 / nrm : 0.0;
    if (C) memcpy(C, br, sizeof(double) * NN);
    free(ar);
    free(ai);
    free(br);
    free(bi);
    free(h);
}

/* ------------------------------------------------------------------------ */
/* Mean angular error of an Eq. (3) fit, the quality figure section 3
 * compares the four methods by (its formula is not given; this is the
 * reading used here): for ROI i the angle between the direction the fitted
 * model assigns to the ROI centre, F r_i, and the measured one,
 * (r_i + q_i) on the screen plane z = Z*, as atan2(|a x b|, a . b); the
 * mean over the n ROIs, in rad.                                           */
double orc_mae(const double* q, const double* cx, const double* cy, int n, double xs, double ys,
               double zs, const double* F)
{
    double sum = 0.0;
    for (int i = 0; i < n; i++) {
        double r[3] = {cx[i] - xs, cy[i] - ys, zs};
        double a[3], b[3] = {r[0] + q[2 * i], r[1] + q[2 * i + 1], zs};
        for (int k = 0; k < 3; k++) a[k] = F[3 * k] * r[0] + F[3 * k + 1] * r[1] + F[3 * k + 2] * r[2];
        double c0 = a[1] * b[2] - a[2] * b[1];
        double c1 = a[2] * b[0] - a[0] * b[2];
        double c2 = a[0] * b[1] - a[1] * b[0];
        sum += atan2(sqrt(c0 * c0 + c1 * c1 + c2 * c2), a[0] * b[0] + a[1] * b[1] + a[2] * b[2]);
    }
    return n > 0 ? sum / n : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Whole pipeline for one pair.
 *   demons (first pass) -> q1 at the ROI centres -> F1 (Eq. 3) ->
 *   R_finite = polar(F1) (Eq. 4-5) -> remap the reference by R_finite ->
 *   XCF per ROI -> q2 -> F_inf (Eq. 3) -> F = F_inf R_finite (Eq. 12),
 *   det F = 1 -> R = polar(F) -> rotation vector.
 * With xcf_passes = P > 1 the remap + XCF + compose step runs P times, pass
 * k remapping by the whole F of pass k-1 in place of R_finite and composing
 * F_inf with that F; q2 and ph are the last pass's.
 * rfin_in (optional) replaces the first pass's R_finite: it lets the second
 * pass be checked in isolation against another implementation's R_finite.
 * first_pass = 1 replaces demons by the conventional first pass (section 1;
 * method (c) of the comparison in section 3, method (a) without the second
 * pass): q1 is the ROI cross-correlation of the normalised, unremapped
 * patterns (same XCF as the second pass), the field is zero and no
 * iterations run; ph then holds that XCF's peak heights unless a second
 * pass overwrites them.  mae1 / mae: mean angular error (orc_mae) of the
 * first fit (F1 to q1) and of the last fit (F_inf to the last q2; F1 to q1
 * without a second pass).
 * Any output pointer may be NULL.                                         */
typedef struct {
    double* field;   /* [2][H][W] full-res px */
    double* q1;      /* [n_roi][2] */
    double* F1;      /* [9] */
    double* Rfin;    /* [9] */
    double* q2;      /* [n_roi][2] */
    double* ph;      /* [n_roi] */
    double* F;       /* [9] */
    double* R;       /* [9] */
    double* rotvec;  /* [3] */
    int32_t* iters;  /* [levels] */
    uint32_t* status;
    double* mae1;    /* [1] */
    double* mae;     /* [1] */
    double* ssim;    /* [1] orc_ssim of the final field (NaN with the XCF first pass) */
    double* omega;   /* [9] Eq. (6)'s rotation tensor of rotvec */
} orc_outputs;

static void store(double* dst, const double* src, size_t n)
{
    if (dst) memcpy(dst, src, sizeof(double) * n);
}

int orc_register_pair(const float* ref, const float* test, int H, int W, const orc_params* p,
                      const double* u_init, const double* rfin_in, const orc_outputs* o)
{
    size_t HW = (size_t)H * W;
    int nr = p->n_roi, N = p->roi_size;
    double* Rn = (double*)malloc(sizeof(double) * HW);
    double* Tn = (double*)malloc(sizeof(double) * HW);
    double* field = (double*)malloc(sizeof(double) * 2 * HW);
    double* cx = (double*)malloc(sizeof(double) * nr);
    double* cy = (double*)malloc(sizeof(double) * nr);
    int32_t* x0 = (int32_t*)malloc(sizeof(int32_t) * nr);
    int32_t* y0 = (int32_t*)malloc(sizeof(int32_t) * nr);
    double* q1 = (double*)malloc(sizeof(double) * 2 * nr);
    double* q2 = (double*)calloc(2 * (size_t)nr, sizeof(double));
    double* ph = (double*)calloc((size_t)nr, sizeof(double));
    int32_t its[ORC_MAX_LEVELS] = {0};
    uint32_t st = 0;
    const double* bg = p->background_static ? p->background : NULL;
    if (bg || p->background_dynamic > 0.0 || p->bandpass_lo > 0.0 || p->bandpass_hi > 0.0) {
        /* background correction, then the pre-filter, then the z-score */
        double* f = (double*)malloc(sizeof(double) * HW);
        double* g = (double*)malloc(sizeof(double) * HW);
        for (int k = 0; k < 2; k++) {
            orc_background(k == 0 ? ref : test, H, W, bg, p->background_dynamic, f);
            orc_bandpass_d(f, H, W, p->bandpass_lo, p->bandpass_hi, g);
            st |= orc_normalize_d(g, (int64_t)HW, k == 0 ? Rn : Tn);
        }
        free(f);
        free(g);
    } else {
        st |= orc_normalize(ref, (int64_t)HW, Rn);
        st |= orc_normalize(test, (int64_t)HW, Tn);
    }
    orc_roi_layout(H, W, p, cx, cy, x0, y0);
    double* a = (double*)malloc(sizeof(double) * N * N);
    double* b = (double*)malloc(sizeof(double) * N * N);
    if (p->first_pass == 1) {
        /* conventional first pass: XCF of each ROI of the unremapped patterns */
        memset(field, 0, sizeof(double) * 2 * HW);
        for (int j = 0; j < nr; j++) {
            for (int y = 0; y < N; y++)
                for (int x = 0; x < N; x++) {
                    a[y * N + x] = Rn[(size_t)(y0[j] + y) * W + x0[j] + x];
                    b[y * N + x] = Tn[(size_t)(y0[j] + y) * W + x0[j] + x];
                }
            orc_xcf_fit(a, b, N, p->window, p->peak_fit, NULL, q1 + 2 * j, ph + j);
        }
    } else {
        st |= orc_demons(Rn, Tn, H, W, p, u_init, field, its);
        double* ux = field;
        double* uy = field + HW;
        for (int j = 0; j < nr; j++) {
            q1[2 * j] = orc_bilinear(ux, H, W, cx[j], cy[j]);
            q1[2 * j + 1] = orc_bilinear(uy, H, W, cx[j], cy[j]);
        }
    }
    double ssim = NAN;
    if (p->first_pass != 1 && o->ssim) {
        double* Tw = (double*)malloc(sizeof(double) * HW);
        orc_warp(Tn, H, W, field, Tw);
        ssim = orc_ssim(Rn, Tw, H, W);
        free(Tw);
    }
    double xs = p->pc_x * W - 0.5, ys = p->pc_y * H - 0.5, zs = p->pc_z * W;
    double F1[9], Rfin[9], F[9], R[9], rv[3];
    st |= orc_solve_F(q1, cx, cy, nr, xs, ys, zs, F1);
    double mae1 = orc_mae(q1, cx, cy, nr, xs, ys, zs, F1), mae = mae1;
    orc_polar(F1, Rfin);
    if (rfin_in) memcpy(Rfin, rfin_in, sizeof Rfin);
    if (p->second_pass) {
        /* pass 1 remaps by R_finite and composes with it (Eq. 12); each
         * further pass remaps by the whole F of the previous pass, the source
         * direction of x' being F^-1 r(x') (orc_remap with (F^-1)^T), and
         * composes with that F. */
        int passes = p->xcf_passes > 1 ? p->xcf_passes : 1;
        double Rcur[9], Fprev[9];
        memcpy(Rcur, Rfin, sizeof Rcur);
        memcpy(Fprev, Rfin, sizeof Fprev);
        double* Rm = (double*)malloc(sizeof(double) * HW);
        for (int pass = 0; pass < passes; pass++) {
            orc_remap(Rn, H, W, Rcur, xs, ys, zs, p->remap_interp, Rm);
            for (int j = 0; j < nr; j++) {
                for (int y = 0; y < N; y++)
                    for (int x = 0; x < N; x++) {
                        a[y * N + x] = Rm[(size_t)(y0[j] + y) * W + x0[j] + x];
                        b[y * N + x] = Tn[(size_t)(y0[j] + y) * W + x0[j] + x];
                    }
                orc_xcf_fit(a, b, N, p->window, p->peak_fit, NULL, q2 + 2 * j, ph + j);
            }
            double Finf[9];
            st |= orc_solve_F(q2, cx, cy, nr, xs, ys, zs, Finf);
            mae = orc_mae(q2, cx, cy, nr, xs, ys, zs, Finf);
            matmul3(Finf, Fprev, F);
            if (det3(F) > 0.0) orc_det_normalize(F);
            memcpy(Fprev, F, sizeof Fprev);
            inv3_transposed(F, Rcur);
        }
        free(Rm);
    } else {
        memcpy(F, F1, sizeof F);
    }
    free(a);
    free(b);
    orc_polar(F, R);
    orc_rotvec(R, rv);
    store(o->field, field, 2 * HW);
    store(o->q1, q1, 2 * (size_t)nr);
    store(o->F1, F1, 9);
    store(o->Rfin, Rfin, 9);
    store(o->q2, q2, 2 * (size_t)nr);
    store(o->ph, ph, (size_t)nr);
    store(o->F, F, 9);
    store(o->R, R, 9);
    store(o->rotvec, rv, 3);
    if (o->omega) orc_omega(rv, o->omega);
    if (o->iters) memcpy(o->iters, its, sizeof(int32_t) * p->levels);
    if (o->status) *o->status = st;
    store(o->mae1, &mae1, 1);
    store(o->mae, &mae, 1);
    store(o->ssim, &ssim, 1);
    free(Rn);
    free(Tn);
    free(field);
    free(cx);
    free(cy);
    free(x0);
    free(y0);
    free(q1);
    free(q2);
    free(ph);
    return 0;
}

/* Batch over pairs (independent scan points), one pair per OpenMP thread.
 * refs/tests: [n][H][W] float; outputs are strided per pair like the
 * single-pair call (field [n][2][H][W], q [n][n_roi][2], F/R [n][9], ...).
 * rfin_in, if not NULL, is [n][9].  Returns the number of threads used.   */
int orc_register_batch(const float* refs, const float* tests, int n, int H, int W,
                       const orc_params* p, const double* rfin_in, const orc_outputs* o)
{
    size_t HW = (size_t)H * W;
    int nr = p->n_roi;
    int used = 1;
    orc_params pb = *p;
    double* bgm = NULL;
    if (p->background_static && !p->background) {
        bgm = (double*)malloc(sizeof(double) * HW);
        orc_mean_pattern(tests, n, H, W, bgm);
        pb.background = bgm;
    }
    p = &pb;
#pragma omp parallel
    {
#ifdef _OPENMP
#pragma omp single
        used = omp_get_num_threads();
#endif
#pragma omp for schedule(dynamic, 1)
        for (int i = 0; i < n; i++) {
            orc_outputs oi;
            oi.field = o->field ? o->field + (size_t)i * 2 * HW : NULL;
            oi.q1 = o->q1 ? o->q1 + (size_t)i * 2 * nr : NULL;
            oi.F1 = o->F1 ? o->F1 + (size_t)i * 9 : NULL;
            oi.Rfin = o->Rfin ? o->Rfin + (size_t)i * 9 : NULL;
            oi.q2 = o->q2 ? o->q2 + (size_t)i * 2 * nr : NULL;
            oi.ph = o->ph ? o->ph + (size_t)i * nr : NULL;
            oi.F = o->F ? o->F + (size_t)i * 9 : NULL;
            oi.R = o->R ? o->R + (size_t)i * 9 : NULL;
            oi.rotvec = o->rotvec ? o->rotvec + (size_t)i * 3 : NULL;
            oi.iters = o->iters ? o->iters + (size_t)i * p->levels : NULL;
            oi.status = o->status ? o->status + i : NULL;
            oi.mae1 = o->mae1 ? o->mae1 + i : NULL;
            oi.mae = o->mae ? o->mae + i : NULL;
            oi.ssim = o->ssim ? o->ssim + i : NULL;
            oi.omega = o->omega ? o->omega + (size_t)i * 9 : NULL;
            orc_register_pair(refs + (size_t)i * HW, tests + (size_t)i * HW, H, W, p, NULL,
                              rfin_in ? rfin_in + (size_t)i * 9 : NULL, &oi);
        }
    }
    free(bgm);
    return used;
}
