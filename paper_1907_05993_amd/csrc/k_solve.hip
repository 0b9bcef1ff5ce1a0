// Per-pair FP64 solves for gfx950 (arXiv:1907.05993 section 2):
//   Eq. (2) projective model r' = r + q = Z* F r / ((F r) . k), Eq. (3) least
//   squares over the ROI shifts (direct linear start, then Gauss-Newton on the
//   8 entries left free by F33 = 1), det F = 1 normalisation (the shifts fix F
//   only up to scale), rotation R = P Q^T of F = P D Q^T (Eq. (4)-(5)) written as
//   R = F (F^T F)^(-1/2), composition F = F_inf R_finite (Eq. (12)) and the
//   rotation vector theta m (axis-angle after Eq. (5)) with theta from atan2 so
//   small angles keep their digits.
// One wavefront per pair for the registration's solves (the sums over the ROIs
// on the lanes, see solve_F_wave); one thread per pair for the traction-free
// solve, whose dense algebra with data-dependent indices (the Jacobi
// eigen-solver, the 12 x 13 Lagrange-Newton system) works on matrices in LDS,
// one column of words per thread, so that no array goes to scratch memory; the
// small fixed-index algebra stays in registers.
#include "ebsd_internal.h"
#include "cnn_internal.h"

#include "../../include/ebsd.h"

namespace ebsd {

namespace {

// Cyclic Jacobi eigen-decomposition of a symmetric n x n matrix (destroyed);
// columns of V are the eigenvectors.  Small n: every loop is unrolled so the
// matrices stay in registers.
template <int n>
__device__ void jacobi_eigen(double (&A)[n][n], double (&ev)[n], double (&V)[n][n])
{
#pragma unroll
    for (int i = 0; i < n; i++)
#pragma unroll
        for (int j = 0; j < n; j++) V[i][j] = i == j ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 60; sweep++) {
        double off = 0.0, diag = 0.0;
#pragma unroll
        for (int i = 0; i < n; i++) {
            diag += A[i][i] * A[i][i];
#pragma unroll
            for (int j = i + 1; j < n; j++) off += 2.0 * A[i][j] * A[i][j];
        }
        if (off == 0.0 || off <= 1e-30 * (off + diag)) break;
#pragma unroll
        for (int p = 0; p < n - 1; p++)
#pragma unroll
            for (int q = p + 1; q < n; q++) {
                const double apq = A[p][q];
                if (apq == 0.0) continue;
                const double tau = (A[q][q] - A[p][p]) / (2.0 * apq);
                const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                const double c = rsqrt(1.0 + t * t), s = t * c;
                for (int k = 0; k < n; k++) {
                    const double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; k++) {
                    const double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; k++) {
                    const double vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = c * vkp - s * vkq;
                    V[k][q] = s * vkp + c * vkq;
                }
            }
    }
    for (int i = 0; i < n; i++) ev[i] = A[i][i];
}

// Threads per block of the kernels that run solve_F, and the LDS words each
// thread needs for a 9 x 9 matrix and its eigenvectors.
constexpr int kSolveThreads = 32;
constexpr int kSolvePool = 2 * 81;

// n x n matrix of one thread in LDS: element (i, j) at p[(i n + j) kSolveThreads],
// p = block pool + thread index (the lanes of a wavefront read consecutive words).
template <int n>
struct LMat {
    double* p;
    __device__ double& operator()(int i, int j) const { return p[(i * n + j) * kSolveThreads]; }
};

// The same cyclic Jacobi iteration (same operation order, hence the same
// results) on LDS matrices.  WANT_V = false skips the eigenvectors (the
// eigenvalues do not depend on them).
template <int n, bool WANT_V = true>
__device__ void jacobi_eigen_l(LMat<n> A, double (&ev)[n], LMat<n> V)
{
    if constexpr (WANT_V) {
#pragma unroll
        for (int i = 0; i < n; i++)
#pragma unroll
            for (int j = 0; j < n; j++) V(i, j) = i == j ? 1.0 : 0.0;
    }
    for (int sweep = 0; sweep < 60; sweep++) {
        double off = 0.0, diag = 0.0;
#pragma unroll
        for (int i = 0; i < n; i++) {
            diag += A(i, i) * A(i, i);
#pragma unroll
            for (int j = i + 1; j < n; j++) off += 2.0 * A(i, j) * A(i, j);
        }
        if (off == 0.0 || off <= 1e-30 * (off + diag)) break;
        for (int p = 0; p < n - 1; p++)
            for (int q = p + 1; q < n; q++) {
                const double apq = A(p, q);
                if (apq == 0.0) continue;
                const double tau = (A(q, q) - A(p, p)) / (2.0 * apq);
                const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                const double c = rsqrt(1.0 + t * t), s = t * c;
                // each update reads its two lines whole before writing them
                // (the element updates of a line are independent), so the
                // LDS reads of a line are in flight together
                double lp[n], lq[n];
#pragma unroll
                for (int k = 0; k < n; k++) {
                    lp[k] = A(k, p);
                    lq[k] = A(k, q);
                }
#pragma unroll
                for (int k = 0; k < n; k++) {
                    A(k, p) = c * lp[k] - s * lq[k];
                    A(k, q) = s * lp[k] + c * lq[k];
                }
#pragma unroll
                for (int k = 0; k < n; k++) {
                    lp[k] = A(p, k);
                    lq[k] = A(q, k);
                }
#pragma unroll
                for (int k = 0; k < n; k++) {
                    A(p, k) = c * lp[k] - s * lq[k];
                    A(q, k) = s * lp[k] + c * lq[k];
                }
                if constexpr (WANT_V) {
#pragma unroll
                    for (int k = 0; k < n; k++) {
                        lp[k] = V(k, p);
                        lq[k] = V(k, q);
                    }
#pragma unroll
                    for (int k = 0; k < n; k++) {
                        V(k, p) = c * lp[k] - s * lq[k];
                        V(k, q) = s * lp[k] + c * lq[k];
                    }
                }
            }
    }
#pragma unroll
    for (int i = 0; i < n; i++) ev[i] = A(i, i);
}

__device__ inline double det3(const double* F)
{
    return F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) +
           F[2] * (F[3] * F[7] - F[4] * F[6]);
}

// ROI geometry in units of Z*: r = ((c - x*)/Z*, 1) and p = (c - x* + q)/Z*.
struct RoiSet {
    const float* q;      // [n][2] shifts
    const double* cx;    // centres, element i at cx[i * cs]
    const double* cy;
    int cs;
    int n;
    double xs, ys, iz;
    __device__ void get(int i, double& r0, double& r1, double& p0, double& p1) const
    {
        const double ax = cx[i * cs] - xs, ay = cy[i * cs] - ys;
        r0 = ax * iz;
        r1 = ay * iz;
        p0 = (ax + (double)q[2 * i]) * iz;
        p1 = (ay + (double)q[2 * i + 1]) * iz;
    }
};

// Normal-equation terms of Eq. (3) at f (F33 = 1) for the ROI set.
__device__ void gn_terms(const double* f, const RoiSet& rs, double (&JtJ)[8][8], double (&Jte)[8])
{
    const int n = rs.n;
#pragma unroll
    for (int a = 0; a < 8; a++) {
        Jte[a] = 0.0;
#pragma unroll
        for (int b = 0; b < 8; b++) JtJ[a][b] = 0.0;
    }
    for (int i = 0; i < n; i++) {
        double r0, r1, pxi, pyi;
        rs.get(i, r0, r1, pxi, pyi);
        const double n1 = f[0] * r0 + f[1] * r1 + f[2];
        const double n2 = f[3] * r0 + f[4] * r1 + f[5];
        const double d = f[6] * r0 + f[7] * r1 + f[8];
        const double id = 1.0 / d;
        const double u = n1 * id, v = n2 * id;
        const double ex = u - pxi, ey = v - pyi;
        // d(u)/d theta and d(v)/d theta, theta = (F11..F23, F31, F32)
        double ju[8] = {r0 * id, r1 * id, id, 0.0, 0.0, 0.0, -u * r0 * id, -u * r1 * id};
        double jv[8] = {0.0, 0.0, 0.0, r0 * id, r1 * id, id, -v * r0 * id, -v * r1 * id};
#pragma unroll
        for (int a = 0; a < 8; a++) {
            Jte[a] += ju[a] * ex + jv[a] * ey;
#pragma unroll
            for (int b = a; b < 8; b++) JtJ[a][b] += ju[a] * ju[b] + jv[a] * jv[b];
        }
    }
#pragma unroll
    for (int a = 0; a < 8; a++)
#pragma unroll
        for (int b = 0; b < a; b++) JtJ[a][b] = JtJ[b][a];
}

// Cholesky solve of the SPD system M x = rhs; false if M is not positive definite.
__device__ bool cholesky_solve8(double (&M)[8][8], const double (&rhs)[8], double (&x)[8])
{
    double Lm[8][8];
#pragma unroll
    for (int i = 0; i < 8; i++)
#pragma unroll
        for (int j = 0; j <= i; j++) {
            double s = M[i][j];
#pragma unroll
            for (int k = 0; k < j; k++) s -= Lm[i][k] * Lm[j][k];
            if (i == j) {
                if (!(s > 0.0)) return false;
                Lm[i][i] = sqrt(s);
            } else {
                Lm[i][j] = s / Lm[j][j];
            }
        }
    double y[8];
#pragma unroll
    for (int i = 0; i < 8; i++) {
        double s = rhs[i];
#pragma unroll
        for (int k = 0; k < i; k++) s -= Lm[i][k] * y[k];
        y[i] = s / Lm[i][i];
    }
#pragma unroll
    for (int i = 7; i >= 0; i--) {
        double s = y[i];
#pragma unroll
        for (int k = i + 1; k < 8; k++) s -= Lm[k][i] * x[k];
        x[i] = s / Lm[i][i];
    }
    return true;
}

// Eq. (3) for one shift set.  Writes det-1 F (row-major), returns status bits.
// pool: this thread's kSolvePool LDS words (stride kSolveThreads).
__device__ uint32_t solve_F(const RoiSet& rs, double* F, double* pool)
{
    const int n = rs.n;
    uint32_t st = 0;
    // Linear start: Eq. (2) multiplied through by its denominator is linear in F, and with
    // F33 = 1 (the normalisation the Gauss-Newton iteration keeps) in the 8 other entries; their
    // least-squares solution (8 x 8 normal equations, Cholesky) starts the iteration, which
    // converges to the same minimiser as from the unit-norm null vector of the 9-column system
    // and takes none of its eigen-decomposition.  A singular system flags the pair and starts
    // from the identity.
    double f[9] = {1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0};
    {
        double A[8][8], rhs[8], sol[8];
#pragma unroll
        for (int a = 0; a < 8; a++) {
            rhs[a] = 0.0;
#pragma unroll
            for (int c = 0; c < 8; c++) A[a][c] = 0.0;
        }
        for (int i = 0; i < n; i++) {
            double rx, ry, px, py;
            rs.get(i, rx, ry, px, py);
            const double ra[8] = {rx, ry, 1.0, 0.0, 0.0, 0.0, -px * rx, -px * ry};
            const double rb[8] = {0.0, 0.0, 0.0, rx, ry, 1.0, -py * rx, -py * ry};
#pragma unroll
            for (int a = 0; a < 8; a++) {
                rhs[a] += ra[a] * px + rb[a] * py;
#pragma unroll
                for (int c = a; c < 8; c++) A[a][c] += ra[a] * ra[c] + rb[a] * rb[c];
            }
        }
#pragma unroll
        for (int a = 0; a < 8; a++)
#pragma unroll
            for (int c = 0; c < a; c++) A[a][c] = A[c][a];
        if (cholesky_solve8(A, rhs, sol)) {
#pragma unroll
            for (int a = 0; a < 8; a++) f[a] = sol[a];
        } else {
            st |= EBSD_SOLVE_ILLCOND;
        }
    }

    double JtJ[8][8], Jte[8];
    for (int it = 0; it < 100; it++) {
        gn_terms(f, rs, JtJ, Jte);
        double rhs[8], dlt[8];
        for (int a = 0; a < 8; a++) rhs[a] = -Jte[a];
        if (!cholesky_solve8(JtJ, rhs, dlt)) {
            st |= EBSD_SOLVE_ILLCOND;
            break;
        }
        double nrm = 0.0;
        for (int a = 0; a < 8; a++) {
            f[a] += dlt[a];
            nrm += dlt[a] * dlt[a];
        }
        if (!isfinite(nrm)) {
            st |= EBSD_SOLVE_ILLCOND;
            break;
        }
        if (sqrt(nrm) < 1e-14) break;
    }
    gn_terms(f, rs, JtJ, Jte);
    double e8[8];
    {
        const LMat<8> A8{pool}, V8{pool + 64 * kSolveThreads};
#pragma unroll
        for (int a = 0; a < 8; a++)
#pragma unroll
            for (int b = 0; b < 8; b++) A8(a, b) = JtJ[a][b];
        jacobi_eigen_l<8, false>(A8, e8, V8);  // eigenvalues only: the conditioning
    }
    double lo = e8[0], hi = e8[0];
    for (int a = 1; a < 8; a++) {
        lo = fmin(lo, e8[a]);
        hi = fmax(hi, e8[a]);
    }
    if (!(lo > 0.0) || hi > 1e12 * lo) st |= EBSD_SOLVE_ILLCOND;
    const double d = det3(f);
    if (d > 0.0) {
        const double s = cbrt(d);
        for (int i = 0; i < 9; i++) f[i] /= s;
    } else {
        st |= EBSD_SOLVE_ILLCOND;
    }
    for (int i = 0; i < 9; i++) F[i] = f[i];
    return st;
}

// ---- Eq. (3) with one wavefront per pair -----------------------------------------
//
// The solve above with its sums over the ROIs spread over the lanes of one
// wavefront (a workgroup of 64 threads per pair).  Lane t < 36 accumulates the
// upper-triangle element (a, c) of the 8 x 8 normal matrix and lane 36 + a the
// right-hand side's element a, each over the ROIs in order and with its products
// grouped as in solve_F, so that every element, and hence F, the status and the
// conditioning, is the same bit for bit.  The 8 x 8 Cholesky solves then run on
// every lane alike (uniform values in registers), and each Jacobi rotation of the
// conditioning check updates its row and column elements on lanes 0..7.  The
// workgroup is one wavefront, so __syncthreads orders the lanes' LDS accesses
// without coupling pairs; every loop bound and branch outside the per-lane
// element work is uniform (computed alike from the same LDS values).
constexpr int kWaveSolveMaxRoi = 256;  // the largest ROI count the entry points accept

struct WaveSolveLds {
    double roi[4][kWaveSolveMaxRoi];  // r0, r1, p0, p1 of each ROI (units of Z*)
    double M[8][8];                   // normal matrix (symmetric)
    double rhs[8];
    double term[kWaveSolveMaxRoi];    // per-ROI terms of the mean angular error
};

// 0 -> x, 1 -> y, 2 -> 1
__device__ inline double sel3(int k, double x, double y) { return k == 0 ? x : (k == 1 ? y : 1.0); }

// Lane t's task: (a, c), a <= c, of the matrix for t < 36 (row-major upper
// triangle), row a of the right-hand side for 36 <= t < 44; idle above.
__device__ inline void wave_task(int t, int& a, int& c)
{
    if (t >= 36) {
        a = t - 36;
        c = -1;
        return;
    }
    a = 0;
    int rem = t;
    while (rem >= 8 - a) {
        rem -= 8 - a;
        a++;
    }
    c = a + rem;
}

// Fill the ROI table (lanes over ROIs).
__device__ void wave_rois(const RoiSet& rs, WaveSolveLds& L)
{
    for (int i = threadIdx.x; i < rs.n; i += 64) {
        double r0, r1, p0, p1;
        rs.get(i, r0, r1, p0, p1);
        L.roi[0][i] = r0;
        L.roi[1][i] = r1;
        L.roi[2][i] = p0;
        L.roi[3][i] = p1;
    }
    __syncthreads();
}

// Store lane results (matrix element or right-hand side element), then every
// lane reads the whole system into registers.
__device__ void wave_gather(double acc, int ta, int tc, WaveSolveLds& L, double (&A)[8][8], double (&r)[8])
{
    if (threadIdx.x < 36) {
        L.M[ta][tc] = acc;
        L.M[tc][ta] = acc;
    } else if (threadIdx.x < 44) {
        L.rhs[ta] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 8; a++) {
        r[a] = L.rhs[a];
#pragma unroll
        for (int c = 0; c < 8; c++) A[a][c] = L.M[a][c];
    }
    __syncthreads();
}

// gn_terms on the lanes: the lane's element of J^T J (tc >= 0) or of J^T e (tc < 0).
__device__ double gn_term_lane(const double (&f)[9], int n, const WaveSolveLds& L, int ta, int tc)
{
    double acc = 0.0;
    for (int i = 0; i < n; i++) {
        const double r0 = L.roi[0][i], r1 = L.roi[1][i], pxi = L.roi[2][i], pyi = L.roi[3][i];
        const double n1 = f[0] * r0 + f[1] * r1 + f[2];
        const double n2 = f[3] * r0 + f[4] * r1 + f[5];
        const double d = f[6] * r0 + f[7] * r1 + f[8];
        const double id = 1.0 / d;
        const double u = n1 * id, v = n2 * id;
        const double ex = u - pxi, ey = v - pyi;
        // d(u)/d theta_k and d(v)/d theta_k as in gn_terms
        auto ju = [&](int k) {
            return k < 3 ? sel3(k, r0, r1) * id : (k < 6 ? 0.0 : (-u * sel3(k - 6, r0, r1)) * id);
        };
        auto jv = [&](int k) {
            return k < 3 ? 0.0 : (k < 6 ? sel3(k - 3, r0, r1) * id : (-v * sel3(k - 6, r0, r1)) * id);
        };
        const double ua = ju(ta), va = jv(ta);
        const double ub = tc < 0 ? ex : ju(tc), vb = tc < 0 ? ey : jv(tc);
        acc += ua * ub + va * vb;
    }
    return acc;
}

// Eigenvalues of the symmetric 8 x 8 matrix in L.M (destroyed): jacobi_eigen_l's
// rotations and convergence test in the same order, the element updates of a
// rotation on lanes 0..7.
__device__ void wave_jacobi8(WaveSolveLds& L, double (&ev)[8])
{
    const int k = threadIdx.x;
    for (int sweep = 0; sweep < 60; sweep++) {
        double off = 0.0, diag = 0.0;
#pragma unroll
        for (int i = 0; i < 8; i++) {
            diag += L.M[i][i] * L.M[i][i];
#pragma unroll
            for (int j = i + 1; j < 8; j++) off += 2.0 * L.M[i][j] * L.M[i][j];
        }
        if (off == 0.0 || off <= 1e-30 * (off + diag)) break;
        for (int p = 0; p < 7; p++)
            for (int q = p + 1; q < 8; q++) {
                const double apq = L.M[p][q];
                if (apq == 0.0) continue;
                const double tau = (L.M[q][q] - L.M[p][p]) / (2.0 * apq);
                const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                const double c = rsqrt(1.0 + t * t), s = t * c;
                __syncthreads();  // every lane has read the rotation's inputs
                if (k < 8) {
                    const double lp = L.M[k][p], lq = L.M[k][q];
                    L.M[k][p] = c * lp - s * lq;
                    L.M[k][q] = s * lp + c * lq;
                }
                __syncthreads();
                if (k < 8) {
                    const double lp = L.M[p][k], lq = L.M[q][k];
                    L.M[p][k] = c * lp - s * lq;
                    L.M[q][k] = s * lp + c * lq;
                }
                __syncthreads();
            }
    }
#pragma unroll
    for (int i = 0; i < 8; i++) ev[i] = L.M[i][i];
    __syncthreads();
}

// solve_F on one wavefront (see above); every lane returns the same F and status.
__device__ uint32_t solve_F_wave(const RoiSet& rs, double* F, WaveSolveLds& L)
{
    const int n = rs.n;
    uint32_t st = 0;
    int ta, tc;
    wave_task(threadIdx.x < 44 ? threadIdx.x : 0, ta, tc);
    wave_rois(rs, L);
    // linear start (see solve_F)
    double f[9] = {1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0};
    {
        double acc = 0.0;
        for (int i = 0; i < n; i++) {
            const double rx = L.roi[0][i], ry = L.roi[1][i], px = L.roi[2][i], py = L.roi[3][i];
            auto ra = [&](int k) { return k < 3 ? sel3(k, rx, ry) : (k < 6 ? 0.0 : -px * sel3(k - 6, rx, ry)); };
            auto rb = [&](int k) { return k < 3 ? 0.0 : (k < 6 ? sel3(k - 3, rx, ry) : -py * sel3(k - 6, rx, ry)); };
            const double ua = ra(ta), va = rb(ta);
            const double ub = tc < 0 ? px : ra(tc), vb = tc < 0 ? py : rb(tc);
            acc += ua * ub + va * vb;
        }
        double A[8][8], rhs[8], sol[8];
        wave_gather(acc, ta, tc, L, A, rhs);
        if (cholesky_solve8(A, rhs, sol)) {
#pragma unroll
            for (int a = 0; a < 8; a++) f[a] = sol[a];
        } else {
            st |= EBSD_SOLVE_ILLCOND;
        }
    }
    double JtJ[8][8], Jte[8];
    for (int it = 0; it < 100; it++) {
        wave_gather(gn_term_lane(f, n, L, ta, tc), ta, tc, L, JtJ, Jte);
        double rhs[8], dlt[8];
        for (int a = 0; a < 8; a++) rhs[a] = -Jte[a];
        if (!cholesky_solve8(JtJ, rhs, dlt)) {
            st |= EBSD_SOLVE_ILLCOND;
            break;
        }
        double nrm = 0.0;
        for (int a = 0; a < 8; a++) {
            f[a] += dlt[a];
            nrm += dlt[a] * dlt[a];
        }
        if (!isfinite(nrm)) {
            st |= EBSD_SOLVE_ILLCOND;
            break;
        }
        if (sqrt(nrm) < 1e-14) break;
    }
    {
        const double acc = gn_term_lane(f, n, L, ta, tc);
        if (threadIdx.x < 36) {
            L.M[ta][tc] = acc;
            L.M[tc][ta] = acc;
        }
        __syncthreads();
    }
    double e8[8];
    wave_jacobi8(L, e8);  // eigenvalues only: the conditioning
    double lo = e8[0], hi = e8[0];
    for (int a = 1; a < 8; a++) {
        lo = fmin(lo, e8[a]);
        hi = fmax(hi, e8[a]);
    }
    if (!(lo > 0.0) || hi > 1e12 * lo) st |= EBSD_SOLVE_ILLCOND;
    const double d = det3(f);
    if (d > 0.0) {
        const double s = cbrt(d);
        for (int i = 0; i < 9; i++) f[i] /= s;
    } else {
        st |= EBSD_SOLVE_ILLCOND;
    }
    for (int i = 0; i < 9; i++) F[i] = f[i];
    return st;
}

// R = F (F^T F)^(-1/2): the rotation of the polar decomposition.
__device__ void polar_rot(const double* F, double* R)
{
    double C[3][3];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            C[i][j] = F[i] * F[j] + F[3 + i] * F[3 + j] + F[6 + i] * F[6 + j];
    double ev[3], Q[3][3];
    jacobi_eigen<3>(C, ev, Q);
    double Ui[3][3];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0.0;
            for (int k = 0; k < 3; k++) s += Q[i][k] * Q[j][k] / sqrt(ev[k]);
            Ui[i][j] = s;
        }
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            R[3 * i + j] = F[3 * i] * Ui[0][j] + F[3 * i + 1] * Ui[1][j] + F[3 * i + 2] * Ui[2][j];
}

__device__ void rotation_vector(const double* R, double* rv)
{
    const double w0 = 0.5 * (R[7] - R[5]), w1 = 0.5 * (R[2] - R[6]), w2 = 0.5 * (R[3] - R[1]);
    const double s = sqrt(w0 * w0 + w1 * w1 + w2 * w2);
    const double c = 0.5 * (R[0] + R[4] + R[8] - 1.0);
    if (s == 0.0) {
        rv[0] = rv[1] = rv[2] = 0.0;
        return;
    }
    const double th = atan2(s, c) / s;
    rv[0] = th * w0;
    rv[1] = th * w1;
    rv[2] = th * w2;
}

// Mean angular error of the fit F to the shifts of rs (the figure section 3
// compares remapping methods by; its formula is not given, this reading is
// used): the mean over the ROIs of the angle between F r_i and r_i + q_i,
// atan2(|a x b|, a . b).  Both vectors are in units of Z*, which leaves the
// angles unchanged.  The angles on the lanes of the pair's wavefront, their sum
// in ROI order.
__device__ double mean_angular_error_wave(const RoiSet& rs, const double* F, WaveSolveLds& L)
{
    for (int i = threadIdx.x; i < rs.n; i += 64) {
        double r0, r1, p0, p1;
        rs.get(i, r0, r1, p0, p1);
        const double a0 = F[0] * r0 + F[1] * r1 + F[2];
        const double a1 = F[3] * r0 + F[4] * r1 + F[5];
        const double a2 = F[6] * r0 + F[7] * r1 + F[8];
        // b = (p0, p1, 1)
        const double c0 = a1 - a2 * p1, c1 = a2 * p0 - a0, c2 = a0 * p1 - a1 * p0;
        L.term[i] = atan2(sqrt(c0 * c0 + c1 * c1 + c2 * c2), a0 * p0 + a1 * p1 + a2);
    }
    __syncthreads();
    double sum = 0.0;
    for (int i = 0; i < rs.n; i++) sum += L.term[i];
    __syncthreads();
    return rs.n > 0 ? sum / rs.n : 0.0;
}

__device__ RoiSet bucket_rois(const Bucket* bk, const float* q)
{
    RoiSet rs;
    rs.q = q;
    rs.cx = bk->roi_c;
    rs.cy = bk->roi_c + 1;
    rs.cs = 2;
    rs.n = bk->n_roi;
    rs.xs = bk->xs;
    rs.ys = bk->ys;
    rs.iz = 1.0 / bk->zs;
    return rs;
}

// One wavefront per pair (workgroup b).
__global__ void __launch_bounds__(64) k_solve_first(const Bucket* __restrict__ bk, float tol)
{
    __shared__ WaveSolveLds L;
    const int b = blockIdx.x;
    if (b >= bk->nb) return;  // uniform
    uint32_t st = bk->test_stat[b].flags | bk->ref_stat[bk->ref_slot[b]].flags;
    if (bk->warm_flag) st |= bk->warm_flag[b];
    if (tol > 0.0f) {
        const uint32_t all = (bk->L >= 32) ? 0xffffffffu : ((1u << bk->L) - 1u);
        if ((bk->state[b].convmask & all) == all) st |= EBSD_CONVERGED;
        else st |= EBSD_HIT_CAP;
    }
    const RoiSet rs = bucket_rois(bk, bk->q1 + 2 * (int64_t)b * bk->n_roi);
    double F1[9], R[9];
    st |= solve_F_wave(rs, F1, L);
    const double mae = mean_angular_error_wave(rs, F1, L);
    polar_rot(F1, R);
    if (threadIdx.x == 0) {
        for (int i = 0; i < 9; i++) {
            bk->F1[9 * (int64_t)b + i] = F1[i];
            bk->Rfin[9 * (int64_t)b + i] = R[i];
        }
        bk->mae1[b] = mae;
        bk->status[b] = st;
    }
}

// Status for the second-pass-only entry: input flags only.
__global__ void k_status_inputs(const Bucket* __restrict__ bk)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= bk->nb) return;
    bk->status[b] = bk->test_stat[b].flags | bk->ref_stat[bk->ref_slot[b]].flags;
}

// pass 0 composes with R_finite (Eq. (12)); pass k > 0 with the F the
// previous pass left in F (read before F is overwritten).  One wavefront per
// pair (workgroup b); lane 0 writes the results.
__global__ void __launch_bounds__(64) k_solve_second(const Bucket* __restrict__ bk, int second_pass, int pass)
{
    __shared__ WaveSolveLds L;
    const int b = blockIdx.x;
    if (b >= bk->nb) return;  // uniform
    double Rf[9];
    const double* Rsrc = (pass == 0 ? bk->Rfin : bk->F) + 9 * (int64_t)b;
    for (int i = 0; i < 9; i++) Rf[i] = Rsrc[i];
    double F[9];
    uint32_t st = bk->status[b];
    double mae;
    __syncthreads();  // every lane has read F before lane 0 overwrites it
    if (second_pass) {
        double Fi[9];
        const RoiSet rs = bucket_rois(bk, bk->q2 + 2 * (int64_t)b * bk->n_roi);
        st |= solve_F_wave(rs, Fi, L);
        mae = mean_angular_error_wave(rs, Fi, L);
        double Ft[9];
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++)
                Ft[3 * i + j] = Fi[3 * i] * Rf[j] + Fi[3 * i + 1] * Rf[3 + j] + Fi[3 * i + 2] * Rf[6 + j];
        const double d = det3(Ft);
        if (d > 0.0) {
            const double s = cbrt(d);
            for (int i = 0; i < 9; i++) Ft[i] /= s;
        }
        for (int i = 0; i < 9; i++) F[i] = Ft[i];
    } else {
        const double* F1 = bk->F1 + 9 * (int64_t)b;
        for (int i = 0; i < 9; i++) F[i] = F1[i];
        mae = bk->mae1[b];
    }
    double R[9], rv[3];
    polar_rot(F, R);
    rotation_vector(R, rv);
    if (threadIdx.x == 0) {
        for (int i = 0; i < 9; i++) {
            bk->F[9 * (int64_t)b + i] = F[i];
            bk->R[9 * (int64_t)b + i] = R[i];
        }
        for (int i = 0; i < 3; i++) bk->rotvec[3 * (int64_t)b + i] = rv[i];
        bk->mae[b] = mae;
        bk->status[b] = st;
    }
}

// One wavefront per shift set (workgroup b).
__global__ void __launch_bounds__(64) k_stage_solve(const float* __restrict__ q, int n, int n_roi,
                              const double* __restrict__ cx, const double* __restrict__ cy,
                              double xs, double ys, double zs, double* __restrict__ F,
                              double* __restrict__ R, uint32_t* __restrict__ status)
{
    __shared__ WaveSolveLds L;
    const int b = blockIdx.x;
    if (b >= n) return;  // uniform
    RoiSet rs;
    rs.q = q + 2 * (int64_t)b * n_roi;
    rs.cx = cx;
    rs.cy = cy;
    rs.cs = 1;
    rs.n = n_roi;
    rs.xs = xs;
    rs.ys = ys;
    rs.iz = 1.0 / zs;
    double Fb[9], Rb[9];
    const uint32_t st = solve_F_wave(rs, Fb, L);
    polar_rot(Fb, Rb);
    if (threadIdx.x == 0) {
        for (int i = 0; i < 9; i++) {
            F[9 * (int64_t)b + i] = Fb[i];
            if (R) R[9 * (int64_t)b + i] = Rb[i];
        }
        if (status) status[b] = st;
    }
}

// ---- traction-free constraint, strain and stress ----------------------------------

// sigma_S of a sample-frame strain e: the strain in crystal coordinates
// g e g^T (g: passive, sample -> crystal), the cubic Hooke law in Voigt form
// (c11 normal, c12 between normals, c44 on the engineering shears), the
// stress back in sample coordinates, g^T sigma_C g.
__device__ void hooke_sample(const double* e, const double* g, const TractionFrame& tf, double* sig)
{
    double t[9], ec[9], sc[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) t[3 * i + j] = g[3 * i] * e[j] + g[3 * i + 1] * e[3 + j] + g[3 * i + 2] * e[6 + j];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) ec[3 * i + j] = t[3 * i] * g[3 * j] + t[3 * i + 1] * g[3 * j + 1] + t[3 * i + 2] * g[3 * j + 2];
    const double tr = ec[0] + ec[4] + ec[8];
    const double dc = tf.c11 - tf.c12;
    sc[0] = dc * ec[0] + tf.c12 * tr;
    sc[4] = dc * ec[4] + tf.c12 * tr;
    sc[8] = dc * ec[8] + tf.c12 * tr;
    sc[1] = sc[3] = tf.c44 * (ec[1] + ec[3]);
    sc[2] = sc[6] = tf.c44 * (ec[2] + ec[6]);
    sc[5] = sc[7] = tf.c44 * (ec[5] + ec[7]);
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) t[3 * i + j] = sc[3 * i] * g[j] + sc[3 * i + 1] * g[3 + j] + sc[3 * i + 2] * g[6 + j];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) sig[3 * i + j] = g[i] * t[j] + g[3 + i] * t[3 + j] + g[6 + i] * t[6 + j];
}

// F_S = S F S^T (Eq. (14)) and B = F_S F_S^T.
__device__ void sample_frame(const double* F, const double* S, double* FS, double* B)
{
    double t[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) t[3 * i + j] = S[3 * i] * F[j] + S[3 * i + 1] * F[3 + j] + S[3 * i + 2] * F[6 + j];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) FS[3 * i + j] = t[3 * i] * S[3 * j] + t[3 * i + 1] * S[3 * j + 1] + t[3 * i + 2] * S[3 * j + 2];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            B[3 * i + j] = FS[3 * i] * FS[3 * j] + FS[3 * i + 1] * FS[3 * j + 1] + FS[3 * i + 2] * FS[3 * j + 2];
}

// Eq. (3) under the traction-free constraint for one shift set (section 2,
// Eq. (16), supplementary Part 2): minimise Eq. (3) over X = F_inf subject to
// sigma_S33 = sigma_S23 = sigma_S13 = 0 for the total F = X M, with
// eps_S = (F_S F_S^T - I) / 2 (Eq. (15)).  Start: the det-1 solution scaled so
// that sigma_S33 = 0 (sigma is (s^2 sigma[B] - sigma[I]) / 2 at scale s); then
// Lagrange-Newton steps [J^T J  A^T; A  0] [d; l] = [-J^T e; -c] over the nine
// entries (e in units of Z*, c the three stresses over c11), the augmented
// 12 x 13 system in this thread's LDS pool.  Writes F, eps_S, sigma_S.
__device__ uint32_t solve_F_traction_free(const RoiSet& rs, const double* M, const double* g,
                                          const TractionFrame& tf, double* F, double* eps, double* sig,
                                          double* pool)
{
    double X[9];
    uint32_t st = solve_F(rs, X, pool);
    const double* S = tf.S;
    double MSt[9];  // M S^T
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) MSt[3 * i + j] = M[3 * i] * S[3 * j] + M[3 * i + 1] * S[3 * j + 1] + M[3 * i + 2] * S[3 * j + 2];
    const double I3[9] = {1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0};
    {
        double Ft[9], FS[9], B[9], sB[9], sI[9];
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) Ft[3 * i + j] = X[3 * i] * M[j] + X[3 * i + 1] * M[3 + j] + X[3 * i + 2] * M[6 + j];
        sample_frame(Ft, S, FS, B);
        hooke_sample(B, g, tf, sB);
        hooke_sample(I3, g, tf, sI);
        double s2 = sI[8] / sB[8];
        if (!(s2 > 0.0) || !isfinite(s2)) {
            st |= EBSD_SOLVE_ILLCOND;
            s2 = 1.0;
        }
        const double sc = sqrt(s2);
        for (int i = 0; i < 9; i++) X[i] *= sc;
    }
    const LMat<13> K{pool};
    bool done = false;
    for (int it = 0; it < 100 && !done; it++) {
        for (int a = 0; a < 12; a++)
            for (int b = 0; b < 13; b++) K(a, b) = 0.0;
        for (int i = 0; i < rs.n; i++) {
            double r0, r1, p0, p1;
            rs.get(i, r0, r1, p0, p1);
            const double n1 = X[0] * r0 + X[1] * r1 + X[2];
            const double n2 = X[3] * r0 + X[4] * r1 + X[5];
            const double id = 1.0 / (X[6] * r0 + X[7] * r1 + X[8]);
            const double u = n1 * id, v = n2 * id;
            const double ex = u - p0, ey = v - p1;
            const double ju[9] = {r0 * id, r1 * id, id, 0.0, 0.0, 0.0, -u * r0 * id, -u * r1 * id, -u * id};
            const double jv[9] = {0.0, 0.0, 0.0, r0 * id, r1 * id, id, -v * r0 * id, -v * r1 * id, -v * id};
            for (int a = 0; a < 9; a++) {
                K(a, 12) -= ju[a] * ex + jv[a] * ey;
                for (int b = a; b < 9; b++) K(a, b) += ju[a] * ju[b] + jv[a] * jv[b];
            }
        }
        for (int a = 1; a < 9; a++)
            for (int b = 0; b < a; b++) K(a, b) = K(b, a);
        // constraints and their derivatives
        double Ft[9], FS[9], B[9], sg[9];
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) Ft[3 * i + j] = X[3 * i] * M[j] + X[3 * i + 1] * M[3 + j] + X[3 * i + 2] * M[6 + j];
        sample_frame(Ft, S, FS, B);
        for (int i = 0; i < 9; i++) B[i] = 0.5 * (B[i] - I3[i]);
        hooke_sample(B, g, tf, sg);
        const double ic = 1.0 / tf.c11;
        K(9, 12) = -sg[8] * ic;
        K(10, 12) = -sg[5] * ic;
        K(11, 12) = -sg[2] * ic;
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                // dF_S for a unit change of X_ab: column a of S times row b of M S^T
                double de[9], ds[9];
                for (int i = 0; i < 3; i++)
                    for (int j = 0; j < 3; j++) {
                        const double d1 = S[3 * i + a] * (MSt[3 * b] * FS[3 * j] + MSt[3 * b + 1] * FS[3 * j + 1] + MSt[3 * b + 2] * FS[3 * j + 2]);
                        const double d2 = S[3 * j + a] * (FS[3 * i] * MSt[3 * b] + FS[3 * i + 1] * MSt[3 * b + 1] + FS[3 * i + 2] * MSt[3 * b + 2]);
                        de[3 * i + j] = 0.5 * (d1 + d2);
                    }
                hooke_sample(de, g, tf, ds);
                const int c = 3 * a + b;
                K(9, c) = K(c, 9) = ds[8] * ic;
                K(10, c) = K(c, 10) = ds[5] * ic;
                K(11, c) = K(c, 11) = ds[2] * ic;
            }
        // Gaussian elimination with partial pivoting on the augmented system
        bool ok = true;
        for (int k = 0; k < 12 && ok; k++) {
            int piv = k;
            for (int i = k + 1; i < 12; i++)
                if (fabs(K(i, k)) > fabs(K(piv, k))) piv = i;
            if (K(piv, k) == 0.0) {
                ok = false;
                break;
            }
            if (piv != k)
                for (int j = k; j < 13; j++) {
                    const double t = K(k, j);
                    K(k, j) = K(piv, j);
                    K(piv, j) = t;
                }
            const double ip = 1.0 / K(k, k);
            for (int i = k + 1; i < 12; i++) {
                const double m = K(i, k) * ip;
                if (m != 0.0)
                    for (int j = k; j < 13; j++) K(i, j) -= m * K(k, j);
            }
        }
        if (!ok) {
            st |= EBSD_SOLVE_ILLCOND;
            break;
        }
        for (int i = 11; i >= 0; i--) {
            double sacc = K(i, 12);
            for (int j = i + 1; j < 12; j++) sacc -= K(i, j) * K(j, 12);
            K(i, 12) = sacc / K(i, i);
        }
        double nrm = 0.0;
        for (int a = 0; a < 9; a++) {
            const double d = K(a, 12);
            X[a] += d;
            nrm += d * d;
        }
        if (!isfinite(nrm)) {
            st |= EBSD_SOLVE_ILLCOND;
            break;
        }
        done = sqrt(nrm) < 1e-14;
    }
    if (!done) st |= EBSD_SOLVE_ILLCOND;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) F[3 * i + j] = X[3 * i] * M[j] + X[3 * i + 1] * M[3 + j] + X[3 * i + 2] * M[6 + j];
    double FS[9], B[9];
    sample_frame(F, S, FS, B);
    for (int i = 0; i < 9; i++) eps[i] = 0.5 * (B[i] - I3[i]);
    hooke_sample(eps, g, tf, sig);
    return st;
}

__global__ void __launch_bounds__(kSolveThreads)
    k_traction_free(const float* __restrict__ q, int n, int n_roi, const double* __restrict__ cx,
                    const double* __restrict__ cy, double xs, double ys, double zs,
                    const double* __restrict__ Mall, const double* __restrict__ gall, TractionFrame tf,
                    double* __restrict__ Fout, double* __restrict__ eout, double* __restrict__ sout,
                    uint32_t* __restrict__ status)
{
    __shared__ double pool[kSolvePool * kSolveThreads];
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    RoiSet rs;
    rs.q = q + 2 * (int64_t)b * n_roi;
    rs.cx = cx;
    rs.cy = cy;
    rs.cs = 1;
    rs.n = n_roi;
    rs.xs = xs;
    rs.ys = ys;
    rs.iz = 1.0 / zs;
    double M[9], g[9], F[9], e[9], sg[9];
    for (int i = 0; i < 9; i++) {
        M[i] = Mall ? Mall[9 * (int64_t)b + i] : (i % 4 == 0 ? 1.0 : 0.0);
        g[i] = gall[9 * (int64_t)b + i];
    }
    const uint32_t st = solve_F_traction_free(rs, M, g, tf, F, e, sg, pool + threadIdx.x);
    for (int i = 0; i < 9; i++) {
        Fout[9 * (int64_t)b + i] = F[i];
        if (eout) eout[9 * (int64_t)b + i] = e[i];
        if (sout) sout[9 * (int64_t)b + i] = sg[i];
    }
    if (status) status[b] = st;
}

__global__ void k_gather_rfin(const Bucket* __restrict__ bk)
{
    const double* __restrict__ rin = bk->rfin_in;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= bk->nb) return;
    const int64_t src = 9 * (int64_t)bk->pair_index[b];
    for (int i = 0; i < 9; i++) bk->Rfin[9 * (int64_t)b + i] = rin[src + i];
}

__global__ void k_scatter(const Bucket* __restrict__ bk)
{
    const OutPtrs o = bk->out;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= bk->nb) return;
    const int64_t g = bk->pair_index[b];
    const int nr = bk->n_roi;
    for (int i = 0; i < 9; i++) {
        if (o.F) o.F[9 * g + i] = bk->F[9 * (int64_t)b + i];
        if (o.R) o.R[9 * g + i] = bk->R[9 * (int64_t)b + i];
        if (o.Rfin) o.Rfin[9 * g + i] = bk->Rfin[9 * (int64_t)b + i];
        if (o.F1) o.F1[9 * g + i] = bk->F1[9 * (int64_t)b + i];
    }
    if (o.rotvec)
        for (int i = 0; i < 3; i++) o.rotvec[3 * g + i] = bk->rotvec[3 * (int64_t)b + i];
    if (o.omega) {
        // Eq. (6): omega_ij = -eps_ijk theta_k
        const double* th = bk->rotvec + 3 * (int64_t)b;
        double* om = o.omega + 9 * g;
        om[0] = 0.0;
        om[1] = -th[2];
        om[2] = th[1];
        om[3] = th[2];
        om[4] = 0.0;
        om[5] = -th[0];
        om[6] = -th[1];
        om[7] = th[0];
        om[8] = 0.0;
    }
    for (int j = 0; j < 2 * nr; j++) {
        if (o.q1) o.q1[2 * nr * g + j] = bk->q1[2 * nr * (int64_t)b + j];
        if (o.q2) o.q2[2 * nr * g + j] = bk->q2[2 * nr * (int64_t)b + j];
    }
    if (o.ph)
        for (int j = 0; j < nr; j++) o.ph[nr * g + j] = bk->ph[nr * (int64_t)b + j];
    if (o.iters)
        for (int l = 0; l < bk->L; l++) o.iters[bk->L * g + l] = bk->iters[bk->L * (int64_t)b + l];
    if (o.status) o.status[g] = bk->status[b];
    if (o.warm_misfit && bk->warm_misfit) o.warm_misfit[g] = bk->warm_misfit[b];
    if (o.mae1) o.mae1[g] = bk->mae1[b];
    if (o.mae) o.mae[g] = bk->mae[b];
    if (o.ssim) o.ssim[g] = bk->ssim ? bk->ssim[b] : __builtin_nan("");
}

// blockIdx.y = pair; the field of one pair is h * w * 2 floats.
__global__ void k_scatter_warm(const Bucket* __restrict__ bk)
{
    const int b = blockIdx.y;
    const int64_t n = 64 * 64 * 2;  // the network's output grid
    const int64_t g = bk->pair_index[b];
    float* dst = bk->out.warm_field + g * n;
    const float* src = bk->warm_field + (int64_t)b * n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}


// ---- warm-start fallback fit ------------------------------------------------------
// One workgroup per pair.  The Eq. (3) model is fitted to the predicted field at
// the coarse grid points (full-resolution coordinates 4 i + 1.5) that lie within
// `radius` of the pattern centre; each thread sums over a strided subset of the
// points and the sums are combined in a fixed order, so the result does not
// depend on scheduling.  All threads then run the same small dense algebra.
constexpr int kFitThreads = 256;

__device__ inline double wave_sum_d(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <int NV>
__device__ void fit_block_sum(double (&v)[NV], double* sh)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; k++) {
        const double w = wave_sum_d(v[k]);
        if (lane == 0) sh[wave * NV + k] = w;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; k++) v[k] = ((sh[k] + sh[NV + k]) + sh[2 * NV + k]) + sh[3 * NV + k];
    __syncthreads();
}

struct GridFit {
    const float* q;  // [gh][gw][2]
    int gh, gw;
    double xs, ys, zs, iz, r2;
    __device__ bool point(int g, double& x, double& y) const
    {
        x = 4.0 * (double)(g % gw) + 1.5;
        y = 4.0 * (double)(g / gw) + 1.5;
        const double dx = x - xs, dy = y - ys;
        return dx * dx + dy * dy <= r2;
    }
};

__global__ void __launch_bounds__(kFitThreads)
k_warm_fit(const float* __restrict__ field, int gh, int gw, double xs, double ys, double zs,
           double radius, double threshold, int model_field, int go, double xsN, double ysN, double zsN,
           float* __restrict__ u_init, float* __restrict__ misfit, uint32_t* __restrict__ flag)
{
    __shared__ double sh[4 * 45];
    const int b = blockIdx.x;
    GridFit gf;
    gf.q = field + (int64_t)b * gh * gw * 2;
    gf.gh = gh;
    gf.gw = gw;
    gf.xs = xs;
    gf.ys = ys;
    gf.zs = zs;
    gf.iz = 1.0 / zs;
    gf.r2 = radius * radius;
    const int ng = gh * gw;

    // Linear start: Eq. (2) multiplied through by its denominator is linear in
    // the 8 entries left free by F33 = 1; its least-squares solution starts the
    // Gauss-Newton iteration (which converges to the same minimiser as from
    // the direct linear start of the ROI solve, with far less work here).
    double f[9] = {1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0};
    double npts;
    {
        double t[45];
#pragma unroll
        for (int k = 0; k < 45; k++) t[k] = 0.0;
        for (int g = threadIdx.x; g < ng; g += kFitThreads) {
            double x, y;
            if (!gf.point(g, x, y)) continue;
            const double ax = x - xs, ay = y - ys;
            const double rx = ax * gf.iz, ry = ay * gf.iz;
            const double px = (ax + (double)gf.q[2 * g]) * gf.iz, py = (ay + (double)gf.q[2 * g + 1]) * gf.iz;
            const double ra[8] = {rx, ry, 1.0, 0.0, 0.0, 0.0, -px * rx, -px * ry};
            const double rb[8] = {0.0, 0.0, 0.0, rx, ry, 1.0, -py * rx, -py * ry};
            int k = 0;
#pragma unroll
            for (int a = 0; a < 8; a++)
#pragma unroll
                for (int c = a; c < 8; c++) t[k++] += ra[a] * ra[c] + rb[a] * rb[c];
#pragma unroll
            for (int a = 0; a < 8; a++) t[36 + a] += ra[a] * px + rb[a] * py;
            t[44] += 1.0;
        }
        fit_block_sum<45>(t, sh);
        npts = t[44];
        double A[8][8], rhs[8], sol[8];
        int k = 0;
        for (int a = 0; a < 8; a++)
            for (int c = a; c < 8; c++) {
                A[a][c] = t[k];
                A[c][a] = t[k];
                k++;
            }
        for (int a = 0; a < 8; a++) rhs[a] = t[36 + a];
        if (cholesky_solve8(A, rhs, sol))
            for (int a = 0; a < 8; a++) f[a] = sol[a];
    }

    // Gauss-Newton on the 8 free entries (|step| < 1e-12 or 100 steps)
    for (int it = 0; it < 100; it++) {
        double t[44];
#pragma unroll
        for (int k = 0; k < 44; k++) t[k] = 0.0;
        for (int g = threadIdx.x; g < ng; g += kFitThreads) {
            double x, y;
            if (!gf.point(g, x, y)) continue;
            const double ax = x - xs, ay = y - ys;
            const double r0 = ax * gf.iz, r1 = ay * gf.iz;
            const double pxi = (ax + (double)gf.q[2 * g]) * gf.iz, pyi = (ay + (double)gf.q[2 * g + 1]) * gf.iz;
            const double n1 = f[0] * r0 + f[1] * r1 + f[2];
            const double n2 = f[3] * r0 + f[4] * r1 + f[5];
            const double d = f[6] * r0 + f[7] * r1 + f[8];
            const double id = 1.0 / d;
            const double u = n1 * id, v = n2 * id;
            const double ex = u - pxi, ey = v - pyi;
            const double ju[8] = {r0 * id, r1 * id, id, 0.0, 0.0, 0.0, -u * r0 * id, -u * r1 * id};
            const double jv[8] = {0.0, 0.0, 0.0, r0 * id, r1 * id, id, -v * r0 * id, -v * r1 * id};
            int k = 0;
#pragma unroll
            for (int a = 0; a < 8; a++)
#pragma unroll
                for (int c = a; c < 8; c++) t[k++] += ju[a] * ju[c] + jv[a] * jv[c];
#pragma unroll
            for (int a = 0; a < 8; a++) t[36 + a] += ju[a] * ex + jv[a] * ey;
        }
        fit_block_sum<44>(t, sh);
        double JtJ[8][8], rhs[8], dlt[8];
        int k = 0;
        for (int a = 0; a < 8; a++)
            for (int c = a; c < 8; c++) {
                JtJ[a][c] = t[k];
                JtJ[c][a] = t[k];
                k++;
            }
        for (int a = 0; a < 8; a++) rhs[a] = -t[36 + a];
        if (!cholesky_solve8(JtJ, rhs, dlt)) break;
        double nrm = 0.0;
        for (int a = 0; a < 8; a++) {
            f[a] += dlt[a];
            nrm += dlt[a] * dlt[a];
        }
        if (!isfinite(nrm) || sqrt(nrm) < 1e-12) break;
    }
    const double dt = det3(f);
    if (dt > 0.0) {
        const double s = cbrt(dt);
        for (int i = 0; i < 9; i++) f[i] /= s;
    }

    // RMS endpoint misfit of the fitted model, full-resolution px
    double ss[1] = {0.0};
    for (int g = threadIdx.x; g < ng; g += kFitThreads) {
        double x, y;
        if (!gf.point(g, x, y)) continue;
        const double rx = x - xs, ry = y - ys;
        const double v0 = f[0] * rx + f[1] * ry + f[2] * zs;
        const double v1 = f[3] * rx + f[4] * ry + f[5] * zs;
        const double v2 = f[6] * rx + f[7] * ry + f[8] * zs;
        const double px = xs + zs * v0 / v2, py = ys + zs * v1 / v2;
        const double dx = px - x - (double)gf.q[2 * g], dy = py - y - (double)gf.q[2 * g + 1];
        ss[0] += dx * dx + dy * dy;
    }
    fit_block_sum<1>(ss, sh);
    const double rms = sqrt(ss[0] / npts);
    // the decision is taken in full-resolution px of the registered pattern:
    // the fit ran in the network's frame (a grid of gw points a side), the
    // pattern's coarse grid has go points a side
    const bool use = rms * (double)go / (double)gw <= threshold;
    if (threadIdx.x == 0) {
        misfit[b] = (float)rms;
        flag[b] = use ? (uint32_t)EBSD_WARM_USED : (uint32_t)EBSD_WARM_FALLBACK;
    }
    // initial field on the coarse grid of the registered pattern (go x go
    // points at 4 i + 1.5 of its own px): the fitted model evaluated there
    // (the projective map is unchanged by a common scaling of the detector
    // coordinates), or the network field resampled from its 64 x 64 grid
    // (same grid: copy; go = 2 gw: prolongation, x 2 in px; go = gw / 2:
    // [1,3,3,1]/8 restriction, x 1/2 in px)
    const int no = go * go;
    float* u = u_init + (int64_t)b * 2 * no;
    for (int g = threadIdx.x; g < no; g += kFitThreads) {
        float ux = 0.0f, uy = 0.0f;
        const int gxo = g % go, gyo = g / go;
        if (use && model_field) {
            const double x = 4.0 * (double)gxo + 1.5, y = 4.0 * (double)gyo + 1.5;
            const double rx = x - xsN, ry = y - ysN;
            const double v0 = f[0] * rx + f[1] * ry + f[2] * zsN;
            const double v1 = f[3] * rx + f[4] * ry + f[5] * zsN;
            const double v2 = f[6] * rx + f[7] * ry + f[8] * zsN;
            ux = (float)(xsN + zsN * v0 / v2 - x);
            uy = (float)(ysN + zsN * v1 / v2 - y);
        } else if (use && go == gw) {
            ux = gf.q[2 * g];
            uy = gf.q[2 * g + 1];
        } else if (use && go == 2 * gw) {
            const float cx = fminf(fmaxf(0.5f * ((float)gxo - 0.5f), 0.0f), (float)(gw - 1));
            const float cy = fminf(fmaxf(0.5f * ((float)gyo - 0.5f), 0.0f), (float)(gh - 1));
            const int x0 = (int)floorf(cx), y0 = (int)floorf(cy);
            const int x1 = min(x0 + 1, gw - 1), y1 = min(y0 + 1, gh - 1);
            const float fx = cx - (float)x0, fy = cy - (float)y0;
            for (int c = 0; c < 2; c++) {
                const float a0 = gf.q[2 * (y0 * gw + x0) + c], a1 = gf.q[2 * (y0 * gw + x1) + c];
                const float b0 = gf.q[2 * (y1 * gw + x0) + c], b1 = gf.q[2 * (y1 * gw + x1) + c];
                const float top = a0 + fx * (a1 - a0), bot = b0 + fx * (b1 - b0);
                const float v = 2.0f * (top + fy * (bot - top));
                if (c == 0) ux = v;
                else uy = v;
            }
        } else if (use && 2 * go == gw) {
            const float wt[4] = {0.125f, 0.375f, 0.375f, 0.125f};
            for (int c = 0; c < 2; c++) {
                float v = 0.0f;
                for (int j = 0; j < 4; j++) {
                    const int yy = min(max(2 * gyo - 1 + j, 0), gh - 1);
                    float rowv = 0.0f;
                    for (int i = 0; i < 4; i++) {
                        const int xx = min(max(2 * gxo - 1 + i, 0), gw - 1);
                        rowv += wt[i] * gf.q[2 * (yy * gw + xx) + c];
                    }
                    v += wt[j] * rowv;
                }
                if (c == 0) ux = 0.5f * v;
                else uy = 0.5f * v;
            }
        }
        u[g] = ux;
        u[no + g] = uy;
    }
}

}  // namespace

hipError_t launch_gather_rfin(const Bucket* d_bk, const Bucket& hb, hipStream_t s)
{
    hipLaunchKernelGGL(k_gather_rfin, dim3((hb.nb + 63) / 64), dim3(64), 0, s, d_bk);
    return hipGetLastError();
}

hipError_t launch_scatter(const Bucket* d_bk, const Bucket& hb, hipStream_t s)
{
    hipLaunchKernelGGL(k_scatter, dim3((hb.nb + 63) / 64), dim3(64), 0, s, d_bk);
    return hipGetLastError();
}

hipError_t launch_scatter_warm(const Bucket* d_bk, const Bucket& hb, hipStream_t s)
{
    const int64_t n = 64 * 64 * 2;
    hipLaunchKernelGGL(k_scatter_warm, dim3((unsigned)((n + 255) / 256), hb.nb), dim3(256), 0, s, d_bk);
    return hipGetLastError();
}

hipError_t launch_solve_first(const Bucket* d_bk, const Bucket& hb, float tol, hipStream_t s)
{
    hipLaunchKernelGGL(k_solve_first, dim3(hb.nb), dim3(64), 0, s, d_bk, tol);
    return hipGetLastError();
}

hipError_t launch_status_inputs(const Bucket* d_bk, const Bucket& hb, hipStream_t s)
{
    hipLaunchKernelGGL(k_status_inputs, dim3((hb.nb + 63) / 64), dim3(64), 0, s, d_bk);
    return hipGetLastError();
}

hipError_t launch_solve_second(const Bucket* d_bk, const Bucket& hb, int second_pass, int pass,
                               hipStream_t s)
{
    hipLaunchKernelGGL(k_solve_second, dim3(hb.nb), dim3(64), 0, s, d_bk, second_pass, pass);
    return hipGetLastError();
}

hipError_t launch_stage_solve(const float* q, int n, int n_roi, const double* cx, const double* cy,
                              double xs, double ys, double zs, double* F, double* R,
                              uint32_t* status, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_stage_solve, dim3(n), dim3(64), 0, s, q, n, n_roi, cx, cy, xs, ys, zs, F, R, status);
    return hipGetLastError();
}

hipError_t launch_traction_free(const float* q, int n, int n_roi, const double* cx, const double* cy,
                                double xs, double ys, double zs, const double* M, const double* g,
                                const TractionFrame& tf, double* F, double* eps, double* sig,
                                uint32_t* status, hipStream_t s)
{
    hipLaunchKernelGGL(k_traction_free, dim3((n + kSolveThreads - 1) / kSolveThreads), dim3(kSolveThreads), 0, s,
                       q, n, n_roi, cx, cy, xs, ys, zs, M, g, tf, F, eps, sig, status);
    return hipGetLastError();
}

hipError_t launch_warm_fit(const float* field, int n, int net_res, double xs, double ys, double zs, double radius,
                           double threshold, int model_field, int N, double xsN, double ysN, double zsN,
                           float* u_init, float* misfit, uint32_t* flag, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int g = net_res / 4, go = N / 4;
    if (!(go == g || go == 2 * g || 2 * go == g)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_warm_fit, dim3(n), dim3(kFitThreads), 0, s, field, g, g, xs, ys, zs, radius, threshold,
                       model_field, go, xsN, ysN, zsN, u_init, misfit, flag);
    return hipGetLastError();
}

}  // namespace ebsd
