// Synthetic Kikuchi-pattern pairs on the GPU: training and benchmark inputs
// with ground-truth labels for the warm-start network and the registration.
//
// A pattern is the gnomonic view of FCC band profiles plus a linear
// background; the test pattern is rendered by pull-back through F^-1, so its
// exact shift field is the projective model of Eq. (2) of arXiv:1907.05993,
// q(x) = pi(F r(x)) - x.  Each pattern is scaled to a mean count and Poisson
// noise is drawn with a counter-based generator (Philox4x32-10, Salmon et al.
// 2011) and the PTRS transformed-rejection sampler (Hormann 1993), so every
// pixel of every pattern is reproducible on its own, independent of the
// launch shape.  Rendering is FP64; outputs are fp32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <set>
#include <tuple>
#include <vector>

#include "../../include/ebsd.h"
#include "ebsd_internal.h"

namespace {

constexpr int kMaxBands = 32;
constexpr int kGenThreads = 256;
constexpr int kGenBlocks = 64;  // blocks per pattern

struct BandTable {
    double n[kMaxBands][3];  // unit plane normals (crystal frame)
    double theta[kMaxBands]; // Bragg half-width (rad)
    double sin_theta[kMaxBands];
    int count;
};

struct GenPair {
    double G[9];     // crystal -> detector
    double Finv[9];  // inverse of the applied deformation gradient
    double F[9];
    double gx, gy, counts;
    uint32_t key0, key1;
    int32_t noise, bands;
};

// ---- Philox4x32-10 ----------------------------------------------------------------
__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
    for (int r = 0; r < 10; r++) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Two doubles in [0, 1) with 53 random bits each from the Philox block of
// counter (pixel, attempt, stream, 0).
__device__ inline void uniforms2(uint32_t p, uint32_t attempt, uint32_t stream, uint32_t k0, uint32_t k1,
                                 double& u, double& v)
{
    uint32_t c[4] = {p, attempt, stream, 0u};
    philox4x32_10(c, k0, k1);
    const double s = 1.0 / 9007199254740992.0;  // 2^-53
    u = (double)(((uint64_t)(c[0] >> 5) << 26) | (uint64_t)(c[1] >> 6)) * s;
    v = (double)(((uint64_t)(c[2] >> 5) << 26) | (uint64_t)(c[3] >> 6)) * s;
}

// Poisson(lam): PTRS for lam >= 10, inversion by sequential search below.
// At most kMaxTries proposals (PTRS accepts more than 90% of them; after the
// cap the rounded mean is returned).
constexpr int kMaxTries = 64;

__device__ double poisson_sample(double lam, uint32_t p, uint32_t stream, uint32_t k0, uint32_t k1)
{
    if (!(lam > 0.0)) return 0.0;
    if (lam < 10.0) {
        double u, v;
        uniforms2(p, 0u, stream, k0, k1, u, v);
        double pk = exp(-lam), cdf = pk;
        int k = 0;
        while (u > cdf && k < 1000) {
            k++;
            pk *= lam / (double)k;
            cdf += pk;
        }
        return (double)k;
    }
    const double slam = sqrt(lam), loglam = log(lam);
    const double b = 0.931 + 2.53 * slam;
    const double a = -0.059 + 0.02483 * b;
    const double invalpha = 1.1239 + 1.1328 / (b - 3.4);
    const double vr = 0.9277 - 3.6224 / (b - 2.0);
    for (int t = 0; t < kMaxTries; t++) {
        double u, v;
        uniforms2(p, (uint32_t)t, stream, k0, k1, u, v);
        u -= 0.5;
        const double us = 0.5 - fabs(u);
        const double k = floor((2.0 * a / us + b) * u + lam + 0.43);
        if (us >= 0.07 && v <= vr) return k;
        if (k < 0.0 || (us < 0.013 && v > us)) continue;
        if (log(v) + log(invalpha) - log(a / (us * us) + b) <= -lam + k * loglam - lgamma(k + 1.0)) return k;
    }
    return floor(lam + 0.5);
}

// ---- rendering ----------------------------------------------------------------------

__device__ double band_sum(const BandTable& bt, const double* G, double dx, double dy, double dz)
{
    const double inv = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
    dx *= inv;
    dy *= inv;
    dz *= inv;
    double acc = 0.0;
    for (int b = 0; b < bt.count; b++) {
        const double nx = G[0] * bt.n[b][0] + G[1] * bt.n[b][1] + G[2] * bt.n[b][2];
        const double ny = G[3] * bt.n[b][0] + G[4] * bt.n[b][1] + G[5] * bt.n[b][2];
        const double nz = G[6] * bt.n[b][0] + G[7] * bt.n[b][1] + G[8] * bt.n[b][2];
        const double s = nx * dx + ny * dy + nz * dz;  // sin of the angle to the plane
        if (fabs(s) <= bt.sin_theta[b]) acc += 0.5 * (1.0 + cos(M_PI * asin(s) / bt.theta[b]));
    }
    return acc;
}

__device__ double intensity(const BandTable& bt, const GenPair& g, int which, int x, int y, int H, int W,
                            double xs, double ys, double zs)
{
    double rx = (double)x - xs, ry = (double)y - ys, rz = zs;
    if (which) {
        const double tx = g.Finv[0] * rx + g.Finv[1] * ry + g.Finv[2] * rz;
        const double ty = g.Finv[3] * rx + g.Finv[4] * ry + g.Finv[5] * rz;
        const double tz = g.Finv[6] * rx + g.Finv[7] * ry + g.Finv[8] * rz;
        rx = tx;
        ry = ty;
        rz = tz;
    }
    const double bg =
        1.0 + 0.2 * (g.gx * ((double)x / (double)(W - 1) - 0.5) + g.gy * ((double)y / (double)(H - 1) - 0.5));
    return g.bands ? bg + 0.5 * band_sum(bt, g.G, rx, ry, rz) : bg;
}

// Pass 1: per-block partial sums of the unscaled intensity (fixed tree order).
// blockIdx.y = 2 * pair + (0 reference, 1 test).
__global__ void __launch_bounds__(kGenThreads)
k_gen_sum(const GenPair* __restrict__ gp, const BandTable* __restrict__ bt_in, int H, int W, double xs, double ys,
          double zs, double* __restrict__ part)
{
    __shared__ BandTable bt;
    __shared__ double sh[kGenThreads];
    if (threadIdx.x == 0) bt = *bt_in;
    __syncthreads();
    const int pat = blockIdx.y;
    const GenPair& g = gp[pat >> 1];
    const int64_t np = (int64_t)H * W;
    double sum = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * kGenThreads + threadIdx.x; p < np; p += (int64_t)kGenBlocks * kGenThreads)
        sum += intensity(bt, g, pat & 1, (int)(p % W), (int)(p / W), H, W, xs, ys, zs);
    sh[threadIdx.x] = sum;
    __syncthreads();
    for (int s = kGenThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)pat * kGenBlocks + blockIdx.x] = sh[0];
}

// Pass 2: scale to the mean count, Poisson noise, fp32 store.
__global__ void __launch_bounds__(kGenThreads)
k_gen_write(const GenPair* __restrict__ gp, const BandTable* __restrict__ bt_in, int H, int W, double xs, double ys,
            double zs, const double* __restrict__ part, float* __restrict__ ref, float* __restrict__ test)
{
    __shared__ BandTable bt;
    if (threadIdx.x == 0) bt = *bt_in;
    __syncthreads();
    const int pat = blockIdx.y;
    const int which = pat & 1;
    const GenPair& g = gp[pat >> 1];
    const int64_t np = (int64_t)H * W;
    double tot = 0.0;
    for (int b = 0; b < kGenBlocks; b++) tot += part[(int64_t)pat * kGenBlocks + b];
    const double scale = g.counts > 0.0 ? g.counts / (tot / (double)np) : 1.0;
    float* dst = (which ? test : ref) + (int64_t)(pat >> 1) * np;
    for (int64_t p = (int64_t)blockIdx.x * kGenThreads + threadIdx.x; p < np; p += (int64_t)kGenBlocks * kGenThreads) {
        double v = intensity(bt, g, which, (int)(p % W), (int)(p / W), H, W, xs, ys, zs) * scale;
        if (g.noise) v = poisson_sample(v, (uint32_t)p, (uint32_t)which, g.key0, g.key1);
        dst[p] = (float)v;
    }
}

// Labels: q = pi(F r(x)) - x at the coarse grid points x = 4 i + 1.5, [H/4][W/4][2].
__global__ void k_gen_labels(const GenPair* __restrict__ gp, int H, int W, double xs, double ys, double zs,
                             float* __restrict__ label)
{
    const int pair = blockIdx.y;
    const int gh = H / 4, gw = W / 4;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= gh * gw) return;
    const GenPair& g = gp[pair];
    const double x = 4.0 * (double)(i % gw) + 1.5, y = 4.0 * (double)(i / gw) + 1.5;
    const double rx = x - xs, ry = y - ys;
    const double v0 = g.F[0] * rx + g.F[1] * ry + g.F[2] * zs;
    const double v1 = g.F[3] * rx + g.F[4] * ry + g.F[5] * zs;
    const double v2 = g.F[6] * rx + g.F[7] * ry + g.F[8] * zs;
    float* out = label + ((int64_t)pair * gh * gw + i) * 2;
    out[0] = (float)(xs + zs * v0 / v2 - x);
    out[1] = (float)(ys + zs * v1 / v2 - y);
}

// The 25 distinct plane normals of the FCC families {111}, {200}, {220},
// {311}; half-width asin((lambda / 2a) |hkl|) with lambda / a = 0.02438
// (20 kV electrons on nickel).
BandTable fcc_bands()
{
    BandTable bt{};
    const int fam[4][3] = {{1, 1, 1}, {2, 0, 0}, {2, 2, 0}, {3, 1, 1}};
    int nb = 0;
    for (auto& f : fam) {
        std::set<std::tuple<int, int, int>> seen;
        int perm[3] = {f[0], f[1], f[2]};
        std::sort(perm, perm + 3);
        do {
            for (int sg = 0; sg < 8; sg++) {
                int v[3];
                for (int j = 0; j < 3; j++) v[j] = (sg >> j & 1) ? -perm[j] : perm[j];
                int first = v[0] != 0 ? v[0] : (v[1] != 0 ? v[1] : v[2]);
                if (first < 0)
                    for (int& c : v) c = -c;
                seen.insert(std::make_tuple(v[0], v[1], v[2]));
            }
        } while (std::next_permutation(perm, perm + 3));
        for (auto& t : seen) {
            const double h = std::get<0>(t), k = std::get<1>(t), l = std::get<2>(t);
            const double gl = std::sqrt(h * h + k * k + l * l);
            bt.n[nb][0] = h / gl;
            bt.n[nb][1] = k / gl;
            bt.n[nb][2] = l / gl;
            bt.theta[nb] = std::asin(0.02438 / 2.0 * gl);
            bt.sin_theta[nb] = std::sin(bt.theta[nb]);
            nb++;
        }
    }
    bt.count = nb;
    return bt;
}

bool inv3(const double* A, double* B)
{
    const double c00 = A[4] * A[8] - A[5] * A[7], c01 = A[5] * A[6] - A[3] * A[8], c02 = A[3] * A[7] - A[4] * A[6];
    const double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
    if (!(std::fabs(det) > 0.0) || !std::isfinite(det)) return false;
    const double id = 1.0 / det;
    B[0] = c00 * id;
    B[1] = (A[2] * A[7] - A[1] * A[8]) * id;
    B[2] = (A[1] * A[5] - A[2] * A[4]) * id;
    B[3] = c01 * id;
    B[4] = (A[0] * A[8] - A[2] * A[6]) * id;
    B[5] = (A[2] * A[3] - A[0] * A[5]) * id;
    B[6] = c02 * id;
    B[7] = (A[1] * A[6] - A[0] * A[7]) * id;
    B[8] = (A[0] * A[4] - A[1] * A[3]) * id;
    return true;
}

struct DevMem {
    void* p = nullptr;
    ~DevMem()
    {
        if (p) (void)hipFree(p);
    }
};

}  // namespace

extern "C" int ebsd_gen_pairs(const ebsd_gen_spec* specs, int32_t n, int32_t H, int32_t W, double pc_x,
                              double pc_y, double pc_z, float* ref, float* test, float* label, void* stream)
{
    if (n < 0 || (n > 0 && (!specs || !ref || !test))) return EBSD_EINVAL;
    if (H < 8 || W < 8 || H > 4096 || W > 4096 || (label && (H % 4 || W % 4))) return EBSD_ESHAPE;
    if (!(pc_z > 0.0) || !std::isfinite(pc_x) || !std::isfinite(pc_y) || !std::isfinite(pc_z)) return EBSD_EINVAL;
    if (n == 0) return EBSD_OK;
    std::vector<GenPair> hp;
    BandTable bt;
    try {
        hp.resize((size_t)n);
        bt = fcc_bands();
    } catch (const std::bad_alloc&) {
        return EBSD_ENOMEM;
    }
    for (int i = 0; i < n; i++) {
        const ebsd_gen_spec& s = specs[i];
        GenPair& g = hp[(size_t)i];
        for (int j = 0; j < 9; j++) {
            if (!std::isfinite(s.G[j]) || !std::isfinite(s.F[j])) return EBSD_EINVAL;
            g.G[j] = s.G[j];
            g.F[j] = s.F[j];
        }
        if (!inv3(g.F, g.Finv)) return EBSD_EINVAL;
        if (!std::isfinite(s.gx) || !std::isfinite(s.gy) || !std::isfinite(s.counts)) return EBSD_EINVAL;
        g.gx = s.gx;
        g.gy = s.gy;
        g.counts = s.counts;
        g.key0 = s.key[0];
        g.key1 = s.key[1];
        g.noise = s.noise != 0;
        g.bands = s.bands != 0;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    ebsd::DeviceWideLock lk(ebsd::capture_mutex());  // the buffers' frees wait for the device
    DevMem dpairs, dbt, dpart;
    if (hipMalloc(&dpairs.p, sizeof(GenPair) * (size_t)n) != hipSuccess ||
        hipMalloc(&dbt.p, sizeof(BandTable)) != hipSuccess ||
        hipMalloc(&dpart.p, sizeof(double) * 2 * (size_t)n * kGenBlocks) != hipSuccess) {
        (void)hipGetLastError();
        return EBSD_ENOMEM;
    }
    if (hipMemcpyAsync(dpairs.p, hp.data(), sizeof(GenPair) * (size_t)n, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(dbt.p, &bt, sizeof(BandTable), hipMemcpyHostToDevice, st) != hipSuccess)
        return EBSD_EDEVICE;
    const double xs = pc_x * W - 0.5, ys = pc_y * H - 0.5, zs = pc_z * W;
    const GenPair* gp = static_cast<const GenPair*>(dpairs.p);
    const BandTable* btp = static_cast<const BandTable*>(dbt.p);
    double* part = static_cast<double*>(dpart.p);
    for (int c0 = 0; c0 < n; c0 += 16384) {  // 2 patterns per pair on grid.y (<= 65535)
        const int cnt = std::min(16384, n - c0);
        const dim3 grid(kGenBlocks, 2 * cnt);
        hipLaunchKernelGGL(k_gen_sum, grid, dim3(kGenThreads), 0, st, gp + c0, btp, H, W, xs, ys, zs,
                           part + (size_t)2 * c0 * kGenBlocks);
        hipLaunchKernelGGL(k_gen_write, grid, dim3(kGenThreads), 0, st, gp + c0, btp, H, W, xs, ys, zs,
                           part + (size_t)2 * c0 * kGenBlocks, ref + (int64_t)c0 * H * W, test + (int64_t)c0 * H * W);
        if (label) {
            const int ng = (H / 4) * (W / 4);
            hipLaunchKernelGGL(k_gen_labels, dim3((ng + 255) / 256, cnt), dim3(256), 0, st, gp + c0, H, W, xs, ys, zs,
                               label + (int64_t)c0 * ng * 2);
        }
    }
    if (hipGetLastError() != hipSuccess) return EBSD_EDEVICE;
    // the temporaries are freed on return: wait for the kernels that read them
    return hipStreamSynchronize(st) == hipSuccess ? EBSD_OK : EBSD_EDEVICE;
}
