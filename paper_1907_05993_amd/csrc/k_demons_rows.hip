// Row-marching demons iteration for gfx950 (multi-resolution demons of
// arXiv:1907.05993 section 1, Eq. (1) force), used for levels up to 256 px wide.
//
// One workgroup of 64 NW threads (NW = 4 wavefronts for 256 px, 2 for 128 px,
// 1 for 64 px) owns a strip of TY output rows of one pair; thread t owns column
// t, so a workgroup spans a whole row and every memory instruction is
// contiguous across the lanes.
// Marching down the strip, for each row y = y0 - r .. y0 + TY - 1 + r:
//   v = u + a grad R / (|grad R|^2 + a^2),  a = R - T(x + u)  (bilinear, clamped;
//       central differences inside, one-sided on the border);
//   horizontal Gaussian taps from a per-wavefront LDS row (border replicated);
//   the filtered row enters a ring of 2r + 1 rows held in registers, and the
//   vertical taps over the ring give u_new of row y - r.
// Two workgroup barriers per row, no 2-D tiles; the redundant work is the 2r halo
// rows per strip, (TY + 2r) / TY.  Per pixel: u (8 B) + R (4 B) + T (4 B gather)
// read, u_new (8 B) written = 24 B from HBM; the other R rows and the halo hit
// the caches.  Strips of one pair are placed on one XCD.
#include "dev_util.h"

namespace ebsd {

namespace {

// One demons iteration over output rows [y0, y0 + TY) of one image pair by a
// workgroup of 64 NW threads; thread t owns column t (w <= 64 NW), so every
// load, gather and store instruction touches consecutive addresses.
//
// Software pipeline per row step: issue the row's T gathers, then prefetch the
// next row's u and its one new R row; the gradient's x-neighbours come from the
// workgroup's LDS copy of the R row, the horizontal taps from its LDS copy of v
// (both double-buffered by row parity, so one barrier per row suffices).  The
// two other R rows and the u rows of the last 2r + 1 steps stay in registers.
// Returns the workgroup's sum of |u_new - u|^2 (all threads) when want_ss.
template <int NW, int RAD, int TY>
__device__ float demons_strip(const float* __restrict__ Rg, const float* __restrict__ Tg,
                              const float* __restrict__ ug, float* __restrict__ ung, int h, int w,
                              int y0, const Taps& tp, bool want_ss)
{
    const unsigned img_bytes = 4u * (unsigned)h * (unsigned)w;
    const __amdgpu_buffer_rsrc_t R = make_rsrc(Rg, img_bytes);
    const __amdgpu_buffer_rsrc_t T = make_rsrc(Tg, img_bytes);
    const __amdgpu_buffer_rsrc_t U = make_rsrc(ug, 2u * img_bytes);
    const __amdgpu_buffer_rsrc_t UN = make_rsrc(ung, 2u * img_bytes);
    constexpr int NR = 2 * RAD + 1;  // ring rows
    constexpr int STEPS = TY + 2 * RAD;
    constexpr int RW = 64 * NW;      // LDS row length
    __shared__ float lds_v[2][2][RW];  // [parity][channel][column]
    __shared__ float lds_r[2][RW];     // [parity][column]
    __shared__ float red[NW];
    const int c = threadIdx.x;
    const bool in = c < w;
    const int x = in ? c : w - 1;
    const int xm = max(x - 1, 0), xp = min(x + 1, w - 1);
    const float sx = (xp - xm == 2) ? 0.5f : 1.0f;
    int tap_col[2 * RAD + 1];
#pragma unroll
    for (int j = 0; j <= 2 * RAD; j++) tap_col[j] = clampi(x + j - RAD, 0, w - 1);
    const unsigned uw4 = 4u * (unsigned)w;
    const unsigned x4 = 4u * (unsigned)x;
    // byte offset of channel 1 of the field
    const unsigned ch1 = img_bytes;

    // Pipeline state at the start of step s (row y = y0 - RAD + s):
    //   r_m, r_c, r_p   R rows ym, yc, yp of row y (registers)
    //   ux, uy          field of row y;  g = T gathers of row y (in flight)
    //   ux1, uy1        field of row y + 1 (in flight)
    auto rowc = [&](int yy) { return clampi(yy, 0, h - 1); };
    int yc = rowc(y0 - RAD);
    int ym = max(yc - 1, 0), yp = min(yc + 1, h - 1);
    float r_m = bload(R, (unsigned)ym * uw4 + x4);
    float r_c = bload(R, (unsigned)yc * uw4 + x4);
    float r_p = bload(R, (unsigned)yp * uw4 + x4);
    float ux = bload(U, (unsigned)yc * uw4 + x4);
    float uy = bload(U, ch1 + (unsigned)yc * uw4 + x4);
    const int yc1 = rowc(y0 - RAD + 1);
    float ux1 = bload(U, (unsigned)yc1 * uw4 + x4);
    float uy1 = bload(U, ch1 + (unsigned)yc1 * uw4 + x4);
    Bilin g = bilinear_issue(T, h, w, (float)x + ux, (float)yc + uy);
    lds_r[0][c] = r_c;
    __syncthreads();

    float ring_x[NR], ring_y[NR], ring_ux[NR], ring_uy[NR];
    float ss = 0.0f;

#pragma unroll 1
    for (int base = 0; base < STEPS; base += NR) {
#pragma unroll
        for (int s = 0; s < NR; s++) {
            const int step = base + s;
            if (step >= STEPS) break;  // uniform
            const int par = step & 1;
            const int y = y0 - RAD + step;
            const bool more = step + 1 < STEPS;
            const bool more2 = step + 2 < STEPS;
            // 1. prefetch: field of row y + 2, the one new R row of row y + 1
            const int nyc = rowc(y + 1);
            const int nym = max(nyc - 1, 0), nyp = min(nyc + 1, h - 1);
            const int yc2 = rowc(y + 2);
            float n_rp = 0.0f, ux2 = 0.0f, uy2 = 0.0f;
            if (more) n_rp = bload(R, (unsigned)nyp * uw4 + x4);
            if (more2) {
                ux2 = bload(U, (unsigned)yc2 * uw4 + x4);
                uy2 = bload(U, ch1 + (unsigned)yc2 * uw4 + x4);
            }
            // 2. gathers of row y + 1 (its field was requested one step ago)
            Bilin g1 = g;
            if (more) g1 = bilinear_issue(T, h, w, (float)x + ux1, (float)nyc + uy1);
            // rows ym/yc of the next step are this step's yc/yp, or repeat at a clamped border
            const float n_rm = (nym == yc) ? r_c : (nym == yp ? r_p : r_m);
            const float n_rc = (nyc == yp) ? r_p : r_c;
            // 3. force of row y (its gathers were requested one step ago)
            const float wv = bilinear_blend(g);
            const float sy = (yp - ym == 2) ? 0.5f : 1.0f;
            const float gyr = (r_p - r_m) * sy;
            const float gxr = (lds_r[par][xp] - lds_r[par][xm]) * sx;
            const float a = r_c - wv;
            const float den = fmaf(gxr, gxr, fmaf(gyr, gyr, a * a));
            float vx = ux, vy = uy;
            if (den > 1e-9f) {
                const float q = a * __builtin_amdgcn_rcpf(den);
                vx = fmaf(q, gxr, ux);
                vy = fmaf(q, gyr, uy);
            }
            lds_v[par][0][c] = vx;
            lds_v[par][1][c] = vy;
            if (more) lds_r[par ^ 1][c] = n_rc;
            ring_ux[s] = ux;
            ring_uy[s] = uy;
            __syncthreads();
            // 4. horizontal taps at clamped columns
            float ax = 0.0f, ay = 0.0f;
#pragma unroll
            for (int j = 0; j <= 2 * RAD; j++) {
                ax = fmaf(tp.w[j], lds_v[par][0][tap_col[j]], ax);
                ay = fmaf(tp.w[j], lds_v[par][1][tap_col[j]], ay);
            }
            ring_x[s] = ax;
            ring_y[s] = ay;
            // 5. vertical taps over the ring: output row y - RAD
            if (step >= 2 * RAD) {
                const int yo = y - RAD;
                if (yo < h && in) {
                    float ox = 0.0f, oy = 0.0f;
#pragma unroll
                    for (int j = 0; j <= 2 * RAD; j++) {
                        // row yo - RAD + j was computed at step (step - 2 RAD + j)
                        const int slot = (s + 1 + j) % NR;
                        ox = fmaf(tp.w[j], ring_x[slot], ox);
                        oy = fmaf(tp.w[j], ring_y[slot], oy);
                    }
                    if (want_ss) {
                        // u of row yo was read at step (step - RAD)
                        const int us = (s + RAD + 1) % NR;
                        const float dx = ox - ring_ux[us], dy = oy - ring_uy[us];
                        ss = fmaf(dx, dx, fmaf(dy, dy, ss));
                    }
                    const unsigned o = (unsigned)yo * uw4 + 4u * (unsigned)c;
                    bstore(UN, o, ox);
                    bstore(UN, ch1 + o, oy);
                }
            }
            // 6. rotate
            r_m = n_rm;
            r_c = n_rc;
            r_p = n_rp;
            ux = ux1;
            uy = uy1;
            ux1 = ux2;
            uy1 = uy2;
            g = g1;
            ym = nym;
            yc = nyc;
            yp = nyp;
        }
    }
    if (!want_ss) return 0.0f;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
    if ((c & 63) == 0) red[c >> 6] = ss;
    __syncthreads();
    float tot = 0.0f;
#pragma unroll
    for (int i = 0; i < NW; i++) tot += red[i];
    __syncthreads();
    return tot;
}

// Two demons iterations over output rows [y0, y0 + TY) in one pass (temporal
// blocking).  Stage 1 is the iteration above, marched over input rows
// y0 - 2r .. y0 + TY + 2r - 1 so that it yields u1 = iteration(u) for rows
// y0 - r .. y0 + TY + r - 1; those rows never leave the workgroup: each
// thread keeps its column of the last 16 of them in an LDS history.  Stage 2
// runs the same iteration on u1, lagging stage 1 by 3r + 2 rows (its input
// row and the next one, whose gathers are issued a row ahead, are then always
// in the history, also at the top of the image where the clamped row index
// selects row 0 again), and writes u2 for the strip's own rows.  HBM traffic per
// pixel for the two iterations: u (8 B) + R (4 B) + two T gathers (8 B) read,
// u2 (8 B) written.  Every value is computed by the same instruction sequence
// as in demons_strip, so u2 equals two single iterations bit for bit.
// Returns the strip's sums of |u1 - u|^2 and |u2 - u1|^2 over its own rows.
template <int NW, int RAD, int TY>
__device__ float2 demons_strip2(const float* __restrict__ Rg, const float* __restrict__ Tg,
                                const float* __restrict__ ug, float* __restrict__ ung, int h, int w,
                                int y0, const Taps& tp, bool want_ss)
{
    const unsigned img_bytes = 4u * (unsigned)h * (unsigned)w;
    const __amdgpu_buffer_rsrc_t R = make_rsrc(Rg, img_bytes);
    const __amdgpu_buffer_rsrc_t T = make_rsrc(Tg, img_bytes);
    const __amdgpu_buffer_rsrc_t U = make_rsrc(ug, 2u * img_bytes);
    const __amdgpu_buffer_rsrc_t UN = make_rsrc(ung, 2u * img_bytes);
    constexpr int NR = 2 * RAD + 1;  // ring rows
    constexpr int S1 = TY + 4 * RAD; // stage-1 input rows
    constexpr int S2 = TY + 2 * RAD; // stage-2 input rows
    // Stage-2 lag: its first input row (clamped to row 0 at the top of the
    // image) must have left stage 1 before the step that issues its gathers.
    constexpr int D = 3 * RAD + 2;
    constexpr int STEPS = D + S2;    // >= S1
    constexpr int RW = 64 * NW;
    // History rows (row index mod NH): stage 2 reads a row up to 2r + 2 steps
    // after stage 1 wrote it, in the step in which stage 1 writes row + 2r + 2.
    constexpr int NH = 16;
    static_assert(2 * RAD + 3 <= NH, "history too short for this radius");
    __shared__ float lds_v[2][2][RW];
    __shared__ float lds_r[2][RW];
    __shared__ float lds_v2[2][2][RW];
    __shared__ float lds_r2[2][RW];
    __shared__ float hist[NH][2][RW];
    __shared__ float red[2][NW];
    const int c = threadIdx.x;
    const bool in = c < w;
    const int x = in ? c : w - 1;
    const int xm = max(x - 1, 0), xp = min(x + 1, w - 1);
    const float sx = (xp - xm == 2) ? 0.5f : 1.0f;
    int tap_col[2 * RAD + 1];
#pragma unroll
    for (int j = 0; j <= 2 * RAD; j++) tap_col[j] = clampi(x + j - RAD, 0, w - 1);
    const unsigned uw4 = 4u * (unsigned)w;
    const unsigned x4 = 4u * (unsigned)x;
    const unsigned ch1 = img_bytes;
    auto rowc = [&](int yy) { return clampi(yy, 0, h - 1); };

    // stage 1 pipeline state (as in demons_strip), starting at input row y0 - 2r
    int yc = rowc(y0 - 2 * RAD);
    int ym = max(yc - 1, 0), yp = min(yc + 1, h - 1);
    float r_m = bload(R, (unsigned)ym * uw4 + x4);
    float r_c = bload(R, (unsigned)yc * uw4 + x4);
    float r_p = bload(R, (unsigned)yp * uw4 + x4);
    float ux = bload(U, (unsigned)yc * uw4 + x4);
    float uy = bload(U, ch1 + (unsigned)yc * uw4 + x4);
    const int yc1 = rowc(y0 - 2 * RAD + 1);
    float ux1 = bload(U, (unsigned)yc1 * uw4 + x4);
    float uy1 = bload(U, ch1 + (unsigned)yc1 * uw4 + x4);
    Bilin g = bilinear_issue(T, h, w, (float)x + ux, (float)yc + uy);
    lds_r[0][c] = r_c;
    // stage 2 state: R rows of its first input row y0 - r; its u1 and gathers
    // are taken from the history one step before its first step
    int zc = rowc(y0 - RAD);
    int zm = max(zc - 1, 0), zp = min(zc + 1, h - 1);
    float q_m = bload(R, (unsigned)zm * uw4 + x4);
    float q_c = bload(R, (unsigned)zc * uw4 + x4);
    float q_p = bload(R, (unsigned)zp * uw4 + x4);
    lds_r2[0][c] = q_c;
    __syncthreads();

    float ring_x[NR], ring_y[NR], ring_ux[NR], ring_uy[NR];
    float ring2_x[NR], ring2_y[NR];
    float v1x = 0.0f, v1y = 0.0f;
    Bilin g2 = g;
    float ss1 = 0.0f, ss2 = 0.0f;

#pragma unroll 1
    for (int base = 0; base < STEPS; base += NR) {
#pragma unroll
        for (int s = 0; s < NR; s++) {
            const int S = base + s;
            if (S >= STEPS) break;  // uniform
            const bool st1 = S < S1;
            const int par = S & 1;
            const int s2 = S - D;  // stage-2 step
            const bool st2 = s2 >= 0;
            const int par2 = s2 & 1;
            const int slot2 = (s + NR - D % NR) % NR;  // s2 mod NR (base is a multiple of NR)

            // ---- stage 1, before the barrier: prefetch, gathers, force of row y ----
            int nym = ym, nyc = yc, nyp = yp;
            float n_rm = r_m, n_rc = r_c, n_rp = r_p, ux2 = 0.0f, uy2 = 0.0f;
            Bilin g1 = g;
            if (st1) {
                const int y = y0 - 2 * RAD + S;
                const bool more = S + 1 < S1;
                const bool more2 = S + 2 < S1;
                nyc = rowc(y + 1);
                nym = max(nyc - 1, 0);
                nyp = min(nyc + 1, h - 1);
                const int yc2 = rowc(y + 2);
                if (more) n_rp = bload(R, (unsigned)nyp * uw4 + x4);
                if (more2) {
                    ux2 = bload(U, (unsigned)yc2 * uw4 + x4);
                    uy2 = bload(U, ch1 + (unsigned)yc2 * uw4 + x4);
                }
                if (more) g1 = bilinear_issue(T, h, w, (float)x + ux1, (float)nyc + uy1);
                n_rm = (nym == yc) ? r_c : (nym == yp ? r_p : r_m);
                n_rc = (nyc == yp) ? r_p : r_c;
                const float wv = bilinear_blend(g);
                const float sy = (yp - ym == 2) ? 0.5f : 1.0f;
                const float gyr = (r_p - r_m) * sy;
                const float gxr = (lds_r[par][xp] - lds_r[par][xm]) * sx;
                const float a = r_c - wv;
                const float den = fmaf(gxr, gxr, fmaf(gyr, gyr, a * a));
                float vx = ux, vy = uy;
                if (den > 1e-9f) {
                    const float q = a * __builtin_amdgcn_rcpf(den);
                    vx = fmaf(q, gxr, ux);
                    vy = fmaf(q, gyr, uy);
                }
                lds_v[par][0][c] = vx;
                lds_v[par][1][c] = vy;
                if (more) lds_r[par ^ 1][c] = n_rc;
                ring_ux[s] = ux;
                ring_uy[s] = uy;
            }
            // ---- stage 2, before the barrier ----
            if (S == D - 1) {  // u1 and gathers of stage 2's first input row
                const int r0 = rowc(y0 - RAD);
                v1x = hist[r0 & (NH - 1)][0][c];
                v1y = hist[r0 & (NH - 1)][1][c];
                g2 = bilinear_issue(T, h, w, (float)x + v1x, (float)r0 + v1y);
            }
            int nzm = zm, nzc = zc, nzp = zp;
            float n_qm = q_m, n_qc = q_c, n_qp = q_p, v1x_n = v1x, v1y_n = v1y;
            Bilin g2n = g2;
            if (st2) {
                const int y2 = y0 - RAD + s2;
                const bool more = s2 + 1 < S2;
                nzc = rowc(y2 + 1);
                nzm = max(nzc - 1, 0);
                nzp = min(nzc + 1, h - 1);
                if (more) {
                    v1x_n = hist[nzc & (NH - 1)][0][c];
                    v1y_n = hist[nzc & (NH - 1)][1][c];
                    g2n = bilinear_issue(T, h, w, (float)x + v1x_n, (float)nzc + v1y_n);
                    n_qp = bload(R, (unsigned)nzp * uw4 + x4);
                }
                n_qm = (nzm == zc) ? q_c : (nzm == zp ? q_p : q_m);
                n_qc = (nzc == zp) ? q_p : q_c;
                const float wv = bilinear_blend(g2);
                const float sy = (zp - zm == 2) ? 0.5f : 1.0f;
                const float gyr = (q_p - q_m) * sy;
                const float gxr = (lds_r2[par2][xp] - lds_r2[par2][xm]) * sx;
                const float a = q_c - wv;
                const float den = fmaf(gxr, gxr, fmaf(gyr, gyr, a * a));
                float vx = v1x, vy = v1y;
                if (den > 1e-9f) {
                    const float q = a * __builtin_amdgcn_rcpf(den);
                    vx = fmaf(q, gxr, v1x);
                    vy = fmaf(q, gyr, v1y);
                }
                lds_v2[par2][0][c] = vx;
                lds_v2[par2][1][c] = vy;
                if (more) lds_r2[par2 ^ 1][c] = n_qc;
            }
            __syncthreads();
            // ---- stage 1, after the barrier: taps, u1 row y - r into the history ----
            if (st1) {
                float ax = 0.0f, ay = 0.0f;
#pragma unroll
                for (int j = 0; j <= 2 * RAD; j++) {
                    ax = fmaf(tp.w[j], lds_v[par][0][tap_col[j]], ax);
                    ay = fmaf(tp.w[j], lds_v[par][1][tap_col[j]], ay);
                }
                ring_x[s] = ax;
                ring_y[s] = ay;
                if (S >= 2 * RAD) {
                    const int yo = y0 - 3 * RAD + S;
                    if (yo >= 0 && yo < h) {
                        float ox = 0.0f, oy = 0.0f;
#pragma unroll
                        for (int j = 0; j <= 2 * RAD; j++) {
                            const int sl = (s + 1 + j) % NR;
                            ox = fmaf(tp.w[j], ring_x[sl], ox);
                            oy = fmaf(tp.w[j], ring_y[sl], oy);
                        }
                        hist[yo & (NH - 1)][0][c] = ox;
                        hist[yo & (NH - 1)][1][c] = oy;
                        if (want_ss && in && yo >= y0 && yo < y0 + TY) {
                            const int us = (s + RAD + 1) % NR;
                            const float dx = ox - ring_ux[us], dy = oy - ring_uy[us];
                            ss1 = fmaf(dx, dx, fmaf(dy, dy, ss1));
                        }
                    }
                }
                r_m = n_rm;
                r_c = n_rc;
                r_p = n_rp;
                ux = ux1;
                uy = uy1;
                ux1 = ux2;
                uy1 = uy2;
                g = g1;
                ym = nym;
                yc = nyc;
                yp = nyp;
            }
            // ---- stage 2, after the barrier: taps, u2 of row y2 - r ----
            if (st2) {
                float ax = 0.0f, ay = 0.0f;
#pragma unroll
                for (int j = 0; j <= 2 * RAD; j++) {
                    ax = fmaf(tp.w[j], lds_v2[par2][0][tap_col[j]], ax);
                    ay = fmaf(tp.w[j], lds_v2[par2][1][tap_col[j]], ay);
                }
                ring2_x[slot2] = ax;
                ring2_y[slot2] = ay;
                if (s2 >= 2 * RAD) {
                    const int yo = y0 - 2 * RAD + s2;
                    if (yo < h && in) {
                        float ox = 0.0f, oy = 0.0f;
#pragma unroll
                        for (int j = 0; j <= 2 * RAD; j++) {
                            const int sl = (slot2 + 1 + j) % NR;
                            ox = fmaf(tp.w[j], ring2_x[sl], ox);
                            oy = fmaf(tp.w[j], ring2_y[sl], oy);
                        }
                        if (want_ss) {
                            const float dx = ox - hist[yo & (NH - 1)][0][c];
                            const float dy = oy - hist[yo & (NH - 1)][1][c];
                            ss2 = fmaf(dx, dx, fmaf(dy, dy, ss2));
                        }
                        const unsigned o = (unsigned)yo * uw4 + 4u * (unsigned)c;
                        bstore(UN, o, ox);
                        bstore(UN, ch1 + o, oy);
                    }
                }
                q_m = n_qm;
                q_c = n_qc;
                q_p = n_qp;
                v1x = v1x_n;
                v1y = v1y_n;
                g2 = g2n;
                zm = nzm;
                zc = nzc;
                zp = nzp;
            }
        }
    }
    if (!want_ss) return make_float2(0.0f, 0.0f);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        ss1 += __shfl_xor(ss1, off, 64);
        ss2 += __shfl_xor(ss2, off, 64);
    }
    if ((c & 63) == 0) {
        red[0][c >> 6] = ss1;
        red[1][c >> 6] = ss2;
    }
    __syncthreads();
    float t1 = 0.0f, t2 = 0.0f;
#pragma unroll
    for (int i = 0; i < NW; i++) {
        t1 += red[0][i];
        t2 += red[1][i];
    }
    __syncthreads();
    return make_float2(t1, t2);
}

template <int NW, int RAD, int TY>
__global__ void __launch_bounds__(64 * NW)
    k_demons_rows(const Bucket* __restrict__ bk, int level, int k, Taps tp, float tol, int nstrips)
{
    __shared__ double sh_sum;
    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int b = lb / nstrips;
    const int strip = lb - b * nstrips;
    const PairState st = bk->state[b];
    if (st.stop >= 0) return;  // uniform
    const int h = bk->H >> level, w = bk->W >> level;
    const int64_t npart = (int64_t)bk->nb * bk->max_tiles;
    if (tol > 0.0f && k > 0) {
        const float* prev = bk->partial + ((k - 1) & 1) * npart + (int64_t)b * bk->max_tiles;
        const double ss = pair_sum(prev, nstrips, &sh_sum);
        const double delta = sqrt(ss / ((double)h * (double)w)) * (double)(1 << level);
        if (delta < (double)tol) {
            if (strip == 0 && threadIdx.x == 0) {
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
    const float ss = demons_strip<NW, RAD, TY>(R, T, u, un, h, w, strip * TY, tp, tol > 0.0f);
    if (tol > 0.0f && threadIdx.x == 0)
        bk->partial[(k & 1) * npart + (int64_t)b * bk->max_tiles + strip] = ss;
}

// Launch L of a level run two iterations at a time: iterations k = 2L and
// k + 1 read the field from buffer (base + L) & 1 and leave u_{k+2} in buffer
// (base + L + 1) & 1; the partial sums of iteration i go to slot i & 3.  The
// second iteration is run before the stop decision on the first is known;
// the next launch takes the decisions in iteration order from the previous
// launch's sums, exactly as single-iteration launches would:
//   |u_{k-1} - u_{k-2}| below tol: the pair stopped after k - 1 iterations,
//     u_{k-1} is recomputed from u_{k-2} (still in buffer (base + L + 1) & 1)
//     into buffer (base + L) & 1;
//   |u_k - u_{k-1}| below tol: stopped after k iterations, u_k is in place.
// A launch with k >= cap only takes these decisions; one with k + 1 == cap
// runs a single iteration.  The final field of a pair that ran n iterations
// is in buffer (base + ceil(n / 2)) & 1.
template <int NW, int RAD, int TY>
__global__ void __launch_bounds__(64 * NW)
    k_demons_rows2(const Bucket* __restrict__ bk, int level, int L, Taps tp, float tol, int nstrips, int cap)
{
    __shared__ double sh_sum;
    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int b = lb / nstrips;
    const int strip = lb - b * nstrips;
    const PairState st = bk->state[b];
    if (st.stop >= 0) return;  // uniform
    const int h = bk->H >> level, w = bk->W >> level;
    const int64_t npart = (int64_t)bk->nb * bk->max_tiles;
    const int64_t pofs = (int64_t)b * bk->max_tiles;
    const int k = 2 * L;
    bool recompute = false;
    if (tol > 0.0f && L > 0) {
        const double hw = (double)h * (double)w, sc = (double)(1 << level);
        const double ssa = pair_sum(bk->partial + ((k - 2) & 3) * npart + pofs, nstrips, &sh_sum);
        if (sqrt(ssa / hw) * sc < (double)tol) {
            recompute = true;
        } else {
            const double ssb = pair_sum(bk->partial + ((k - 1) & 3) * npart + pofs, nstrips, &sh_sum);
            if (sqrt(ssb / hw) * sc < (double)tol) {
                if (strip == 0 && threadIdx.x == 0) {
                    bk->state[b].stop = k;
                    bk->state[b].convmask = st.convmask | (1u << level);
                }
                return;
            }
        }
    }
    const int64_t slot = (int64_t)b * 2 * bk->H * bk->W;
    const float* R = bk->ref_pyr + (int64_t)bk->ref_slot[b] * bk->pyr_elems + bk->lvl_off[level];
    const float* T = bk->test_pyr + (int64_t)b * bk->pyr_elems + bk->lvl_off[level];
    float* fa = bk->field[(st.base + L) & 1] + slot;
    float* fb = bk->field[(st.base + L + 1) & 1] + slot;
    if (recompute) {
        if (strip == 0 && threadIdx.x == 0) {
            bk->state[b].stop = k - 1;
            bk->state[b].convmask = st.convmask | (1u << level);
        }
        demons_strip<NW, RAD, TY>(R, T, fb, fa, h, w, strip * TY, tp, false);
        return;
    }
    if (k >= cap) return;
    if (k + 1 < cap) {
        const float2 ss = demons_strip2<NW, RAD, TY>(R, T, fa, fb, h, w, strip * TY, tp, tol > 0.0f);
        if (tol > 0.0f && threadIdx.x == 0) {
            bk->partial[(k & 3) * npart + pofs + strip] = ss.x;
            bk->partial[((k + 1) & 3) * npart + pofs + strip] = ss.y;
        }
    } else {
        const float ss = demons_strip<NW, RAD, TY>(R, T, fa, fb, h, w, strip * TY, tp, tol > 0.0f);
        if (tol > 0.0f && threadIdx.x == 0) bk->partial[(k & 3) * npart + pofs + strip] = ss;
    }
}

// Stand-alone variant: one workgroup per pair walks its strips in order.
template <int NW, int RAD, int TY>
__global__ void __launch_bounds__(64 * NW)
    k_demons_rows_stage(const float* __restrict__ R, const float* __restrict__ T, int h, int w,
                        const float* __restrict__ u, Taps tp, float* __restrict__ un,
                        double* __restrict__ rms)
{
    const int b = blockIdx.x;
    const int64_t hw = (int64_t)h * w;
    double acc = 0.0;
    for (int y0 = 0; y0 < h; y0 += TY)
        acc += (double)demons_strip<NW, RAD, TY>(R + b * hw, T + b * hw, u + 2 * b * hw,
                                                  un + 2 * b * hw, h, w, y0, tp, true);
    if (rms && threadIdx.x == 0) rms[b] = sqrt(acc / (double)hw);
}

template <int CPL, int RAD, int TY>
void launch_rows(const Bucket* d_bk, int nb, int h, int level, int k, const Taps& tp, float tol,
                 hipStream_t s)
{
    const int nstrips = (h + TY - 1) / TY;
    hipLaunchKernelGGL((k_demons_rows<CPL, RAD, TY>), dim3(nb * nstrips), dim3(64 * CPL), 0, s, d_bk,
                       level, k, tp, tol, nstrips);
}

template <int CPL, int RAD>
bool dispatch_ty(const Bucket* d_bk, int nb, int h, int level, int k, const Taps& tp, float tol,
                 int ty, hipStream_t s)
{
    switch (ty) {
    case 16: launch_rows<CPL, RAD, 16>(d_bk, nb, h, level, k, tp, tol, s); return true;
    case 32: launch_rows<CPL, RAD, 32>(d_bk, nb, h, level, k, tp, tol, s); return true;
    case 64: launch_rows<CPL, RAD, 64>(d_bk, nb, h, level, k, tp, tol, s); return true;
    case 128: launch_rows<CPL, RAD, 128>(d_bk, nb, h, level, k, tp, tol, s); return true;
    default: return false;
    }
}

template <int CPL>
bool dispatch_rad(const Bucket* d_bk, int nb, int h, int level, int k, const Taps& tp, int radius,
                  float tol, int ty, hipStream_t s)
{
    switch (radius) {
    case 0: return dispatch_ty<CPL, 0>(d_bk, nb, h, level, k, tp, tol, ty, s);
    case 1: return dispatch_ty<CPL, 1>(d_bk, nb, h, level, k, tp, tol, ty, s);
    case 2: return dispatch_ty<CPL, 2>(d_bk, nb, h, level, k, tp, tol, ty, s);
    case 3: return dispatch_ty<CPL, 3>(d_bk, nb, h, level, k, tp, tol, ty, s);
    case 4: return dispatch_ty<CPL, 4>(d_bk, nb, h, level, k, tp, tol, ty, s);
    default: return false;
    }
}

template <int CPL, int RAD, int TY>
void launch_rows2(const Bucket* d_bk, int nb, int h, int level, int L, const Taps& tp, float tol, int cap,
                  hipStream_t s)
{
    const int nstrips = (h + TY - 1) / TY;
    hipLaunchKernelGGL((k_demons_rows2<CPL, RAD, TY>), dim3(nb * nstrips), dim3(64 * CPL), 0, s, d_bk, level, L,
                       tp, tol, nstrips, cap);
}

template <int CPL, int RAD>
bool dispatch_ty2(const Bucket* d_bk, int nb, int h, int level, int L, const Taps& tp, float tol, int cap, int ty,
                  hipStream_t s)
{
    switch (ty) {
    case 32: launch_rows2<CPL, RAD, 32>(d_bk, nb, h, level, L, tp, tol, cap, s); return true;
    case 64: launch_rows2<CPL, RAD, 64>(d_bk, nb, h, level, L, tp, tol, cap, s); return true;
    case 128: launch_rows2<CPL, RAD, 128>(d_bk, nb, h, level, L, tp, tol, cap, s); return true;
    default: return false;
    }
}

template <int CPL>
bool dispatch_rad2(const Bucket* d_bk, int nb, int h, int level, int L, const Taps& tp, int radius, float tol,
                   int cap, int ty, hipStream_t s)
{
    switch (radius) {
    case 0: return dispatch_ty2<CPL, 0>(d_bk, nb, h, level, L, tp, tol, cap, ty, s);
    case 1: return dispatch_ty2<CPL, 1>(d_bk, nb, h, level, L, tp, tol, cap, ty, s);
    case 2: return dispatch_ty2<CPL, 2>(d_bk, nb, h, level, L, tp, tol, cap, ty, s);
    case 3: return dispatch_ty2<CPL, 3>(d_bk, nb, h, level, L, tp, tol, cap, ty, s);
    case 4: return dispatch_ty2<CPL, 4>(d_bk, nb, h, level, L, tp, tol, cap, ty, s);
    default: return false;
    }
}

constexpr int kStageTY = 64;

template <int CPL, int RAD>
void launch_rows_stage(const float* R, const float* T, int n, int h, int w, const float* u,
                       const Taps& tp, float* un, double* rms, hipStream_t s)
{
    hipLaunchKernelGGL((k_demons_rows_stage<CPL, RAD, kStageTY>), dim3(n), dim3(64 * CPL), 0, s, R, T,
                       h, w, u, tp, un, rms);
}

template <int CPL>
bool dispatch_rad_stage(const float* R, const float* T, int n, int h, int w, const float* u,
                        const Taps& tp, int radius, float* un, double* rms, hipStream_t s)
{
    switch (radius) {
    case 0: launch_rows_stage<CPL, 0>(R, T, n, h, w, u, tp, un, rms, s); return true;
    case 1: launch_rows_stage<CPL, 1>(R, T, n, h, w, u, tp, un, rms, s); return true;
    case 2: launch_rows_stage<CPL, 2>(R, T, n, h, w, u, tp, un, rms, s); return true;
    case 3: launch_rows_stage<CPL, 3>(R, T, n, h, w, u, tp, un, rms, s); return true;
    case 4: launch_rows_stage<CPL, 4>(R, T, n, h, w, u, tp, un, rms, s); return true;
    default: return false;
    }
}

}  // namespace

int rows_cpl(int w)
{
    if (w <= 64) return 1;
    if (w <= 128) return 2;
    if (w <= 256) return 4;
    return 0;
}

bool rows_ty_supported(int ty) { return ty == 16 || ty == 32 || ty == 64 || ty == 128; }

bool rows2_ty_supported(int ty) { return ty == 32 || ty == 64 || ty == 128; }

bool launch_demons_rows2(const Bucket* d_bk, const Bucket& hb, int level, int L, const Taps& tp, int radius,
                         float tol, int cap, int ty, hipStream_t s)
{
    const int h = hb.H >> level, w = hb.W >> level;
    switch (rows_cpl(w)) {
    case 1: return dispatch_rad2<1>(d_bk, hb.nb, h, level, L, tp, radius, tol, cap, ty, s);
    case 2: return dispatch_rad2<2>(d_bk, hb.nb, h, level, L, tp, radius, tol, cap, ty, s);
    case 4: return dispatch_rad2<4>(d_bk, hb.nb, h, level, L, tp, radius, tol, cap, ty, s);
    default: return false;
    }
}

int rows_units(int h, int ty) { return (h + ty - 1) / ty; }

bool launch_demons_rows(const Bucket* d_bk, const Bucket& hb, int level, int k, const Taps& tp,
                        int radius, float tol, int ty, hipStream_t s)
{
    const int h = hb.H >> level, w = hb.W >> level;
    switch (rows_cpl(w)) {
    case 1: return dispatch_rad<1>(d_bk, hb.nb, h, level, k, tp, radius, tol, ty, s);
    case 2: return dispatch_rad<2>(d_bk, hb.nb, h, level, k, tp, radius, tol, ty, s);
    case 4: return dispatch_rad<4>(d_bk, hb.nb, h, level, k, tp, radius, tol, ty, s);
    default: return false;
    }
}

bool launch_demons_rows_stage(const float* R, const float* T, int n, int h, int w, const float* u,
                              const Taps& tp, int radius, float* un, double* rms, hipStream_t s)
{
    switch (rows_cpl(w)) {
    case 1: return dispatch_rad_stage<1>(R, T, n, h, w, u, tp, radius, un, rms, s);
    case 2: return dispatch_rad_stage<2>(R, T, n, h, w, u, tp, radius, un, rms, s);
    case 4: return dispatch_rad_stage<4>(R, T, n, h, w, u, tp, radius, un, rms, s);
    default: return false;
    }
}

}  // namespace ebsd
