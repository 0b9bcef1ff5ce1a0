// Row-marching demons iteration for gfx950 (kernel templates; each
// k_demons_rows_w<NW>.hip instantiates one row width) (multi-resolution demons of
// arXiv:1907.05993 section 1, Eq. (1) force).
//
// One workgroup of 64 NW threads (NW = 8 wavefronts for 512 px, 4 for 256 px,
// 2 for 128 px, 1 for 64 px) owns a strip of TY output rows of one pair; thread t owns column
// t, so a workgroup spans a whole row and every memory instruction is
// contiguous across the lanes.  A level wider than 512 px is cut into column
// segments: lane t owns column sx0 + t, the kSegHalo lanes at either end
// recompute their neighbours' columns (their own gradients and taps reach
// past the segment and are wrong, which two iterations of radius r carry at
// most 2r + 1 lanes inward), and only columns [ws, we) are written.
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
#pragma once

#include <type_traits>

#include "dev_util.h"

namespace ebsd {

namespace {

// LDS rows of the strip kernels.  The field row (vx, vy) is stored as pairs
// with RAD replicated border columns on each side and the R row with one, so
// every horizontal tap and both gradient neighbours of column x are at fixed
// offsets from one per-lane base (immediate offsets of the LDS reads, no
// clamped column indices); lane 0 and lane w - 1 also write the border copies.
// Two copies by row parity: one barrier per row suffices.
template <int NW, int RAD>
struct StripRows {
    static constexpr int RW = 64 * NW;
    static constexpr int PW = RW + 2 * RAD;  // padded (vx, vy) row
    static constexpr int PR = RW + 2;        // padded R row
    float2 v[2 * PW];
    float r[2 * PR];
};

// Byte bases of column x in the two parities of a StripRows.
struct RowBase {
    unsigned v, r;
};
template <int NW, int RAD>
__device__ inline void row_bases(int x, RowBase& a, RowBase& b)
{
    a.v = 8u * (unsigned)x;
    a.r = 4u * (unsigned)x;
    b.v = a.v + 8u * StripRows<NW, RAD>::PW;
    b.r = a.r + 4u * StripRows<NW, RAD>::PR;
}
template <class T>
__device__ inline T& lds_at(void* base, unsigned byte)
{
    return *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte);
}

// Store the force result of column x (and its border copies) into the field
// row at base rb; taps of column x then read rb + 8 j, j = 0 .. 2 RAD.
template <int RAD>
__device__ inline void put_v(float2* rows, unsigned rb, int c, int w, float vx, float vy)
{
    const float2 v = make_float2(vx, vy);
    lds_at<float2>(rows, rb + 8u * RAD) = v;
    if (c == 0) {
#pragma unroll
        for (int j = 0; j < RAD; j++) lds_at<float2>(rows, rb + 8u * j) = v;
    }
    if (c == w - 1) {
#pragma unroll
        for (int j = 0; j < RAD; j++) lds_at<float2>(rows, rb + 8u * (RAD + 1 + j)) = v;
    }
}
// Store the R value of column x (and its border copies) at base rb; the
// gradient of column x reads rb and rb + 8.
__device__ inline void put_r(float* rows, unsigned rb, int c, int w, float r)
{
    lds_at<float>(rows, rb + 4u) = r;
    if (c == 0) lds_at<float>(rows, rb) = r;
    if (c == w - 1) lds_at<float>(rows, rb + 8u) = r;
}
template <int RAD>
__device__ inline void taps_h(float2* rows, unsigned rb, const Taps& tp, float& ax, float& ay)
{
    ax = 0.0f;
    ay = 0.0f;
#pragma unroll
    for (int j = 0; j <= 2 * RAD; j++) {
        const float2 t = lds_at<float2>(rows, rb + 8u * j);
        ax = fmaf(tp.w[j], t.x, ax);
        ay = fmaf(tp.w[j], t.y, ay);
    }
}

// One demons iteration over output rows [y0, y0 + TY) of one image pair by a
// workgroup of 64 NW threads; thread t owns column t (w <= 64 NW), so every
// load, gather and store instruction touches consecutive addresses.
//
// Software pipeline per row step: issue the row's T gathers, then prefetch the
// next row's u and its one new R row; the gradient's x-neighbours and the
// horizontal taps come from the workgroup's LDS rows (StripRows).  The two
// other R rows and the u rows of the last 2r + 1 steps stay in registers.
// Row offsets are uniform (scalar offset operands of the buffer accesses).
// Returns the workgroup's sum of |u_new - u|^2 (all threads) when want_ss.
template <int NW, int RAD, int TY>
__device__ float demons_strip(const float* __restrict__ Rg, const float* __restrict__ Tg,
                              const float* __restrict__ ug, float* __restrict__ ung, int h, int w,
                              int y0, int sx0, int ws, int we, const Taps& tp, bool want_ss)
{
    const unsigned img_bytes = 4u * (unsigned)h * (unsigned)w;
    const __amdgpu_buffer_rsrc_t R = make_rsrc(Rg, img_bytes);
    const __amdgpu_buffer_rsrc_t T = make_rsrc(Tg, img_bytes);
    const __amdgpu_buffer_rsrc_t U = make_rsrc(ug, 2u * img_bytes);
    const __amdgpu_buffer_rsrc_t UN = make_rsrc(ung, 2u * img_bytes);
    constexpr int NR = 2 * RAD + 1;  // ring rows
    constexpr int STEPS = TY + 2 * RAD;
    __shared__ StripRows<NW, RAD> L;
    __shared__ float red[NW];
    const int c = threadIdx.x;
    const int gx = sx0 + c;  // the lane's column; written when inside [ws, we)
    const bool in = gx >= ws && gx < we;
    const int x = clampi(gx, 0, w - 1);
    const int xm = max(x - 1, 0), xp = min(x + 1, w - 1);
    const float sx = (xp - xm == 2) ? 0.5f : 1.0f;
    const BilGeom gg = bil_geom(h, w);
    const unsigned uw4 = 4u * (unsigned)w;
    const unsigned x4 = 4u * (unsigned)x;
    // byte offset of channel 1 of the field
    const unsigned ch1 = img_bytes;
    RowBase cur, oth;
    row_bases<NW, RAD>(x - sx0, cur, oth);

    // Pipeline state at the start of step s (row y = y0 - RAD + s):
    //   r_m, r_c, r_p   R rows ym, yc, yp of row y (registers)
    //   ux, uy          field of row y;  g = T gathers of row y (in flight)
    //   ux1, uy1        field of row y + 1 (in flight)
    auto rowc = [&](int yy) { return clampi(yy, 0, h - 1); };
    int yc = rowc(y0 - RAD);
    int ym = max(yc - 1, 0), yp = min(yc + 1, h - 1);
    float r_m = bload_s(R, x4, (unsigned)ym * uw4);
    float r_c = bload_s(R, x4, (unsigned)yc * uw4);
    float r_p = bload_s(R, x4, (unsigned)yp * uw4);
    float ux = bload_s(U, x4, (unsigned)yc * uw4);
    float uy = bload_s(U, x4, ch1 + (unsigned)yc * uw4);
    const int yc1 = rowc(y0 - RAD + 1);
    float ux1 = bload_s(U, x4, (unsigned)yc1 * uw4);
    float uy1 = bload_s(U, x4, ch1 + (unsigned)yc1 * uw4);
    Bilin g = bilinear_issue_g(T, gg, (float)x + ux, (float)yc + uy);
    put_r(L.r, cur.r, gx, w, r_c);
    __syncthreads();

    float ring_x[NR], ring_y[NR], ring_ux[NR], ring_uy[NR];
    float ss = 0.0f;

#pragma unroll 1
    for (int base = 0; base < STEPS; base += NR) {
#pragma unroll
        for (int s = 0; s < NR; s++) {
            const int step = base + s;
            if (step >= STEPS) break;  // uniform
            const int y = y0 - RAD + step;
            const bool more = step + 1 < STEPS;
            const bool more2 = step + 2 < STEPS;
            // 1. prefetch: field of row y + 2, the one new R row of row y + 1
            const int nyc = rowc(y + 1);
            const int nym = max(nyc - 1, 0), nyp = min(nyc + 1, h - 1);
            const int yc2 = rowc(y + 2);
            float n_rp = 0.0f, ux2 = 0.0f, uy2 = 0.0f;
            if (more) n_rp = bload_s(R, x4, (unsigned)nyp * uw4);
            if (more2) {
                ux2 = bload_s(U, x4, (unsigned)yc2 * uw4);
                uy2 = bload_s(U, x4, ch1 + (unsigned)yc2 * uw4);
            }
            // 2. gathers of row y + 1 (its field was requested one step ago)
            Bilin g1 = g;
            if (more) g1 = bilinear_issue_g(T, gg, (float)x + ux1, (float)nyc + uy1);
            // rows ym/yc of the next step are this step's yc/yp, or repeat at a clamped border
            const float n_rm = (nym == yc) ? r_c : (nym == yp ? r_p : r_m);
            const float n_rc = (nyc == yp) ? r_p : r_c;
            // 3. force of row y (its gathers were requested one step ago)
            const float wv = bilinear_blend_g(g);
            const float sy = (yp - ym == 2) ? 0.5f : 1.0f;
            const float gyr = (r_p - r_m) * sy;
            const float gxr = (lds_at<float>(L.r, cur.r + 8u) - lds_at<float>(L.r, cur.r)) * sx;
            const float a = r_c - wv;
            const float den = fmaf(gxr, gxr, fmaf(gyr, gyr, a * a));
            float vx = ux, vy = uy;
            if (den > 1e-9f) {
                const float q = a * __builtin_amdgcn_rcpf(den);
                vx = fmaf(q, gxr, ux);
                vy = fmaf(q, gyr, uy);
            }
            put_v<RAD>(L.v, cur.v, gx, w, vx, vy);
            if (more) put_r(L.r, oth.r, gx, w, n_rc);
            ring_ux[s] = ux;
            ring_uy[s] = uy;
            __syncthreads();
            // 4. horizontal taps (border columns replicated in the LDS row)
            taps_h<RAD>(L.v, cur.v, tp, ring_x[s], ring_y[s]);
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
                    const unsigned o = (unsigned)yo * uw4;
                    bstore_s(UN, x4, o, ox);
                    bstore_s(UN, x4, ch1 + o, oy);
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
            const RowBase t = cur;
            cur = oth;
            oth = t;
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
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// Loop-invariant context of demons_strip2.
template <int NW, int RAD>
struct Strip2Ctx {
    __amdgpu_buffer_rsrc_t R, T, U, UN;
    BilGeom gg;
    unsigned uw4, x4, ch1;
    int c, gx, x, h, w, y0;
    bool in, want_ss;
    float sx;
    StripRows<NW, RAD>* L1;
    StripRows<NW, RAD>* L2;
    float2 (*hist)[64 * NW];
    __device__ int rowc(int yy) const { return clampi(yy, 0, h - 1); }
};

// Pipeline state of the two stages (see demons_strip for stage 1; stage 2
// is the same iteration on the rows of u1 that stage 1 leaves in the history).
template <int RAD>
struct Strip2State {
    static constexpr int NR = 2 * RAD + 1;
    int ym, yc, yp;
    float r_m, r_c, r_p, ux, uy, ux1, uy1;
    Bilin g;
    float ring_x[NR], ring_y[NR], ring_ux[NR], ring_uy[NR];
    RowBase cur1, oth1;
    float ss1;
    int zm, zc, zp;
    float q_m, q_c, q_p, v1x, v1y;
    Bilin g2;
    float ring2_x[NR], ring2_y[NR];
    RowBase cur2, oth2;
    float ss2;
};

// One step S of the two-stage march.  SL1, SL2: ring slots of the stages
// (S mod NR, (S - D) mod NR); DO1, DO2: which stages run; OUT1, OUT2: whether
// a stage's vertical taps complete a row in this step; INIT2: the step before
// stage 2's first (S = D - 1), which fetches its first input row.  All are
// compile-time in every phase of the march, so the ring slots are fixed
// registers and no state is merged across branches.  The prefetches of a
// stage's last step are issued anyway (clamped rows, always inside the image).
template <int NW, int RAD, int TY, int SL1, int SL2, bool DO1, bool DO2, bool OUT1, bool OUT2, bool INIT2>
__device__ __forceinline__ void strip2_step(const Strip2Ctx<NW, RAD>& k, const Taps& tp, Strip2State<RAD>& st,
                                            int S)
{
    constexpr int NR = 2 * RAD + 1;
    constexpr int D = 3 * RAD + 2;
    constexpr int NH = 16;
    // ---- stage 1, before the barrier: prefetch, gathers, force of row y ----
    int nym = 0, nyc = 0, nyp = 0;
    float n_rm = 0.0f, n_rc = 0.0f, n_rp = 0.0f, ux2 = 0.0f, uy2 = 0.0f;
    Bilin g1 = st.g;
    if constexpr (DO1) {
        const int y = k.y0 - 2 * RAD + S;
        nyc = k.rowc(y + 1);
        nym = max(nyc - 1, 0);
        nyp = min(nyc + 1, k.h - 1);
        const int yc2 = k.rowc(y + 2);
        n_rp = bload_s(k.R, k.x4, (unsigned)nyp * k.uw4);
        ux2 = bload_s(k.U, k.x4, (unsigned)yc2 * k.uw4);
        uy2 = bload_s(k.U, k.x4, k.ch1 + (unsigned)yc2 * k.uw4);
        g1 = bilinear_issue_g(k.T, k.gg, (float)k.x + st.ux1, (float)nyc + st.uy1);
        n_rm = (nym == st.yc) ? st.r_c : (nym == st.yp ? st.r_p : st.r_m);
        n_rc = (nyc == st.yp) ? st.r_p : st.r_c;
        const float wv = bilinear_blend_g(st.g);
        const float sy = (st.yp - st.ym == 2) ? 0.5f : 1.0f;
        const float gyr = (st.r_p - st.r_m) * sy;
        const float gxr = (lds_at<float>(k.L1->r, st.cur1.r + 8u) - lds_at<float>(k.L1->r, st.cur1.r)) * k.sx;
        const float a = st.r_c - wv;
        const float den = fmaf(gxr, gxr, fmaf(gyr, gyr, a * a));
        float vx = st.ux, vy = st.uy;
        if (den > 1e-9f) {
            const float q = a * __builtin_amdgcn_rcpf(den);
            vx = fmaf(q, gxr, st.ux);
            vy = fmaf(q, gyr, st.uy);
        }
        put_v<RAD>(k.L1->v, st.cur1.v, k.gx, k.w, vx, vy);
        put_r(k.L1->r, st.oth1.r, k.gx, k.w, n_rc);
        st.ring_ux[SL1] = st.ux;
        st.ring_uy[SL1] = st.uy;
    }
    // ---- stage 2, before the barrier ----
    if constexpr (INIT2) {  // u1 and gathers of stage 2's first input row
        const int r0 = k.rowc(k.y0 - RAD);
        const float2 v1 = k.hist[r0 & (NH - 1)][k.c];
        st.v1x = v1.x;
        st.v1y = v1.y;
        st.g2 = bilinear_issue_g(k.T, k.gg, (float)k.x + st.v1x, (float)r0 + st.v1y);
    }
    int nzm = 0, nzc = 0, nzp = 0;
    float n_qm = 0.0f, n_qc = 0.0f, n_qp = 0.0f, v1x_n = 0.0f, v1y_n = 0.0f;
    Bilin g2n = st.g2;
    if constexpr (DO2) {
        const int y2 = k.y0 - RAD + (S - D);
        nzc = k.rowc(y2 + 1);
        nzm = max(nzc - 1, 0);
        nzp = min(nzc + 1, k.h - 1);
        const float2 v1 = k.hist[nzc & (NH - 1)][k.c];
        v1x_n = v1.x;
        v1y_n = v1.y;
        g2n = bilinear_issue_g(k.T, k.gg, (float)k.x + v1x_n, (float)nzc + v1y_n);
        n_qp = bload_s(k.R, k.x4, (unsigned)nzp * k.uw4);
        n_qm = (nzm == st.zc) ? st.q_c : (nzm == st.zp ? st.q_p : st.q_m);
        n_qc = (nzc == st.zp) ? st.q_p : st.q_c;
        const float wv = bilinear_blend_g(st.g2);
        const float sy = (st.zp - st.zm == 2) ? 0.5f : 1.0f;
        const float gyr = (st.q_p - st.q_m) * sy;
        const float gxr = (lds_at<float>(k.L2->r, st.cur2.r + 8u) - lds_at<float>(k.L2->r, st.cur2.r)) * k.sx;
        const float a = st.q_c - wv;
        const float den = fmaf(gxr, gxr, fmaf(gyr, gyr, a * a));
        float vx = st.v1x, vy = st.v1y;
        if (den > 1e-9f) {
            const float q = a * __builtin_amdgcn_rcpf(den);
            vx = fmaf(q, gxr, st.v1x);
            vy = fmaf(q, gyr, st.v1y);
        }
        put_v<RAD>(k.L2->v, st.cur2.v, k.gx, k.w, vx, vy);
        put_r(k.L2->r, st.oth2.r, k.gx, k.w, n_qc);
    }
    __syncthreads();
    // ---- stage 1, after the barrier: taps, u1 row y - r into the history ----
    if constexpr (DO1) {
        taps_h<RAD>(k.L1->v, st.cur1.v, tp, st.ring_x[SL1], st.ring_y[SL1]);
        if constexpr (OUT1) {
            const int yo = k.y0 - 3 * RAD + S;
            if (yo >= 0 && yo < k.h) {
                float ox = 0.0f, oy = 0.0f;
#pragma unroll
                for (int j = 0; j <= 2 * RAD; j++) {
                    ox = fmaf(tp.w[j], st.ring_x[(SL1 + 1 + j) % NR], ox);
                    oy = fmaf(tp.w[j], st.ring_y[(SL1 + 1 + j) % NR], oy);
                }
                k.hist[yo & (NH - 1)][k.c] = make_float2(ox, oy);
                if (k.want_ss && k.in && yo >= k.y0 && yo < k.y0 + TY) {
                    constexpr int us = (SL1 + RAD + 1) % NR;
                    const float dx = ox - st.ring_ux[us], dy = oy - st.ring_uy[us];
                    st.ss1 = fmaf(dx, dx, fmaf(dy, dy, st.ss1));
                }
            }
        }
        st.r_m = n_rm;
        st.r_c = n_rc;
        st.r_p = n_rp;
        st.ux = st.ux1;
        st.uy = st.uy1;
        st.ux1 = ux2;
        st.uy1 = uy2;
        st.g = g1;
        st.ym = nym;
        st.yc = nyc;
        st.yp = nyp;
    }
    // ---- stage 2, after the barrier: taps, u2 of row y2 - r ----
    if constexpr (DO2) {
        taps_h<RAD>(k.L2->v, st.cur2.v, tp, st.ring2_x[SL2], st.ring2_y[SL2]);
        if constexpr (OUT2) {
            const int yo = k.y0 - 2 * RAD + (S - D);
            if (yo < k.h && k.in) {
                float ox = 0.0f, oy = 0.0f;
#pragma unroll
                for (int j = 0; j <= 2 * RAD; j++) {
                    ox = fmaf(tp.w[j], st.ring2_x[(SL2 + 1 + j) % NR], ox);
                    oy = fmaf(tp.w[j], st.ring2_y[(SL2 + 1 + j) % NR], oy);
                }
                if (k.want_ss) {
                    const float2 u1 = k.hist[yo & (NH - 1)][k.c];
                    const float dx = ox - u1.x;
                    const float dy = oy - u1.y;
                    st.ss2 = fmaf(dx, dx, fmaf(dy, dy, st.ss2));
                }
                const unsigned o = (unsigned)yo * k.uw4;
                bstore_s(k.UN, k.x4, o, ox);
                bstore_s(k.UN, k.x4, k.ch1 + o, oy);
            }
        }
        st.q_m = n_qm;
        st.q_c = n_qc;
        st.q_p = n_qp;
        st.v1x = v1x_n;
        st.v1y = v1y_n;
        st.g2 = g2n;
        st.zm = nzm;
        st.zc = nzc;
        st.zp = nzp;
    }
    RowBase t = st.cur1;
    st.cur1 = st.oth1;
    st.oth1 = t;
    t = st.cur2;
    st.cur2 = st.oth2;
    st.oth2 = t;
}

template <int NW, int RAD, int TY>
__device__ float2 demons_strip2(const float* __restrict__ Rg, const float* __restrict__ Tg,
                                const float* __restrict__ ug, float* __restrict__ ung, int h, int w,
                                int y0, int sx0, int ws, int we, const Taps& tp, bool want_ss)
{
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
    static_assert(S1 - D >= NR, "strip too short for the two-stage march");
    __shared__ StripRows<NW, RAD> L1, L2;
    __shared__ float2 hist[NH][RW];
    __shared__ float red[2][NW];
    Strip2Ctx<NW, RAD> k;
    const unsigned img_bytes = 4u * (unsigned)h * (unsigned)w;
    k.R = make_rsrc(Rg, img_bytes);
    k.T = make_rsrc(Tg, img_bytes);
    k.U = make_rsrc(ug, 2u * img_bytes);
    k.UN = make_rsrc(ung, 2u * img_bytes);
    k.c = threadIdx.x;
    k.gx = sx0 + k.c;  // the lane's column; written when inside [ws, we)
    k.in = k.gx >= ws && k.gx < we;
    k.x = clampi(k.gx, 0, w - 1);
    k.h = h;
    k.w = w;
    k.y0 = y0;
    k.want_ss = want_ss;
    const int xm = max(k.x - 1, 0), xp = min(k.x + 1, w - 1);
    k.sx = (xp - xm == 2) ? 0.5f : 1.0f;
    k.gg = bil_geom(h, w);
    k.uw4 = 4u * (unsigned)w;
    k.x4 = 4u * (unsigned)k.x;
    k.ch1 = img_bytes;
    k.L1 = &L1;
    k.L2 = &L2;
    k.hist = hist;

    Strip2State<RAD> st;
    // LDS bases: stage 1 uses parity S & 1 at step S, stage 2 parity (S - D) & 1
    row_bases<NW, RAD>(k.x - sx0, st.cur1, st.oth1);
    if (D & 1) row_bases<NW, RAD>(k.x - sx0, st.oth2, st.cur2);
    else row_bases<NW, RAD>(k.x - sx0, st.cur2, st.oth2);
    const unsigned uw4 = k.uw4, x4 = k.x4, ch1 = k.ch1;
    // stage 1 pipeline state (as in demons_strip), starting at input row y0 - 2r
    st.yc = k.rowc(y0 - 2 * RAD);
    st.ym = max(st.yc - 1, 0);
    st.yp = min(st.yc + 1, h - 1);
    st.r_m = bload_s(k.R, x4, (unsigned)st.ym * uw4);
    st.r_c = bload_s(k.R, x4, (unsigned)st.yc * uw4);
    st.r_p = bload_s(k.R, x4, (unsigned)st.yp * uw4);
    st.ux = bload_s(k.U, x4, (unsigned)st.yc * uw4);
    st.uy = bload_s(k.U, x4, ch1 + (unsigned)st.yc * uw4);
    const int yc1 = k.rowc(y0 - 2 * RAD + 1);
    st.ux1 = bload_s(k.U, x4, (unsigned)yc1 * uw4);
    st.uy1 = bload_s(k.U, x4, ch1 + (unsigned)yc1 * uw4);
    st.g = bilinear_issue_g(k.T, k.gg, (float)k.x + st.ux, (float)st.yc + st.uy);
    put_r(L1.r, st.cur1.r, k.gx, w, st.r_c);
    // stage 2 state: R rows of its first input row y0 - r; its u1 and gathers
    // are taken from the history one step before its first step
    st.zc = k.rowc(y0 - RAD);
    st.zm = max(st.zc - 1, 0);
    st.zp = min(st.zc + 1, h - 1);
    st.q_m = bload_s(k.R, x4, (unsigned)st.zm * uw4);
    st.q_c = bload_s(k.R, x4, (unsigned)st.zc * uw4);
    st.q_p = bload_s(k.R, x4, (unsigned)st.zp * uw4);
    put_r(L2.r, (D & 1) ? st.oth2.r : st.cur2.r, k.gx, w, st.q_c);  // parity 0 of stage 2
    st.v1x = st.v1y = 0.0f;
    st.g2 = st.g;
    st.ss1 = st.ss2 = 0.0f;
    __syncthreads();

    // phase A: steps 0 .. D-1, stage 1 only
    static_for<0, D>([&](auto ic) {
        constexpr int S = decltype(ic)::value;
        strip2_step<NW, RAD, TY, S % NR, 0, true, false, (S >= 2 * RAD), false, (S == D - 1)>(k, tp, st, S);
    });
    // phase B: steps D .. S1-1, both stages; the first NR steps (stage 2's
    // ring filling), then whole groups of NR, then the remainder
    static_for<0, NR>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        strip2_step<NW, RAD, TY, (D + i) % NR, i, true, true, true, (i >= 2 * RAD), false>(k, tp, st, D + i);
    });
    constexpr int QB = (S1 - D) / NR, RB = (S1 - D) % NR;
#pragma unroll 1
    for (int m = 1; m < QB; m++) {
        static_for<0, NR>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            strip2_step<NW, RAD, TY, (D + i) % NR, i, true, true, true, true, false>(k, tp, st, D + NR * m + i);
        });
    }
    static_for<0, RB>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        strip2_step<NW, RAD, TY, (D + i) % NR, i, true, true, true, true, false>(k, tp, st, D + NR * QB + i);
    });
    // phase C: steps S1 .. STEPS-1, stage 2 only
    static_for<0, STEPS - S1>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        strip2_step<NW, RAD, TY, 0, (S1 - D + i) % NR, false, true, false, true, false>(k, tp, st, S1 + i);
    });

    float ss1 = st.ss1, ss2 = st.ss2;
    const int c = k.c;
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

// SEG: the level is cut into column segments (levels wider than 64 NW px);
// without it nsegs is 1 and every lane's column is its index.
template <int NW, int RAD, int TY, bool SEG>
__global__ void __launch_bounds__(64 * NW)
    k_demons_rows(const Bucket* __restrict__ bk, int level, int k, Taps tp, float tol, int nstrips, int nsegs_arg)
{
    __shared__ double sh_sum;
    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int nsegs = SEG ? nsegs_arg : 1;
    const int nunits = nstrips * nsegs;  // units of a pair: strips x column segments
    const int b = lb / nunits;
    const int unit = lb - b * nunits;
    const int strip = unit / nsegs, seg = unit - strip * nsegs;
    const PairState st = bk->state[b];
    if (st.stop >= 0) return;  // uniform
    const int h = bk->lh[level], w = bk->lw[level];
    const int64_t npart = (int64_t)bk->nb * bk->max_tiles;
    if (tol > 0.0f && k > 0) {
        const float* prev = bk->partial + ((k - 1) & 1) * npart + (int64_t)b * bk->max_tiles;
        const double ss = pair_sum(prev, nunits, &sh_sum);
        const double delta = sqrt(ss / ((double)h * (double)w)) * (double)(1 << level);
        if (delta < (double)tol) {
            if (unit == 0 && threadIdx.x == 0) {
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
    int sx0 = 0, ws = 0, we = w;
    if constexpr (SEG) rows_seg_cols(seg, nsegs, w, NW, sx0, ws, we);
    const float ss = demons_strip<NW, RAD, TY>(R, T, u, un, h, w, strip * TY, sx0, ws, we, tp, tol > 0.0f);
    if (tol > 0.0f && threadIdx.x == 0)
        bk->partial[(k & 1) * npart + (int64_t)b * bk->max_tiles + unit] = ss;
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
template <int NW, int RAD, int TY, bool SEG>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(3)))
    k_demons_rows2(const Bucket* __restrict__ bk, int level, int L, Taps tp, float tol, int nstrips, int nsegs_arg,
                   int cap)
{
    __shared__ double sh_sum;
    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int nsegs = SEG ? nsegs_arg : 1;
    const int nunits = nstrips * nsegs;  // units of a pair: strips x column segments
    const int b = lb / nunits;
    const int unit = lb - b * nunits;
    const int strip = unit / nsegs, seg = unit - strip * nsegs;
    const PairState st = bk->state[b];
    const int k = 2 * L;
    // A stop at k - 1 can only have been written by unit 0 of this launch
    // (earlier launches record stops at most k - 2); the other units of the
    // pair still owe the recompute of their strips below, and each reaches
    // that decision again from the same partial sums.  Any unit may start
    // after unit 0 has written the state when the grid exceeds one dispatch
    // wave, so the early exit must not take that stop.
    if (st.stop >= 0 && st.stop != k - 1) return;  // uniform
    const int h = bk->lh[level], w = bk->lw[level];
    const int64_t npart = (int64_t)bk->nb * bk->max_tiles;
    const int64_t pofs = (int64_t)b * bk->max_tiles;
    bool recompute = false;
    if (tol > 0.0f && L > 0) {
        const double hw = (double)h * (double)w, sc = (double)(1 << level);
        const double ssa = pair_sum(bk->partial + ((k - 2) & 3) * npart + pofs, nunits, &sh_sum);
        if (sqrt(ssa / hw) * sc < (double)tol) {
            recompute = true;
        } else {
            const double ssb = pair_sum(bk->partial + ((k - 1) & 3) * npart + pofs, nunits, &sh_sum);
            if (sqrt(ssb / hw) * sc < (double)tol) {
                if (unit == 0 && threadIdx.x == 0) {
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
    int sx0 = 0, ws = 0, we = w;
    if constexpr (SEG) rows_seg_cols(seg, nsegs, w, NW, sx0, ws, we);
    if (recompute) {
        if (unit == 0 && threadIdx.x == 0) {
            bk->state[b].stop = k - 1;
            bk->state[b].convmask = st.convmask | (1u << level);
        }
        demons_strip<NW, RAD, TY>(R, T, fb, fa, h, w, strip * TY, sx0, ws, we, tp, false);
        return;
    }
    if (k >= cap) return;
    if (k + 1 < cap) {
        const float2 ss = demons_strip2<NW, RAD, TY>(R, T, fa, fb, h, w, strip * TY, sx0, ws, we, tp, tol > 0.0f);
        if (tol > 0.0f && threadIdx.x == 0) {
            bk->partial[(k & 3) * npart + pofs + unit] = ss.x;
            bk->partial[((k + 1) & 3) * npart + pofs + unit] = ss.y;
        }
    } else {
        const float ss = demons_strip<NW, RAD, TY>(R, T, fa, fb, h, w, strip * TY, sx0, ws, we, tp, tol > 0.0f);
        if (tol > 0.0f && threadIdx.x == 0) bk->partial[(k & 3) * npart + pofs + unit] = ss;
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
                                                  un + 2 * b * hw, h, w, y0, 0, 0, w, tp, true);
    if (rms && threadIdx.x == 0) rms[b] = sqrt(acc / (double)hw);
}

template <int CPL, int RAD, int TY>
void launch_rows(const Bucket* d_bk, int nb, int h, int w, int level, int k, const Taps& tp, float tol,
                 hipStream_t s)
{
    const int nstrips = (h + TY - 1) / TY, nsegs = rows_segs(w, CPL);
    if constexpr (CPL >= 4) {
        if (nsegs > 1) {
            hipLaunchKernelGGL((k_demons_rows<CPL, RAD, TY, true>), dim3(nb * nstrips * nsegs), dim3(64 * CPL), 0,
                               s, d_bk, level, k, tp, tol, nstrips, nsegs);
            return;
        }
    }
    hipLaunchKernelGGL((k_demons_rows<CPL, RAD, TY, false>), dim3(nb * nstrips), dim3(64 * CPL), 0, s, d_bk,
                       level, k, tp, tol, nstrips, 1);
}

template <int CPL, int RAD>
bool dispatch_ty(const Bucket* d_bk, int nb, int h, int w, int level, int k, const Taps& tp, float tol,
                 int ty, hipStream_t s)
{
    switch (ty) {
    case 16: launch_rows<CPL, RAD, 16>(d_bk, nb, h, w, level, k, tp, tol, s); return true;
    case 32: launch_rows<CPL, RAD, 32>(d_bk, nb, h, w, level, k, tp, tol, s); return true;
    case 64: launch_rows<CPL, RAD, 64>(d_bk, nb, h, w, level, k, tp, tol, s); return true;
    case 128: launch_rows<CPL, RAD, 128>(d_bk, nb, h, w, level, k, tp, tol, s); return true;
    default: return false;
    }
}

template <int CPL>
bool dispatch_rad(const Bucket* d_bk, int nb, int h, int w, int level, int k, const Taps& tp, int radius,
                  float tol, int ty, hipStream_t s)
{
    switch (radius) {
    case 0: return dispatch_ty<CPL, 0>(d_bk, nb, h, w, level, k, tp, tol, ty, s);
    case 1: return dispatch_ty<CPL, 1>(d_bk, nb, h, w, level, k, tp, tol, ty, s);
    case 2: return dispatch_ty<CPL, 2>(d_bk, nb, h, w, level, k, tp, tol, ty, s);
    case 3: return dispatch_ty<CPL, 3>(d_bk, nb, h, w, level, k, tp, tol, ty, s);
    case 4: return dispatch_ty<CPL, 4>(d_bk, nb, h, w, level, k, tp, tol, ty, s);
    default: return false;
    }
}

template <int CPL, int RAD, int TY>
void launch_rows2(const Bucket* d_bk, int nb, int h, int w, int level, int L, const Taps& tp, float tol, int cap,
                  hipStream_t s)
{
    const int nstrips = (h + TY - 1) / TY, nsegs = rows_segs(w, CPL);
    if constexpr (CPL >= 4) {
        if (nsegs > 1) {
            hipLaunchKernelGGL((k_demons_rows2<CPL, RAD, TY, true>), dim3(nb * nstrips * nsegs), dim3(64 * CPL), 0,
                               s, d_bk, level, L, tp, tol, nstrips, nsegs, cap);
            return;
        }
    }
    hipLaunchKernelGGL((k_demons_rows2<CPL, RAD, TY, false>), dim3(nb * nstrips), dim3(64 * CPL), 0, s, d_bk,
                       level, L, tp, tol, nstrips, 1, cap);
}

template <int CPL, int RAD>
bool dispatch_ty2(const Bucket* d_bk, int nb, int h, int w, int level, int L, const Taps& tp, float tol, int cap, int ty,
                  hipStream_t s)
{
    switch (ty) {
    case 8:  // rows of at most 128 px only (a single small pair's latency)
        if constexpr (CPL <= 2) {
            launch_rows2<CPL, RAD, 8>(d_bk, nb, h, w, level, L, tp, tol, cap, s);
            return true;
        }
        return false;
    case 16: launch_rows2<CPL, RAD, 16>(d_bk, nb, h, w, level, L, tp, tol, cap, s); return true;
    case 32: launch_rows2<CPL, RAD, 32>(d_bk, nb, h, w, level, L, tp, tol, cap, s); return true;
    case 64: launch_rows2<CPL, RAD, 64>(d_bk, nb, h, w, level, L, tp, tol, cap, s); return true;
    case 128: launch_rows2<CPL, RAD, 128>(d_bk, nb, h, w, level, L, tp, tol, cap, s); return true;
    default: return false;
    }
}

template <int CPL>
bool dispatch_rad2(const Bucket* d_bk, int nb, int h, int w, int level, int L, const Taps& tp, int radius, float tol,
                   int cap, int ty, hipStream_t s)
{
    switch (radius) {
    case 0: return dispatch_ty2<CPL, 0>(d_bk, nb, h, w, level, L, tp, tol, cap, ty, s);
    case 1: return dispatch_ty2<CPL, 1>(d_bk, nb, h, w, level, L, tp, tol, cap, ty, s);
    case 2: return dispatch_ty2<CPL, 2>(d_bk, nb, h, w, level, L, tp, tol, cap, ty, s);
    case 3: return dispatch_ty2<CPL, 3>(d_bk, nb, h, w, level, L, tp, tol, cap, ty, s);
    case 4: return dispatch_ty2<CPL, 4>(d_bk, nb, h, w, level, L, tp, tol, cap, ty, s);
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

}  // namespace ebsd
