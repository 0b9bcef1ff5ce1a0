// Kernels of the warm-start network: 3x3 convolutions and their weight
// gradients on the gfx950 matrix cores (bf16 operands, fp32 accumulation,
// v_mfma_f32_32x32x16_bf16), and the element-wise passes between them.
//
// Matrix-core operand layout of the 32x32x16 bf16 instruction (wave64): lane l
// supplies row l % 32 of A with the 8 consecutive k values 8 (l / 32) .. +7,
// and column l % 32 of B with the same 8 k values; it receives the 16
// accumulator values C[8 (i / 4) + 4 (l / 32) + i % 4][l % 32], i = 0..15.
#include "cnn_internal.h"
#include "dev_util.h"

#include "../../include/ebsd.h"

namespace ebsd {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(uint16_t)))) uint16_t u16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

__device__ inline bf16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
    return (bf16_t)(u >> 16);
}

__device__ inline float bf2f(bf16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ inline f32x16 mfma16(const bf16x8& a, const bf16x8& b, const f32x16& c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// ---- 3x3 convolution (forward and input gradient) ------------------------------
//
// Workgroup: 4 waves, output tile of 8 rows x 32 columns x (32 NT) channels;
// wave w computes rows 2w, 2w+1 (one 32-pixel M tile each) for all NT N tiles.
// For each chunk of CK input channels the (8+2) x (32+2) input halo and the
// 9 taps of weights are staged in LDS (the next chunk's global loads are in
// flight during the current chunk's matrix-core loop); the K loop walks
// (tap, 8-channel group) pairs, two per 16-wide MFMA step (one per half wave).  Pixel rows in LDS are
// padded to 80 bytes for CK = 32 so that 8 consecutive lanes of a 16-byte read
// cover all banks.
constexpr int kConvTH = 8, kConvTW = 32;

template <int CK, int NT, bool UP = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_conv3x3(ConvArgs a)
{
    constexpr int HP = kConvTH + 2, WP = kConvTW + 2;
    constexpr int PS = (CK == 32) ? 40 : CK;
    constexpr int BN = 32 * NT;
    constexpr int G = CK / 8;
    constexpr int NF = 9 * G;
    constexpr int NS = (NF + 1) / 2;
    // LDS: the input halo (sA) and the weights (sB) during the K loop; the
    // output tile of each wave afterwards (transposed so that every lane
    // stores whole 16-byte groups of channels).
    constexpr int SA = HP * WP * PS, SB = 9 * BN * PS;
    constexpr int ST0 = 4 * 64 * (BN + 8) * 2;  // bf16 output tiles, bytes
    constexpr int ST1 = 4 * 32 * (BN + 4) * 4;  // fp32 output half tiles, bytes
    constexpr int SMEM0 = 2 * (SA + SB);
    constexpr int SMEM = SMEM0 > ST0 ? (SMEM0 > ST1 ? SMEM0 : ST1) : (ST0 > ST1 ? ST0 : ST1);
    __shared__ __attribute__((aligned(16))) char smem[SMEM];
    bf16_t* const sA = reinterpret_cast<bf16_t*>(smem);
    bf16_t* const sB = sA + SA;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, l32 = lane & 31;
    int b = blockIdx.x;
    const int nbk = a.Cout / BN, txn = a.W / kConvTW, tyn = a.H / kConvTH;
    const int nb = b % nbk;
    b /= nbk;
    const int tx = b % txn;
    b /= txn;
    const int ty = b % tyn;
    const int img = b / tyn;
    const int x0 = tx * kConvTW, y0 = ty * kConvTH, co0 = nb * BN;
    const int Cin = a.Cin;
    const bf16_t* __restrict__ xin = a.x + (int64_t)img * a.H * a.W * Cin;
    const bf16_t* __restrict__ x2in = UP ? a.x2 + (int64_t)img * (a.H >> 1) * (a.W >> 1) * a.c2 : nullptr;

    f32x16 acc[2][NT];
    for (int r = 0; r < 2; r++)
        for (int j = 0; j < NT; j++)
            for (int i = 0; i < 16; i++) acc[r][j][i] = 0.0f;

    // Global loads of the next chunk are issued before the current chunk's
    // matrix-core loop and written to LDS after it (registers pa, pb).
    constexpr int NA_TOT = HP * WP * G, NB_TOT = 9 * BN * G;
    constexpr int NA = (NA_TOT + 255) / 256, NB = (NB_TOT + 255) / 256;
    static_assert(NA <= 32, "halo mask");
    uint4 pa[NA], pb[NB];
    uint32_t amask = 0;  // bit k: pa[k] lies inside the image (else the halo value is zero)
    // Halo loads without branches (addresses clamped into the image; the zero of the padding
    // is selected when the chunk is stored): with the loads under branches the compiler waited
    // for them in the middle of the prefetch, before the current chunk's matrix-core loop.
    auto fetch = [&](int c0) {
        amask = 0;
        const bool up = UP && c0 < a.c2;  // uniform: the chunk lies in the upsampled source
#pragma unroll
        for (int k = 0; k < NA; k++) {
            const int i = min(tid + 256 * k, NA_TOT - 1);
            const int g = i % G, p = i / G;
            const int hx = p % WP, hy = p / WP;
            const int yy = y0 + hy - 1, xx = x0 + hx - 1;
            const bool in = yy >= 0 && yy < a.H && xx >= 0 && xx < a.W;
            const int yc = min(max(yy, 0), a.H - 1), xc = min(max(xx, 0), a.W - 1);
            const bf16_t* src = up ? x2in + ((int64_t)(yc >> 1) * (a.W >> 1) + (xc >> 1)) * a.c2
                                   : xin + ((int64_t)yc * a.W + xc) * Cin;
            pa[k] = *reinterpret_cast<const uint4*>(src + c0 + 8 * g);
            amask |= (in ? 1u : 0u) << k;
        }
#pragma unroll
        for (int k = 0; k < NB; k++) {
            // (a guarded load here: the clamped form makes the compiler keep pb in scratch)
            const int i = tid + 256 * k;
            const int g = i % G, r = i / G;
            const int co = r % BN, t = r / BN;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (i < NB_TOT)
                v = *reinterpret_cast<const uint4*>(a.w + ((int64_t)(co0 + co) * 9 + t) * Cin + c0 + 8 * g);
            pb[k] = v;
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int k = 0; k < NA; k++) {
            const int i = tid + 256 * k;
            const uint4 v = (amask >> k) & 1u ? pa[k] : make_uint4(0u, 0u, 0u, 0u);
            if (i < NA_TOT) *reinterpret_cast<uint4*>(sA + (i / G) * PS + 8 * (i % G)) = v;
        }
#pragma unroll
        for (int k = 0; k < NB; k++) {
            const int i = tid + 256 * k;
            if (i < NB_TOT) {
                const int g = i % G, r = i / G;
                *reinterpret_cast<uint4*>(sB + ((r / BN) * BN + r % BN) * PS + 8 * g) = pb[k];
            }
        }
    };
    fetch(0);
    stash();
    __syncthreads();
    for (int c0 = 0; c0 < Cin; c0 += CK) {
        const bool next = c0 + CK < Cin;
        if (next) fetch(c0 + CK);
        for (int s = 0; s < NS; s++) {
            const int f = 2 * s + h;
            const bool valid = f < NF;  // false only for the padding group of an odd group count
            const int fc = valid ? f : 0;
            const int t = fc / G, g = fc - G * (fc / G);
            const int ky = t / 3, kx = t - 3 * (t / 3);
            bf16x8 av[2], bv[NT];
            for (int r = 0; r < 2; r++) {
                const int row = 2 * wave + r;
                av[r] = *reinterpret_cast<const bf16x8*>(sA + ((row + ky) * WP + l32 + kx) * PS + 8 * g);
            }
            for (int j = 0; j < NT; j++) {
                u16x8 raw = *reinterpret_cast<const u16x8*>(sB + (t * BN + 32 * j + l32) * PS + 8 * g);
                if (!valid) raw = (u16x8){0, 0, 0, 0, 0, 0, 0, 0};
                bv[j] = __builtin_bit_cast(bf16x8, raw);
            }
            for (int r = 0; r < 2; r++)
                for (int j = 0; j < NT; j++) acc[r][j] = mfma16(av[r], bv[j], acc[r][j]);
        }
        __syncthreads();
        if (next) {
            stash();
            __syncthreads();
        }
    }

    // epilogue (the K loop ended with a barrier: LDS is free)
    if (a.mode != 1) {
        constexpr int RP = BN + 8;  // staging row pitch (bf16)
        bf16_t* stg = reinterpret_cast<bf16_t*>(smem) + wave * 64 * RP;
        for (int j = 0; j < NT; j++) {
            const int col = 32 * j + l32;
            const float bias = a.bias[co0 + col];
            for (int r = 0; r < 2; r++)
                for (int i = 0; i < 16; i++) {
                    const int px = 32 * r + 8 * (i >> 2) + 4 * h + (i & 3);
                    stg[px * RP + col] = f2bf(fmaxf(acc[r][j][i] + bias, 0.0f));
                }
        }
        __syncthreads();
        bf16_t* out = static_cast<bf16_t*>(a.out);
        if (a.mode != 2) {
            for (int v = lane; v < 64 * (BN / 8); v += 64) {
                const int px = v / (BN / 8), g = v - (BN / 8) * (v / (BN / 8));
                const int yy = y0 + 2 * wave + (px >> 5), xx = x0 + (px & 31);
                const int64_t p = ((int64_t)img * a.H + yy) * a.W + xx;
                *reinterpret_cast<uint4*>(out + p * a.out_cs + a.out_co + co0 + 8 * g) =
                    *reinterpret_cast<const uint4*>(stg + px * RP + 8 * g);
            }
        }
        if (a.mode != 0) {
            // 2 x 2 max-pool of the wave's two rows (the selection of k_maxpool: first
            // of the largest in the order (0,0), (0,1), (1,0), (1,1)) into the
            // half-size output, pooled row y0 / 2 + wave, columns x0 / 2 .. + 15
            // (mode 3: into out2, channels from 0)
            bf16_t* const pout = a.mode == 3 ? a.out2 : out;
            const int pcs = a.mode == 3 ? a.out2_cs : a.out_cs, pco = a.mode == 3 ? 0 : a.out_co;
            const int Hp = a.H / 2, Wp = a.W / 2;
            for (int v = lane; v < 16 * (BN / 8); v += 64) {
                const int q = v / (BN / 8), g = v - (BN / 8) * (v / (BN / 8));
                const bf16_t* s0 = stg + (2 * q) * RP + 8 * g;
                const bf16_t* s1 = s0 + RP;
                const bf16_t* s2 = s0 + 32 * RP;
                const bf16_t* s3 = s2 + RP;
                u16x8 o;
                for (int e = 0; e < 8; e++) {
                    uint16_t m = s0[e];
                    if (bf2f(s1[e]) > bf2f(m)) m = s1[e];
                    if (bf2f(s2[e]) > bf2f(m)) m = s2[e];
                    if (bf2f(s3[e]) > bf2f(m)) m = s3[e];
                    o[e] = m;
                }
                const int64_t p = ((int64_t)img * Hp + (y0 >> 1) + wave) * Wp + (x0 >> 1) + q;
                *reinterpret_cast<u16x8*>(pout + p * pcs + pco + co0 + 8 * g) = o;
            }
        }
    } else {
        constexpr int RP = BN + 4;  // staging row pitch (fp32)
        float* stg = reinterpret_cast<float*>(smem) + wave * 32 * RP;
        float* out = static_cast<float*>(a.out);
        for (int r = 0; r < 2; r++) {
            for (int j = 0; j < NT; j++)
                for (int i = 0; i < 16; i++) {
                    const int px = 8 * (i >> 2) + 4 * h + (i & 3);
                    stg[px * RP + 32 * j + l32] = acc[r][j][i];
                }
            __syncthreads();
            const int yy = y0 + 2 * wave + r;
            for (int v = lane; v < 32 * (BN / 4); v += 64) {
                const int px = v / (BN / 4), g = v - (BN / 4) * (v / (BN / 4));
                const int64_t p = ((int64_t)img * a.H + yy) * a.W + x0 + px;
                *reinterpret_cast<float4*>(out + p * a.out_cs + a.out_co + co0 + 4 * g) =
                    *reinterpret_cast<const float4*>(stg + px * RP + 4 * g);
            }
            __syncthreads();
        }
    }
}

// 16 bytes per lane from a buffer resource into LDS at dst + 16 * lane (dst
// wave-uniform); offsets past the resource's end deliver zeros.  (Kept out of the
// kernel templates: called from a template body directly, the builtin makes the
// host pass drop the kernel's launch stub.)
typedef __attribute__((address_space(3))) char lds_char;
__device__ inline void lds_load16(__amdgpu_buffer_rsrc_t r, lds_char* dst, unsigned voff, unsigned soff)
{
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void*)dst, 16, voff, soff, 0, 0);
}

// Inference variant of k_conv3x3<32, NT, UP> with the input chunks moved into
// LDS by the buffer unit (buffer_load_dwordx4 ... lds): no staging registers
// and no store phase, two LDS buffers so that chunk c + 1 loads while chunk c
// is multiplied, one barrier per chunk.  16 x 32 output pixels per workgroup of
// 8 waves (wave w on rows 2w, 2w + 1), one workgroup per CU (2 x 74 KiB of
// buffers).  The K loop is k_conv3x3's for CK = 32 (the same products in the
// same order), so the outputs are equal bit for bit.  A pixel's (or a weight
// row's) four 16-byte quarters sit in LDS rotated by bits 2..3 of its index
// (16-byte slot 4p + (g ^ ((p >> 2) & 3))), so that the 16-byte reads of 16
// consecutive lanes fall in 16 different 16-byte groups of the 256 bytes the
// LDS serves per cycle (rotating by bits 1..2 left pixels p and p + 8 in the
// same group: twice the bank-conflict cycles, measured); each lane's buffer
// load fetches the quarter that lands in its slot (the buffer unit writes lane
// l's 16 bytes at the instruction's LDS base + 16 l).  Halo pixels outside the
// image get an offset past the end of the resource, which reads as zeros.
constexpr int kLdsTH = 16;

template <int NT, bool UP>
__global__ void __launch_bounds__(512) k_conv3x3_lds(ConvArgs a)
{
    constexpr int HP = kLdsTH + 2, WP = kConvTW + 2;
    constexpr int BN = 32 * NT;
    constexpr int G = 4;              // 8-channel groups of a 32-channel chunk
    constexpr int NA = HP * WP * G;   // 16-byte pieces of a chunk's halo
    constexpr int NB = 9 * BN * G;    // and of its weights
    constexpr int KA = (NA + 511) / 512, KB = (NB + 511) / 512;
    constexpr int BUF = (NA + NB) * 16;  // bytes of one buffer
    constexpr int RP = BN + 8;           // epilogue staging row pitch (bf16)
    constexpr int ST = 8 * 64 * RP * 2;
    constexpr int SMEM = 2 * BUF > ST ? 2 * BUF : ST;
    __shared__ __attribute__((aligned(16))) char smem[SMEM];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, l32 = lane & 31;
    int b = blockIdx.x;
    const int nbk = a.Cout / BN, txn = a.W / kConvTW, tyn = a.H / kLdsTH;
    const int nb = b % nbk;
    b /= nbk;
    const int tx = b % txn;
    b /= txn;
    const int ty = b % tyn;
    const int img = b / tyn;
    const int x0 = tx * kConvTW, y0 = ty * kLdsTH, co0 = nb * BN;
    const int Cin = a.Cin;
    constexpr unsigned kOut = 0x80000000u;  // past the end of every resource: reads as zero
    const __amdgpu_buffer_rsrc_t rx =
        make_rsrc(a.x + (int64_t)img * a.H * a.W * Cin, 2u * (unsigned)a.H * (unsigned)a.W * (unsigned)Cin);
    const __amdgpu_buffer_rsrc_t rw = make_rsrc(a.w, 2u * (unsigned)a.Cout * 9u * (unsigned)Cin);
    __amdgpu_buffer_rsrc_t rx2 = rx;
    if constexpr (UP)
        rx2 = make_rsrc(a.x2 + (int64_t)img * (a.H >> 1) * (a.W >> 1) * a.c2,
                        2u * (unsigned)(a.H >> 1) * (unsigned)(a.W >> 1) * (unsigned)a.c2);

    // this thread's byte offsets of its pieces, before the chunk's channel offset
    unsigned oa[KA], oa2[KA], ob[KB];
#pragma unroll
    for (int k = 0; k < KA; k++) {
        const int i = k * 512 + tid;
        const int p = i >> 2, g = (i & 3) ^ ((p >> 2) & 3);
        const int hy = p / WP, hx = p - WP * (p / WP);
        const int yy = y0 + hy - 1, xx = x0 + hx - 1;
        const bool in = i < NA && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W;
        oa[k] = in ? 2u * ((unsigned)(yy * a.W + xx) * (unsigned)Cin + 8u * g) : kOut;
        oa2[k] = (UP && in) ? 2u * ((unsigned)((yy >> 1) * (a.W >> 1) + (xx >> 1)) * (unsigned)a.c2 + 8u * g)
                            : kOut;
    }
#pragma unroll
    for (int k = 0; k < KB; k++) {
        const int i = k * 512 + tid;
        const int r = i >> 2, g = (i & 3) ^ ((r >> 2) & 3);
        const int t = r / BN, co = r - BN * (r / BN);
        ob[k] = i < NB ? 2u * ((unsigned)((co0 + co) * 9 + t) * (unsigned)Cin + 8u * g) : kOut;
    }
    auto fetch = [&](int c0, int buf) {
        lds_char* base = (lds_char*)smem + buf * BUF;
        const bool up = UP && c0 < a.c2;  // uniform: the chunk lies in the upsampled source
        const unsigned so = 2u * (unsigned)c0;
#pragma unroll
        for (int k = 0; k < KA; k++) {
            if (k * 512 + wave * 64 >= NA) continue;  // uniform: nothing of this wave's block is needed
            lds_char* dst = base + (k * 512 + wave * 64) * 16;
            if (k * 512 + tid < NA) {
                if (up) lds_load16(rx2, dst, oa2[k], so);
                else lds_load16(rx, dst, oa[k], so);
            }
        }
#pragma unroll
        for (int k = 0; k < KB; k++) {
            if (k * 512 + wave * 64 >= NB) continue;
            lds_char* dst = base + NA * 16 + (k * 512 + wave * 64) * 16;
            if (k * 512 + tid < NB) lds_load16(rw, dst, ob[k], so);
        }
    };

    f32x16 acc[2][NT];
    for (int r = 0; r < 2; r++)
        for (int j = 0; j < NT; j++)
            for (int i = 0; i < 16; i++) acc[r][j][i] = 0.0f;

    const int nck = Cin / 32;
    fetch(0, 0);
    for (int c = 0; c < nck; c++) {
        __builtin_amdgcn_s_waitcnt(0);  // this thread's loads of chunk c are in LDS
        __syncthreads();                // everyone's, and chunk c - 1's buffer is free again
        if (c + 1 < nck) fetch(32 * (c + 1), (c + 1) & 1);
        const char* sA = smem + (c & 1) * BUF;
        const char* sB = sA + NA * 16;
        // k_conv3x3's K loop: step s takes (tap, group) pairs 2s (lanes 0..31) and 2s + 1 (32..63)
        for (int s = 0; s < 9 * G / 2; s++) {
            const int f = 2 * s + h;
            const int t = f / G, g = f - G * (f / G);
            const int ky = t / 3, kx = t - 3 * (t / 3);
            bf16x8 av[2], bv[NT];
            for (int r = 0; r < 2; r++) {
                const int p = (2 * wave + r + ky) * WP + l32 + kx;
                av[r] = *reinterpret_cast<const bf16x8*>(sA + (4 * p + (g ^ ((p >> 2) & 3))) * 16);
            }
            for (int j = 0; j < NT; j++) {
                const int rr = t * BN + 32 * j + l32;
                bv[j] = *reinterpret_cast<const bf16x8*>(sB + (4 * rr + (g ^ ((rr >> 2) & 3))) * 16);
            }
            for (int r = 0; r < 2; r++)
                for (int j = 0; j < NT; j++) acc[r][j] = mfma16(av[r], bv[j], acc[r][j]);
        }
    }
    __syncthreads();  // the buffers become the epilogue's staging area

    // epilogue of k_conv3x3 (modes 0, 2, 3)
    bf16_t* stg = reinterpret_cast<bf16_t*>(smem) + wave * 64 * RP;
    for (int j = 0; j < NT; j++) {
        const int col = 32 * j + l32;
        const float bias = a.bias[co0 + col];
        for (int r = 0; r < 2; r++)
            for (int i = 0; i < 16; i++) {
                const int px = 32 * r + 8 * (i >> 2) + 4 * h + (i & 3);
                stg[px * RP + col] = f2bf(fmaxf(acc[r][j][i] + bias, 0.0f));
            }
    }
    __syncthreads();
    bf16_t* out = static_cast<bf16_t*>(a.out);
    if (a.mode != 2) {
        for (int v = lane; v < 64 * (BN / 8); v += 64) {
            const int px = v / (BN / 8), g = v - (BN / 8) * (v / (BN / 8));
            const int yy = y0 + 2 * wave + (px >> 5), xx = x0 + (px & 31);
            const int64_t p = ((int64_t)img * a.H + yy) * a.W + xx;
            *reinterpret_cast<uint4*>(out + p * a.out_cs + a.out_co + co0 + 8 * g) =
                *reinterpret_cast<const uint4*>(stg + px * RP + 8 * g);
        }
    }
    if (a.mode != 0) {
        bf16_t* const pout = a.mode == 3 ? a.out2 : out;
        const int pcs = a.mode == 3 ? a.out2_cs : a.out_cs, pco = a.mode == 3 ? 0 : a.out_co;
        const int Hp = a.H / 2, Wp = a.W / 2;
        for (int v = lane; v < 16 * (BN / 8); v += 64) {
            const int q = v / (BN / 8), g = v - (BN / 8) * (v / (BN / 8));
            const bf16_t* s0 = stg + (2 * q) * RP + 8 * g;
            const bf16_t* s1 = s0 + RP;
            const bf16_t* s2 = s0 + 32 * RP;
            const bf16_t* s3 = s2 + RP;
            u16x8 o;
            for (int e = 0; e < 8; e++) {
                uint16_t m = s0[e];
                if (bf2f(s1[e]) > bf2f(m)) m = s1[e];
                if (bf2f(s2[e]) > bf2f(m)) m = s2[e];
                if (bf2f(s3[e]) > bf2f(m)) m = s3[e];
                o[e] = m;
            }
            const int64_t p = ((int64_t)img * Hp + (y0 >> 1) + wave) * Wp + (x0 >> 1) + q;
            *reinterpret_cast<u16x8*>(pout + p * pcs + pco + co0 + 8 * g) = o;
        }
    }
}

// Row-blocked variant (Cin a multiple of 16, H of 16; see launch_conv3x3 for
// where it is used): output tile 16 rows x
// 32 columns x (32 NT) channels, wave w computes rows 4w .. 4w + 3.  Input
// chunks of 16 channels (one 16-wide MFMA step per tap: lanes 0..31 carry
// channels 0..7 of the chunk, lanes 32..63 channels 8..15).  For each kx the
// wave reads the six input rows its four output rows need once and uses each
// for up to three ky taps; for each ky it reads the NT weight fragments once
// and uses them for the four rows: 6 + 3 NT fragment reads per 12 NT MFMAs
// (against 2 + NT per 2 NT in k_conv3x3), so the LDS read port no longer sets
// the pace.  Pixel rows in LDS are padded to 48 bytes (conflict-free 16-byte
// reads); the next chunk's global loads are in flight during the current
// chunk's MFMAs, as in k_conv3x3.
constexpr int kR4TH = 16;

template <int NT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_conv3x3_r4(ConvArgs a)
{
    constexpr int CK = 16, PS = 24;
    constexpr int HP = kR4TH + 2, WP = kConvTW + 2;
    constexpr int BN = 32 * NT;
    constexpr int SA = HP * WP * PS, SB = 9 * BN * PS;  // bf16 elements
    constexpr int RP0 = BN + 8, RP1 = BN + 4;           // staging row pitches (bf16, fp32)
    constexpr int ST0 = 4 * 128 * RP0 * 2;              // bf16 output tiles, bytes
    constexpr int ST1 = 4 * 32 * RP1 * 4;               // fp32 output rows, bytes
    constexpr int SMEM0 = 2 * (SA + SB);
    constexpr int SMEM = SMEM0 > ST0 ? (SMEM0 > ST1 ? SMEM0 : ST1) : (ST0 > ST1 ? ST0 : ST1);
    __shared__ __attribute__((aligned(16))) char smem[SMEM];
    bf16_t* const sA = reinterpret_cast<bf16_t*>(smem);
    bf16_t* const sB = sA + SA;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, l32 = lane & 31;
    int b = blockIdx.x;
    const int nbk = a.Cout / BN, txn = a.W / kConvTW, tyn = a.H / kR4TH;
    const int nb = b % nbk;
    b /= nbk;
    const int tx = b % txn;
    b /= txn;
    const int ty = b % tyn;
    const int img = b / tyn;
    const int x0 = tx * kConvTW, y0 = ty * kR4TH, co0 = nb * BN;
    const int Cin = a.Cin;
    const bf16_t* __restrict__ xin = a.x + (int64_t)img * a.H * a.W * Cin;

    f32x16 acc[4][NT];
    for (int r = 0; r < 4; r++)
        for (int j = 0; j < NT; j++)
            for (int i = 0; i < 16; i++) acc[r][j][i] = 0.0f;

    constexpr int NA_TOT = HP * WP * 2, NB_TOT = 9 * BN * 2;
    constexpr int NA = (NA_TOT + 255) / 256, NB = (NB_TOT + 255) / 256;
    uint4 pa[NA], pb[NB];
    uint32_t amask = 0;  // bit k: pa[k] lies inside the image
    auto fetch = [&](int c0) {
        amask = 0;
#pragma unroll
        for (int k = 0; k < NA; k++) {
            const int i = min(tid + 256 * k, NA_TOT - 1);
            const int g = i & 1, p = i >> 1;
            const int hx = p % WP, hy = p / WP;
            const int yy = y0 + hy - 1, xx = x0 + hx - 1;
            const bool in = yy >= 0 && yy < a.H && xx >= 0 && xx < a.W;
            const int yc = min(max(yy, 0), a.H - 1), xc = min(max(xx, 0), a.W - 1);
            pa[k] = *reinterpret_cast<const uint4*>(xin + ((int64_t)yc * a.W + xc) * Cin + c0 + 8 * g);
            amask |= (in ? 1u : 0u) << k;
        }
#pragma unroll
        for (int k = 0; k < NB; k++) {
            const int i = tid + 256 * k;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (i < NB_TOT) {
                const int g = i & 1, r = i >> 1;
                const int co = r % BN, t = r / BN;
                v = *reinterpret_cast<const uint4*>(a.w + ((int64_t)(co0 + co) * 9 + t) * Cin + c0 + 8 * g);
            }
            pb[k] = v;
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int k = 0; k < NA; k++) {
            const int i = tid + 256 * k;
            const uint4 v = (amask >> k) & 1u ? pa[k] : make_uint4(0u, 0u, 0u, 0u);
            if (i < NA_TOT) *reinterpret_cast<uint4*>(sA + (i >> 1) * PS + 8 * (i & 1)) = v;
        }
#pragma unroll
        for (int k = 0; k < NB; k++) {
            const int i = tid + 256 * k;
            if (i < NB_TOT) *reinterpret_cast<uint4*>(sB + (i >> 1) * PS + 8 * (i & 1)) = pb[k];
        }
    };
    fetch(0);
    stash();
    __syncthreads();
    for (int c0 = 0; c0 < Cin; c0 += CK) {
        const bool next = c0 + CK < Cin;
        if (next) fetch(c0 + CK);
#pragma unroll
        for (int kx = 0; kx < 3; kx++) {
            bf16x8 av[6];
#pragma unroll
            for (int i = 0; i < 6; i++)
                av[i] = *reinterpret_cast<const bf16x8*>(sA + ((4 * wave + i) * WP + l32 + kx) * PS + 8 * h);
#pragma unroll
            for (int ky = 0; ky < 3; ky++) {
                const int t = 3 * ky + kx;
                bf16x8 bv[NT];
#pragma unroll
                for (int j = 0; j < NT; j++)
                    bv[j] = *reinterpret_cast<const bf16x8*>(sB + (t * BN + 32 * j + l32) * PS + 8 * h);
#pragma unroll
                for (int r = 0; r < 4; r++)
#pragma unroll
                    for (int j = 0; j < NT; j++) acc[r][j] = mfma16(av[r + ky], bv[j], acc[r][j]);
            }
        }
        __syncthreads();
        if (next) {
            stash();
            __syncthreads();
        }
    }

    // epilogue (the K loop ended with a barrier: LDS is free)
    if (a.mode == 0 || a.mode == 2) {
        bf16_t* stg = reinterpret_cast<bf16_t*>(smem) + wave * 128 * RP0;
        for (int j = 0; j < NT; j++) {
            const int col = 32 * j + l32;
            const float bias = a.bias[co0 + col];
            for (int r = 0; r < 4; r++)
                for (int i = 0; i < 16; i++) {
                    const int px = 32 * r + 8 * (i >> 2) + 4 * h + (i & 3);
                    stg[px * RP0 + col] = f2bf(fmaxf(acc[r][j][i] + bias, 0.0f));
                }
        }
        __syncthreads();
        bf16_t* out = static_cast<bf16_t*>(a.out);
        if (a.mode == 0) {
            for (int v = lane; v < 128 * (BN / 8); v += 64) {
                const int px = v / (BN / 8), g = v - (BN / 8) * (v / (BN / 8));
                const int yy = y0 + 4 * wave + (px >> 5), xx = x0 + (px & 31);
                const int64_t p = ((int64_t)img * a.H + yy) * a.W + xx;
                *reinterpret_cast<uint4*>(out + p * a.out_cs + a.out_co + co0 + 8 * g) =
                    *reinterpret_cast<const uint4*>(stg + px * RP0 + 8 * g);
            }
        } else {
            // 2 x 2 max-pool of the wave's rows (the selection of k_maxpool: first of the
            // largest in the order (0,0), (0,1), (1,0), (1,1)): pooled rows y0 / 2 + 2 wave
            // and + 1, columns x0 / 2 .. + 15
            const int Hp = a.H / 2, Wp = a.W / 2;
            for (int v = lane; v < 32 * (BN / 8); v += 64) {
                const int q = v / (BN / 8), g = v - (BN / 8) * (v / (BN / 8));
                const int pr = q >> 4, qc = q & 15;
                const bf16_t* s0 = stg + (64 * pr + 2 * qc) * RP0 + 8 * g;
                const bf16_t* s1 = s0 + RP0;
                const bf16_t* s2 = s0 + 32 * RP0;
                const bf16_t* s3 = s2 + RP0;
                u16x8 o;
                for (int e = 0; e < 8; e++) {
                    uint16_t m = s0[e];
                    if (bf2f(s1[e]) > bf2f(m)) m = s1[e];
                    if (bf2f(s2[e]) > bf2f(m)) m = s2[e];
                    if (bf2f(s3[e]) > bf2f(m)) m = s3[e];
                    o[e] = m;
                }
                const int64_t p = ((int64_t)img * Hp + (y0 >> 1) + 2 * wave + pr) * Wp + (x0 >> 1) + qc;
                *reinterpret_cast<u16x8*>(out + p * a.out_cs + a.out_co + co0 + 8 * g) = o;
            }
        }
    } else {
        float* stg = reinterpret_cast<float*>(smem) + wave * 32 * RP1;
        float* out = static_cast<float*>(a.out);
        for (int r = 0; r < 4; r++) {
            for (int j = 0; j < NT; j++)
                for (int i = 0; i < 16; i++) {
                    const int px = 8 * (i >> 2) + 4 * h + (i & 3);
                    stg[px * RP1 + 32 * j + l32] = acc[r][j][i];
                }
            __syncthreads();
            const int yy = y0 + 4 * wave + r;
            for (int v = lane; v < 32 * (BN / 4); v += 64) {
                const int px = v / (BN / 4), g = v - (BN / 4) * (v / (BN / 4));
                const int64_t p = ((int64_t)img * a.H + yy) * a.W + x0 + px;
                *reinterpret_cast<float4*>(out + p * a.out_cs + a.out_co + co0 + 4 * g) =
                    *reinterpret_cast<const float4*>(stg + px * RP1 + 4 * g);
            }
            __syncthreads();
        }
    }
}

// ---- fused first encoder block (inference) ---------------------------------------
//
// c1a (2 -> 32 channels, input packed as 8 channels) and c1b (32 -> 32), each a
// 3x3 convolution with bias and ReLU, then the 2 x 2 max-pool, for one 16 x 32
// tile of c1b's output per workgroup.  c1a is evaluated on the 18 x 34 halo
// that c1b reads and kept in LDS as bf16 (zero outside the image: c1b's zero
// padding), so the full-resolution activations never reach HBM.
//
// Both products run transposed (A = weights, B = activations: a lane's
// accumulators hold 16 channels, 8 q + 4 h + e, of one pixel), so that each
// lane converts and stores whole groups of channels and the pooling is a
// maximum over its own two rows and its neighbour lane's.  The bf16 rounding
// (round to nearest even) is monotonic, as are the bias and the ReLU, so the
// pooled value bf16(relu(max of the four sums + bias)) is the value that the
// per-layer kernels select after rounding each of the four.  Each sum is the
// same matrix-core dot product in the same order as in the per-layer kernels
// (c1a: one tap per half wave and k step, as k_conv3x3<8, 1>; c1b: 16-channel
// halves, kx, ky, as k_conv3x3_r4<1>), so the output equals theirs bit for bit.
constexpr int kStemTH = 16, kStemTW = 32;

// two floats to packed bf16, round to nearest even (v_cvt_pk_bf16_f32)
__device__ inline uint32_t pack_bf16x2(float lo, float hi)
{
    typedef float f2 __attribute__((ext_vector_type(2)));
    typedef __bf16 b2 __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f2){lo, hi}, b2));
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_conv_stem(const bf16_t* __restrict__ x0, const bf16_t* __restrict__ w1a, const float* __restrict__ b1a,
            const bf16_t* __restrict__ w1b, const float* __restrict__ b1b, int H, int W, bf16_t* __restrict__ p1)
{
    constexpr int XH = kStemTH + 4, XW = kStemTW + 4;  // c1a input halo
    constexpr int AH = kStemTH + 2, AW = kStemTW + 2;  // c1a output = c1b input halo
    constexpr int NPX = AH * AW, MT = (NPX + 31) / 32;
    constexpr int PS = 40;                             // bf16 per pixel row in LDS (80 B)
    constexpr int SXB = XH * XW * 4, SAB = NPX * PS * 2, SBB = 9 * 32 * PS * 2;
    __shared__ __attribute__((aligned(16))) char smem[SXB + SAB + SBB];
    uint32_t* const sX = reinterpret_cast<uint32_t*>(smem);
    bf16_t* const sA = reinterpret_cast<bf16_t*>(smem + SXB);
    bf16_t* const sB = reinterpret_cast<bf16_t*>(smem + SXB + SAB);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, l32 = lane & 31;
    int b = blockIdx.x;
    const int txn = W / kStemTW, tyn = H / kStemTH;
    const int tx = b % txn;
    b /= txn;
    const int ty = b % tyn;
    const int img = b / tyn;
    const int x0t = tx * kStemTW, y0t = ty * kStemTH;

    // every global load in flight at once (registers), then the LDS stores: the packed
    // input's first two channels (ref, test) on the c1a halo, zero outside; c1b's weights
    // [co][t][ci] (to sB[t][co][ci]); c1a's A fragments: tap f = 2 s + h of output channel
    // l32 (8 packed channels), zero past tap 8.  Addresses are clamped into the buffers and
    // the values selected afterwards, so that no load sits under a branch that waits for it.
    constexpr int NXL = (XH * XW + 255) / 256, NWL = (9 * 32 * 4 + 255) / 256;
    uint32_t xv[NXL];
    uint4 wv[NWL];
    u16x8 wa[5];
#pragma unroll
    for (int k = 0; k < NXL; k++) {
        const int i = tid + 256 * k;
        const int iy = i / XW, ix = i - XW * (i / XW);
        const int yy = y0t - 2 + iy, xx = x0t - 2 + ix;
        const bool in = i < XH * XW && yy >= 0 && yy < H && xx >= 0 && xx < W;
        const int yc = min(max(yy, 0), H - 1), xc = min(max(xx, 0), W - 1);
        const uint32_t v = *reinterpret_cast<const uint32_t*>(x0 + (((int64_t)img * H + yc) * W + xc) * 8);
        xv[k] = in ? v : 0u;
    }
#pragma unroll
    for (int k = 0; k < NWL; k++) {
        const int i = min(tid + 256 * k, 9 * 32 * 4 - 1);
        const int g = i & 3, r = i >> 2;
        const int co = r % 32, t = r / 32;
        wv[k] = *reinterpret_cast<const uint4*>(w1b + ((int64_t)co * 9 + t) * 32 + 8 * g);
    }
#pragma unroll
    for (int s = 0; s < 5; s++) {
        const int f = 2 * s + h;
        const u16x8 v = *reinterpret_cast<const u16x8*>(w1a + ((int64_t)l32 * 9 + min(f, 8)) * 8);
        wa[s] = f < 9 ? v : (u16x8){0, 0, 0, 0, 0, 0, 0, 0};
    }
    // biases of this lane's channels 8 q + 4 h + e
    float4 bias_a[4], bias_b[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        bias_a[q] = *reinterpret_cast<const float4*>(b1a + 8 * q + 4 * h);
        bias_b[q] = *reinterpret_cast<const float4*>(b1b + 8 * q + 4 * h);
    }
    // the weight values pass through an empty asm here, which pins their loads ahead of it
    // (the compiler would otherwise sink each load to its store and wait for it there)
#pragma unroll
    for (int k = 0; k < NWL; k++) {
        uint32_t q0 = wv[k].x, q1 = wv[k].y, q2 = wv[k].z, q3 = wv[k].w;
        asm volatile("" : "+v"(q0), "+v"(q1), "+v"(q2), "+v"(q3));
        wv[k] = make_uint4(q0, q1, q2, q3);
    }
#pragma unroll
    for (int k = 0; k < NXL; k++) {
        const int i = tid + 256 * k;
        if (i < XH * XW) sX[i] = xv[k];
    }
#pragma unroll
    for (int k = 0; k < NWL; k++) {
        const int i = tid + 256 * k;
        const int g = i & 3, r = i >> 2;
        const int co = r % 32, t = r / 32;
        if (i < 9 * 32 * 4) *reinterpret_cast<uint4*>(sB + (t * 32 + co) * PS + 8 * g) = wv[k];
    }
    __syncthreads();

    // c1a on the halo, 32 consecutive halo pixels per product (this lane: pixel 32 m + l32),
    // wave w taking products w, w + 4, ...
    for (int m = wave; m < MT; m += 4) {
        const int p = 32 * m + l32;
        const int pa = min(p, NPX - 1);  // lanes past the halo compute a copy, never stored
        const int ay = pa / AW, ax = pa - AW * (pa / AW);
        f32x16 acc;
        for (int i = 0; i < 16; i++) acc[i] = 0.0f;
#pragma unroll
        for (int s = 0; s < 5; s++) {
            const int f = 2 * s + h;
            const int t = f < 9 ? f : 0;  // the padding step reads tap 0 against zero weights
            const int ky = t / 3, kx = t - 3 * (t / 3);
            const uint32_t v = sX[(ay + ky) * XW + ax + kx];
            const u16x8 raw = (u16x8){(uint16_t)(v & 0xFFFFu), (uint16_t)(v >> 16), 0, 0, 0, 0, 0, 0};
            acc = mfma16(__builtin_bit_cast(bf16x8, wa[s]), __builtin_bit_cast(bf16x8, raw), acc);
        }
        const int yy = y0t - 1 + ay, xx = x0t - 1 + ax;
        const bool in = yy >= 0 && yy < H && xx >= 0 && xx < W;
        if (p < NPX) {
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const float4 bq = bias_a[q];
                uint2 o;
                o.x = pack_bf16x2(fmaxf(acc[4 * q] + bq.x, 0.0f), fmaxf(acc[4 * q + 1] + bq.y, 0.0f));
                o.y = pack_bf16x2(fmaxf(acc[4 * q + 2] + bq.z, 0.0f), fmaxf(acc[4 * q + 3] + bq.w, 0.0f));
                if (!in) o = make_uint2(0u, 0u);
                *reinterpret_cast<uint2*>(sA + p * PS + 8 * q + 4 * h) = o;
            }
        }
    }
    __syncthreads();

    // c1b: wave w computes output rows 4w .. 4w + 3 of the tile (this lane: column l32)
    f32x16 acc[4];
    for (int r = 0; r < 4; r++)
        for (int i = 0; i < 16; i++) acc[r][i] = 0.0f;
#pragma unroll
    for (int c16 = 0; c16 < 2; c16++) {
#pragma unroll
        for (int kx = 0; kx < 3; kx++) {
            bf16x8 av[6];
#pragma unroll
            for (int i = 0; i < 6; i++)
                av[i] = *reinterpret_cast<const bf16x8*>(sA + ((4 * wave + i) * AW + l32 + kx) * PS + 16 * c16 + 8 * h);
#pragma unroll
            for (int ky = 0; ky < 3; ky++) {
                const bf16x8 bv =
                    *reinterpret_cast<const bf16x8*>(sB + ((3 * ky + kx) * 32 + l32) * PS + 16 * c16 + 8 * h);
#pragma unroll
                for (int r = 0; r < 4; r++) acc[r] = mfma16(bv, av[r + ky], acc[r]);
            }
        }
    }

    // epilogue: 2 x 2 max of the sums (rows 2 pr, 2 pr + 1 of this lane and of the neighbour
    // lane l32 ^ 1), then bias, ReLU and bf16; even lanes hold pooled column l32 / 2
    const int Hp = H / 2, Wp = W / 2;
#pragma unroll
    for (int pr = 0; pr < 2; pr++) {
        float mx[16];
#pragma unroll
        for (int i = 0; i < 16; i++) {
            const float v = fmaxf(acc[2 * pr][i], acc[2 * pr + 1][i]);
            mx[i] = fmaxf(v, __shfl_xor(v, 1));
        }
        if ((l32 & 1) == 0) {
            const int64_t po = ((int64_t)img * Hp + (y0t >> 1) + 2 * wave + pr) * Wp + (x0t >> 1) + (l32 >> 1);
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const float4 bq = bias_b[q];
                uint2 o;
                o.x = pack_bf16x2(fmaxf(mx[4 * q] + bq.x, 0.0f), fmaxf(mx[4 * q + 1] + bq.y, 0.0f));
                o.y = pack_bf16x2(fmaxf(mx[4 * q + 2] + bq.z, 0.0f), fmaxf(mx[4 * q + 3] + bq.w, 0.0f));
                *reinterpret_cast<uint2*>(p1 + po * 32 + 8 * q + 4 * h) = o;
            }
        }
    }
}

// ---- 3x3 weight gradient -------------------------------------------------------
//
// Workgroup: 3 waves; wave w owns the three taps of kernel row ky = w for a
// block of 32 input channels x (32 NT) output channels.  GEMM view per tap:
// M = input channel, N = output channel, K = pixel.  A k-step takes 16 pixels
// of one output row (8 per half wave); the three taps of a wave read the input
// at 10 consecutive halo columns, shared between them.  The workgroup walks a
// contiguous range of 4 x 32 pixel tiles and writes its fp32 partial sums.
constexpr int kWgTH = 4, kWgTW = 32, kWgCB = 32, kWgThreads = 192;

template <int NT>
__global__ void __launch_bounds__(kWgThreads) k_wgrad3x3(WgradArgs a)
{
    constexpr int HP = kWgTH + 2, WP = kWgTW + 2;
    constexpr int BN = 32 * NT;
    __shared__ __attribute__((aligned(16))) bf16_t sX[HP * WP * kWgCB];
    __shared__ __attribute__((aligned(16))) bf16_t sD[kWgTH * kWgTW * BN];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, l32 = lane & 31;
    int b = blockIdx.x;
    const int ncb = (a.Cin + kWgCB - 1) / kWgCB, nob = a.Cout / BN;
    const int ob = b % nob;
    b /= nob;
    const int cb = b % ncb;
    const int split = b / ncb;
    const int ci0 = cb * kWgCB, co0 = ob * BN;
    const int txn = a.W / kWgTW, tyn = a.H / kWgTH, tpi = txn * tyn;
    const int total = a.n * tpi;
    const int t_begin = split * a.tiles_per_split;
    const int t_end = min(total, t_begin + a.tiles_per_split);
    const int cvec = min(kWgCB, a.Cin - ci0) / 8;

    f32x16 acc[3][NT];
    for (int k = 0; k < 3; k++)
        for (int j = 0; j < NT; j++)
            for (int i = 0; i < 16; i++) acc[k][j][i] = 0.0f;

    for (int tile = t_begin; tile < t_end; tile++) {
        const int img = tile / tpi, rem = tile - tpi * img;
        const int y0 = (rem / txn) * kWgTH, x0 = (rem - txn * (rem / txn)) * kWgTW;
        const bf16_t* __restrict__ xin = a.x + (int64_t)img * a.H * a.W * a.Cin;
        const bf16_t* __restrict__ din = a.dz + (int64_t)img * a.H * a.W * a.Cout;
        for (int i = tid; i < HP * WP * 4; i += kWgThreads) {
            const int g = i & 3, p = i >> 2;
            const int hx = p % WP, hy = p / WP;
            const int yy = y0 + hy - 1, xx = x0 + hx - 1;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (g < cvec && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W)
                v = *reinterpret_cast<const uint4*>(xin + ((int64_t)yy * a.W + xx) * a.Cin + ci0 + 8 * g);
            *reinterpret_cast<uint4*>(sX + p * kWgCB + 8 * g) = v;
        }
        for (int i = tid; i < kWgTH * kWgTW * (BN / 8); i += kWgThreads) {
            const int g = i % (BN / 8), p = i / (BN / 8);
            const int yy = y0 + p / kWgTW, xx = x0 + p % kWgTW;
            *reinterpret_cast<uint4*>(sD + p * BN + 8 * g) =
                *reinterpret_cast<const uint4*>(din + ((int64_t)yy * a.W + xx) * a.Cout + co0 + 8 * g);
        }
        __syncthreads();
        for (int row = 0; row < kWgTH; row++) {
            for (int xb = 0; xb < kWgTW; xb += 16) {
                const int px = xb + 8 * h;  // first pixel (tile column) of this half wave
                uint16_t xv[10];
                for (int m = 0; m < 10; m++) xv[m] = sX[((row + wave) * WP + px + m) * kWgCB + l32];
                bf16x8 av[3];
                for (int kx = 0; kx < 3; kx++) {
                    u16x8 t;
                    for (int j = 0; j < 8; j++) t[j] = xv[kx + j];
                    av[kx] = __builtin_bit_cast(bf16x8, t);
                }
                for (int jn = 0; jn < NT; jn++) {
                    u16x8 t;
                    for (int j = 0; j < 8; j++) t[j] = sD[(row * kWgTW + px + j) * BN + 32 * jn + l32];
                    const bf16x8 bv = __builtin_bit_cast(bf16x8, t);
                    for (int kx = 0; kx < 3; kx++) acc[kx][jn] = mfma16(av[kx], bv, acc[kx][jn]);
                }
            }
        }
        __syncthreads();
    }

    const int keep = a.cin_keep;
    for (int kx = 0; kx < 3; kx++) {
        const int t = 3 * wave + kx;
        for (int jn = 0; jn < NT; jn++) {
            const int co = co0 + 32 * jn + l32;
            for (int i = 0; i < 16; i++) {
                const int ci = ci0 + 8 * (i >> 2) + 4 * h + (i & 3);
                if (ci < keep)
                    a.part[(((int64_t)split * 9 + t) * keep + ci) * a.Cout + co] = acc[kx][jn][i];
            }
        }
    }
}

// ---- element-wise passes ---------------------------------------------------------

// Block: 32 columns x 8 row lanes over rows [blockIdx.y * chunk, + chunk);
// lane r sums rows r, r + 8, ... of the chunk; the 8 lane sums are then added
// in increasing r.  out has one row per chunk.
__global__ void __launch_bounds__(256) k_colsum(const float* __restrict__ part, int64_t nb, int64_t ncols,
                                                int64_t chunk, float* __restrict__ out)
{
    __shared__ float sh[8][32];
    const int cl = threadIdx.x & 31, r = threadIdx.x >> 5;
    const int64_t c = (int64_t)blockIdx.x * 32 + cl;
    const int64_t b0 = (int64_t)blockIdx.y * chunk, b1 = min(nb, b0 + chunk);
    float s = 0.0f;
    if (c < ncols)
        for (int64_t b = b0 + r; b < b1; b += 8) s += part[b * ncols + c];
    sh[r][cl] = s;
    __syncthreads();
    if (r == 0 && c < ncols) {
        float t = sh[0][cl];
        for (int k = 1; k < 8; k++) t += sh[k][cl];
        out[(int64_t)blockIdx.y * ncols + c] = t;
    }
}

__global__ void k_pack_input(const float* __restrict__ rb, int64_t rs, const int32_t* __restrict__ slot,
                             const float* __restrict__ tb, int64_t ts, int n, int64_t hw,
                             bf16_t* __restrict__ x)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n * hw) return;
    const int64_t pair = i / hw, p = i - pair * hw;
    const int64_t rsl = slot ? slot[pair] : pair;
    const float r = rb[rsl * rs + p], t = tb[pair * ts + p];
    uint4 v;
    v.x = (uint32_t)f2bf(r) | ((uint32_t)f2bf(t) << 16);
    v.y = 0u;
    v.z = 0u;
    v.w = 0u;
    *reinterpret_cast<uint4*>(x + 8 * i) = v;
}

__device__ inline float up2_sample(const float* __restrict__ img, int h, int w, int X, int Y)
{
    const float cx = fminf(fmaxf(0.5f * ((float)X - 0.5f), 0.0f), (float)(w - 1));
    const float cy = fminf(fmaxf(0.5f * ((float)Y - 0.5f), 0.0f), (float)(h - 1));
    const int x0 = (int)floorf(cx), y0 = (int)floorf(cy);
    const int x1 = min(x0 + 1, w - 1), y1 = min(y0 + 1, h - 1);
    const float fx = cx - (float)x0, fy = cy - (float)y0;
    const float a0 = img[y0 * w + x0], a1 = img[y0 * w + x1], b0 = img[y1 * w + x0], b1 = img[y1 * w + x1];
    const float top = a0 + fx * (a1 - a0), bot = b0 + fx * (b1 - b0);
    return top + fy * (bot - top);
}

__global__ void k_pack_input_up2(const float* __restrict__ rb, int64_t rs, const int32_t* __restrict__ slot,
                                 const float* __restrict__ tb, int64_t ts, int n, int h, int w,
                                 bf16_t* __restrict__ x)
{
    const int W2 = 2 * w, H2 = 2 * h;
    const int64_t hw2 = (int64_t)H2 * W2;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n * hw2) return;
    const int64_t pair = i / hw2, p = i - pair * hw2;
    const int X = (int)(p % W2), Y = (int)(p / W2);
    const int64_t rsl = slot ? slot[pair] : pair;
    const float r = up2_sample(rb + rsl * rs, h, w, X, Y), t = up2_sample(tb + pair * ts, h, w, X, Y);
    uint4 v;
    v.x = (uint32_t)f2bf(r) | ((uint32_t)f2bf(t) << 16);
    v.y = 0u;
    v.z = 0u;
    v.w = 0u;
    *reinterpret_cast<uint4*>(x + 8 * i) = v;
}

// One thread per (pooled pixel, 8-channel group).
__global__ void k_maxpool(const bf16_t* __restrict__ in, int n, int H, int W, int C, int cs, int co,
                          bf16_t* __restrict__ out)
{
    const int cg = C / 8;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int h2 = H / 2, w2 = W / 2;
    if (i >= (int64_t)n * h2 * w2 * cg) return;
    const int g = (int)(i % cg);
    const int64_t q = i / cg;
    const int x = (int)(q % w2);
    const int64_t r = q / w2;
    const int y = (int)(r % h2);
    const int64_t img = r / h2;
    const bf16_t* base = in + ((img * H + 2 * y) * W + 2 * x) * cs + co + 8 * g;
    const u16x8 v0 = *reinterpret_cast<const u16x8*>(base);
    const u16x8 v1 = *reinterpret_cast<const u16x8*>(base + cs);
    const u16x8 v2 = *reinterpret_cast<const u16x8*>(base + (int64_t)W * cs);
    const u16x8 v3 = *reinterpret_cast<const u16x8*>(base + (int64_t)W * cs + cs);
    u16x8 o;
    for (int j = 0; j < 8; j++) {
        uint16_t m = v0[j];
        if (bf2f(v1[j]) > bf2f(m)) m = v1[j];
        if (bf2f(v2[j]) > bf2f(m)) m = v2[j];
        if (bf2f(v3[j]) > bf2f(m)) m = v3[j];
        o[j] = m;
    }
    *reinterpret_cast<u16x8*>(out + q * C + 8 * g) = o;
}

// One thread per (pooled pixel, channel): route g to the first maximum.
__global__ void k_maxpool_back(const float* __restrict__ g, const bf16_t* __restrict__ act, int n, int H,
                               int W, int C, int cs, int co, const float* __restrict__ add, int add_cs,
                               int add_co, float* __restrict__ gin)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int h2 = H / 2, w2 = W / 2;
    if (i >= (int64_t)n * h2 * w2 * C) return;
    const int c = (int)(i % C);
    const int64_t q = i / C;
    const int x = (int)(q % w2);
    const int64_t r = q / w2;
    const int y = (int)(r % h2);
    const int64_t img = r / h2;
    int64_t pix[4];
    pix[0] = (img * H + 2 * y) * W + 2 * x;
    pix[1] = pix[0] + 1;
    pix[2] = pix[0] + W;
    pix[3] = pix[2] + 1;
    int k = 0;
    float m = bf2f(act[pix[0] * cs + co + c]);
    for (int j = 1; j < 4; j++) {
        const float v = bf2f(act[pix[j] * cs + co + c]);
        if (v > m) {
            m = v;
            k = j;
        }
    }
    const float gv = g[i];
    for (int j = 0; j < 4; j++) {
        float v = j == k ? gv : 0.0f;
        if (add) v += add[pix[j] * add_cs + add_co + c];
        gin[pix[j] * C + c] = v;
    }
}

__global__ void k_upsample_into(const bf16_t* __restrict__ in, int n, int h, int w, int C,
                                bf16_t* __restrict__ out, int cs)
{
    const int cg = C / 8;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n * h * w * cg) return;
    const int g = (int)(i % cg);
    const int64_t q = i / cg;
    const int x = (int)(q % w);
    const int64_t r = q / w;
    const int y = (int)(r % h);
    const int64_t img = r / h;
    const uint4 v = *reinterpret_cast<const uint4*>(in + q * C + 8 * g);
    const int W2 = 2 * w;
    const int64_t o = ((img * 2 * h + 2 * y) * W2 + 2 * x) * cs + 8 * g;
    *reinterpret_cast<uint4*>(out + o) = v;
    *reinterpret_cast<uint4*>(out + o + cs) = v;
    *reinterpret_cast<uint4*>(out + o + (int64_t)W2 * cs) = v;
    *reinterpret_cast<uint4*>(out + o + (int64_t)W2 * cs + cs) = v;
}

__global__ void k_upsample_back(const float* __restrict__ gout, int n, int h, int w, int C, int cs,
                                float* __restrict__ g)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n * h * w * C) return;
    const int c = (int)(i % C);
    const int64_t q = i / C;
    const int x = (int)(q % w);
    const int64_t r = q / w;
    const int y = (int)(r % h);
    const int64_t img = r / h;
    const int W2 = 2 * w;
    const int64_t o = ((img * 2 * h + 2 * y) * W2 + 2 * x) * cs + c;
    g[i] = ((gout[o] + gout[o + cs]) + gout[o + (int64_t)W2 * cs]) + gout[o + (int64_t)W2 * cs + cs];
}

// One thread per (pixel, 8-channel group): 16-byte loads of the activation,
// 32-byte loads of the gradient, a 16-byte store of dz.  A block covers
// 2048 / C pixels; its partial bias sums add the block's pixels in order.
// C must be 32, 64, 128 or 256.
__global__ void __launch_bounds__(256) k_mask_round(const float* __restrict__ g, const bf16_t* __restrict__ act,
                                                    int64_t P, int C, int act_cs, int act_co,
                                                    bf16_t* __restrict__ dz, float* __restrict__ part)
{
    __shared__ float sh[256][9];
    const int tid = threadIdx.x;
    const int cg = C >> 3, ppb = 256 / cg;
    const int64_t p = (int64_t)blockIdx.x * ppb + tid / cg;
    const int q = tid % cg;
    float v[8];
    for (int j = 0; j < 8; j++) v[j] = 0.0f;
    if (p < P) {
        const u16x8 a = *reinterpret_cast<const u16x8*>(act + p * act_cs + act_co + 8 * q);
        const float4 g0 = *reinterpret_cast<const float4*>(g + p * C + 8 * q);
        const float4 g1 = *reinterpret_cast<const float4*>(g + p * C + 8 * q + 4);
        const float gv[8] = {g0.x, g0.y, g0.z, g0.w, g1.x, g1.y, g1.z, g1.w};
        u16x8 o;
        for (int j = 0; j < 8; j++) {
            v[j] = bf2f(a[j]) > 0.0f ? gv[j] : 0.0f;
            o[j] = f2bf(v[j]);
        }
        *reinterpret_cast<u16x8*>(dz + p * C + 8 * q) = o;
    }
    for (int j = 0; j < 8; j++) sh[tid][j] = v[j];
    __syncthreads();
    if (tid < C) {
        const int qq = tid >> 3, j = tid & 7;
        float t = 0.0f;
        for (int k = 0; k < ppb; k++) t += sh[k * cg + qq][j];
        part[(int64_t)blockIdx.x * C + tid] = t;
    }
}

// 16 threads per pixel, each 8 channels (one 16-byte load); the 16 partial
// dot products are combined by a fixed xor tree.  C must be 128.
__global__ void __launch_bounds__(256) k_head_fwd(const bf16_t* __restrict__ act, int64_t P, int C,
                                                  const float* __restrict__ hw, const float* __restrict__ hb,
                                                  float* __restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t p = t >> 4;
    const int g = (int)(t & 15);
    float s0 = 0.0f, s1 = 0.0f;
    if (p < P) {
        const u16x8 v = *reinterpret_cast<const u16x8*>(act + p * C + 8 * g);
        for (int j = 0; j < 8; j++) {
            const float a = bf2f(v[j]);
            const int c = 8 * g + j;
            s0 += a * hw[2 * c];
            s1 += a * hw[2 * c + 1];
        }
    }
    for (int o = 1; o < 16; o <<= 1) {
        s0 += __shfl_xor(s0, o, 16);
        s1 += __shfl_xor(s1, o, 16);
    }
    if (p < P && g == 0) {
        out[2 * p] = s0 + hb[0];
        out[2 * p + 1] = s1 + hb[1];
    }
}

constexpr int kLossPB = 256;

__global__ void __launch_bounds__(kLossPB) k_loss(const float* __restrict__ out, const float* __restrict__ label,
                                                  int64_t P, float* __restrict__ gout, float* __restrict__ part)
{
    __shared__ float sh[kLossPB];
    const int64_t p = (int64_t)blockIdx.x * kLossPB + threadIdx.x;
    float e = 0.0f;
    if (p < P) {
        const float dx = out[2 * p] - label[2 * p], dy = out[2 * p + 1] - label[2 * p + 1];
        const float sc = 2.0f / (float)P;
        gout[2 * p] = sc * dx;
        gout[2 * p + 1] = sc * dy;
        e = dx * dx + dy * dy;
    }
    sh[threadIdx.x] = e;
    __syncthreads();
    for (int s = kLossPB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

constexpr int kHeadPB = 256;

// Columns of the partial sums: dhw[c][o] at 2c + o, dhb[o] at 2C + o.
__global__ void __launch_bounds__(256) k_head_back(const bf16_t* __restrict__ act, const float* __restrict__ gout,
                                                   int64_t P, int C, const float* __restrict__ hw,
                                                   float* __restrict__ gact, float* __restrict__ part)
{
    const int tid = threadIdx.x;
    const int64_t p0 = (int64_t)blockIdx.x * kHeadPB;
    const int64_t p1 = min(P, p0 + kHeadPB);
    const int ncol = 2 * C + 2;
    for (int col = tid; col < ncol; col += 256) {
        float s = 0.0f;
        if (col < 2 * C) {
            const int c = col >> 1, o = col & 1;
            for (int64_t p = p0; p < p1; p++) s += bf2f(act[p * C + c]) * gout[2 * p + o];
        } else {
            const int o = col - 2 * C;
            for (int64_t p = p0; p < p1; p++) s += gout[2 * p + o];
        }
        part[(int64_t)blockIdx.x * ncol + col] = s;
    }
    for (int64_t i = tid; i < (p1 - p0) * C; i += 256) {
        const int64_t p = p0 + i / C;
        const int c = (int)(i % C);
        gact[p * C + c] = gout[2 * p] * hw[2 * c] + gout[2 * p + 1] * hw[2 * c + 1];
    }
}

__global__ void k_pack_weights(const float* __restrict__ w, int cin, int cin_pad, int cout,
                               bf16_t* __restrict__ fwd, bf16_t* __restrict__ dgr)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nf = (int64_t)cout * 9 * cin_pad;
    if (i < nf) {
        const int ci = (int)(i % cin_pad);
        const int64_t r = i / cin_pad;
        const int t = (int)(r % 9);
        const int co = (int)(r / 9);
        fwd[i] = ci < cin ? f2bf(w[((int64_t)t * cin + ci) * cout + co]) : (bf16_t)0;
    }
    const int64_t nd = (int64_t)cin * 9 * cout;
    if (dgr && i < nd) {
        const int co = (int)(i % cout);
        const int64_t r = i / cout;
        const int t = (int)(r % 9);
        const int ci = (int)(r / 9);
        dgr[i] = f2bf(w[((int64_t)(8 - t) * cin + ci) * cout + co]);
    }
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float bc1,
                       float bc2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / bc1, vh = vi / bc2;
    p[i] = p[i] - lr * mh / (sqrtf(vh) + eps);
}

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

constexpr int64_t kColsumChunk = 512;

}  // namespace

bool conv3x3_supported(int H, int W, int Cin, int Cout)
{
    return H > 0 && W > 0 && H % kConvTH == 0 && W % kConvTW == 0 && (Cin % 32 == 0 || Cin == 8) &&
           Cout > 0 && Cout % 32 == 0;
}

hipError_t launch_conv3x3(const ConvArgs& a, hipStream_t s)
{
    if (!conv3x3_supported(a.H, a.W, a.Cin, a.Cout) || a.n <= 0) return hipErrorInvalidValue;
    if (a.mode < 0 || a.mode > 3 || (a.mode == 3 && (!a.out2 || a.out2_cs < a.Cout)) ||
        (a.c2 != 0 && (a.c2 < 0 || a.c2 % 32 != 0 || a.c2 > a.Cin || !a.x2 || a.Cin == 8)))
        return hipErrorInvalidValue;
    const int nt = a.Cout % 64 == 0 ? 2 : 1;
    const dim3 block(256);
    // The row-blocked kernel (16-row tiles, half the LDS fragment reads per product, input
    // chunks of 16 channels) for 32 output channels, and for two N tiles when the input has
    // only 32 channels (one 32-channel chunk in k_conv3x3: nothing to overlap the loads with);
    // elsewhere both take the same time (measured per layer of the network).
    if (a.Cin % 16 == 0 && a.H % kR4TH == 0 && a.mode != 3 && a.c2 == 0 && (nt == 1 || a.Cin == 32)) {
        const int64_t tiles4 = (int64_t)a.n * (a.H / kR4TH) * (a.W / kConvTW) * (a.Cout / (32 * nt));
        if (nt == 2) hipLaunchKernelGGL((k_conv3x3_r4<2>), dim3((unsigned)tiles4), block, 0, s, a);
        else hipLaunchKernelGGL((k_conv3x3_r4<1>), dim3((unsigned)tiles4), block, 0, s, a);
        return hipGetLastError();
    }
    // k_conv3x3_lds (two N tiles) where the input has at least 8 chunks of 32 channels: measured per layer of
    // the network (256 pairs), 256 -> 256 at 32 x 32 px 287 -> 261 us and the decoder's 384-channel
    // layer 805 -> 699 us; with 128 input channels both kernels take the same time, with 64 the
    // register-staged one is faster (350 against 376 us: two chunks leave the loads nothing to
    // overlap)
    if (a.lds_dma && a.mode != 1 && nt == 2 && a.Cin % 32 == 0 && a.Cin >= 256 && a.H % kLdsTH == 0) {
        const int64_t t16 = (int64_t)a.n * (a.H / kLdsTH) * (a.W / kConvTW) * (a.Cout / 64);
        if (a.c2 != 0) hipLaunchKernelGGL((k_conv3x3_lds<2, true>), dim3((unsigned)t16), dim3(512), 0, s, a);
        else hipLaunchKernelGGL((k_conv3x3_lds<2, false>), dim3((unsigned)t16), dim3(512), 0, s, a);
        return hipGetLastError();
    }
    const int64_t tiles = (int64_t)a.n * (a.H / kConvTH) * (a.W / kConvTW) * (a.Cout / (32 * nt));
    const dim3 grid((unsigned)tiles);
    if (a.Cin == 8) {
        if (nt == 2) hipLaunchKernelGGL((k_conv3x3<8, 2>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_conv3x3<8, 1>), grid, block, 0, s, a);
    } else if (a.c2 != 0) {
        if (nt == 2) hipLaunchKernelGGL((k_conv3x3<32, 2, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_conv3x3<32, 1, true>), grid, block, 0, s, a);
    } else {
        if (nt == 2) hipLaunchKernelGGL((k_conv3x3<32, 2>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_conv3x3<32, 1>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_conv_stem(const bf16_t* x0, const bf16_t* w1a, const float* b1a, const bf16_t* w1b,
                            const float* b1b, int n, int H, int W, bf16_t* p1, hipStream_t s)
{
    if (n <= 0 || H <= 0 || W <= 0 || H % kStemTH != 0 || W % kStemTW != 0) return hipErrorInvalidValue;
    const int64_t tiles = (int64_t)n * (H / kStemTH) * (W / kStemTW);
    hipLaunchKernelGGL(k_conv_stem, dim3((unsigned)tiles), dim3(256), 0, s, x0, w1a, b1a, w1b, b1b, H, W, p1);
    return hipGetLastError();
}

int wgrad_splits(int n, int H, int W, int Cin, int Cout, int* tiles_per_split)
{
    const int nt = Cout % 64 == 0 ? 2 : 1;
    const int ncb = (Cin + kWgCB - 1) / kWgCB, nob = Cout / (32 * nt);
    const int64_t total = (int64_t)n * (H / kWgTH) * (W / kWgTW);
    int64_t splits = 1536 / (ncb * nob);
    if (splits < 1) splits = 1;
    if (splits > total) splits = total;
    const int64_t tps = (total + splits - 1) / splits;
    *tiles_per_split = (int)tps;
    return (int)((total + tps - 1) / tps);
}

hipError_t launch_wgrad3x3(const WgradArgs& a, hipStream_t s)
{
    if (a.n <= 0 || a.H % kWgTH || a.W % kWgTW || a.Cout % 32 || !(a.Cin % 32 == 0 || a.Cin == 8))
        return hipErrorInvalidValue;
    const int nt = a.Cout % 64 == 0 ? 2 : 1;
    const int ncb = (a.Cin + kWgCB - 1) / kWgCB, nob = a.Cout / (32 * nt);
    const dim3 grid((unsigned)((int64_t)a.splits * ncb * nob)), block(kWgThreads);
    if (nt == 2) hipLaunchKernelGGL(k_wgrad3x3<2>, grid, block, 0, s, a);
    else hipLaunchKernelGGL(k_wgrad3x3<1>, grid, block, 0, s, a);
    return hipGetLastError();
}

hipError_t launch_colsum(const float* part, int64_t nb, int64_t ncols, float* out, float* tmp, int64_t tmp_floats,
                         hipStream_t s)
{
    if (nb > kColsumChunk) {
        const int64_t nch = (nb + kColsumChunk - 1) / kColsumChunk;
        if (!tmp || nch * ncols > tmp_floats || nch > 65535) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_colsum, dim3(blocks_for(ncols, 32), (unsigned)nch), dim3(256), 0, s, part, nb, ncols,
                           (int64_t)kColsumChunk, tmp);
        part = tmp;
        nb = nch;
    }
    hipLaunchKernelGGL(k_colsum, dim3(blocks_for(ncols, 32), 1), dim3(256), 0, s, part, nb, ncols, nb, out);
    return hipGetLastError();
}

hipError_t launch_pack_input(const float* ref_base, int64_t ref_stride, const int32_t* ref_slot,
                             const float* test_base, int64_t test_stride, int n, int H, int W,
                             bf16_t* x, hipStream_t s)
{
    const int64_t hw = (int64_t)H * W;
    hipLaunchKernelGGL(k_pack_input, dim3(blocks_for((int64_t)n * hw, 256)), dim3(256), 0, s, ref_base,
                       ref_stride, ref_slot, test_base, test_stride, n, hw, x);
    return hipGetLastError();
}

hipError_t launch_pack_input_up2(const float* ref_base, int64_t ref_stride, const int32_t* ref_slot,
                                 const float* test_base, int64_t test_stride, int n, int h, int w,
                                 bf16_t* x, hipStream_t s)
{
    const int64_t hw2 = (int64_t)4 * h * w;
    hipLaunchKernelGGL(k_pack_input_up2, dim3(blocks_for((int64_t)n * hw2, 256)), dim3(256), 0, s, ref_base,
                       ref_stride, ref_slot, test_base, test_stride, n, h, w, x);
    return hipGetLastError();
}

hipError_t launch_maxpool(const bf16_t* in, int n, int H, int W, int C, int cs, int co, bf16_t* out,
                          hipStream_t s)
{
    const int64_t items = (int64_t)n * (H / 2) * (W / 2) * (C / 8);
    hipLaunchKernelGGL(k_maxpool, dim3(blocks_for(items, 256)), dim3(256), 0, s, in, n, H, W, C, cs, co, out);
    return hipGetLastError();
}

hipError_t launch_maxpool_back(const float* g, const bf16_t* act, int n, int H, int W, int C, int cs,
                               int co, const float* add, int add_cs, int add_co, float* g_in,
                               hipStream_t s)
{
    const int64_t items = (int64_t)n * (H / 2) * (W / 2) * C;
    hipLaunchKernelGGL(k_maxpool_back, dim3(blocks_for(items, 256)), dim3(256), 0, s, g, act, n, H, W, C, cs,
                       co, add, add_cs, add_co, g_in);
    return hipGetLastError();
}

hipError_t launch_upsample_into(const bf16_t* in, int n, int h, int w, int C, bf16_t* out, int cs,
                                hipStream_t s)
{
    const int64_t items = (int64_t)n * h * w * (C / 8);
    hipLaunchKernelGGL(k_upsample_into, dim3(blocks_for(items, 256)), dim3(256), 0, s, in, n, h, w, C, out, cs);
    return hipGetLastError();
}

hipError_t launch_upsample_back(const float* gout, int n, int h, int w, int C, int cs, float* g,
                                hipStream_t s)
{
    const int64_t items = (int64_t)n * h * w * C;
    hipLaunchKernelGGL(k_upsample_back, dim3(blocks_for(items, 256)), dim3(256), 0, s, gout, n, h, w, C, cs, g);
    return hipGetLastError();
}

int mask_blocks(int64_t P, int C) { return (int)((P * C / 8 + 255) / 256); }

hipError_t launch_mask_round(const float* g, const bf16_t* act, int64_t P, int C, int act_cs,
                             int act_co, bf16_t* dz, float* bias_part, hipStream_t s)
{
    if (C != 32 && C != 64 && C != 128 && C != 256) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mask_round, dim3(mask_blocks(P, C)), dim3(256), 0, s, g, act, P, C, act_cs, act_co, dz,
                       bias_part);
    return hipGetLastError();
}

hipError_t launch_head_fwd(const bf16_t* act, int64_t P, int C, const float* hw, const float* hb,
                           float* out, hipStream_t s)
{
    if (C != 128) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_head_fwd, dim3(blocks_for(16 * P, 256)), dim3(256), 0, s, act, P, C, hw, hb, out);
    return hipGetLastError();
}

int loss_blocks(int64_t P) { return (int)((P + kLossPB - 1) / kLossPB); }

hipError_t launch_loss(const float* out, const float* label, int64_t P, float* gout, float* loss_part,
                       hipStream_t s)
{
    hipLaunchKernelGGL(k_loss, dim3(loss_blocks(P)), dim3(kLossPB), 0, s, out, label, P, gout, loss_part);
    return hipGetLastError();
}

int head_blocks(int64_t P) { return (int)((P + kHeadPB - 1) / kHeadPB); }

hipError_t launch_head_back(const bf16_t* act, const float* gout, int64_t P, int C, const float* hw,
                            float* gact, float* part, hipStream_t s)
{
    hipLaunchKernelGGL(k_head_back, dim3(head_blocks(P)), dim3(256), 0, s, act, gout, P, C, hw, gact, part);
    return hipGetLastError();
}

hipError_t launch_pack_weights(const float* w, int cin, int cin_pad, int cout, bf16_t* fwd,
                               bf16_t* dgr, hipStream_t s)
{
    const int64_t nf = (int64_t)cout * 9 * cin_pad, nd = (int64_t)cin * 9 * cout;
    const int64_t n = nf > nd ? nf : nd;
    hipLaunchKernelGGL(k_pack_weights, dim3(blocks_for(n, 256)), dim3(256), 0, s, w, cin, cin_pad, cout, fwd, dgr);
    return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, float bc1, float bc2, hipStream_t s)
{
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, bc1,
                       bc2);
    return hipGetLastError();
}

}  // namespace ebsd
