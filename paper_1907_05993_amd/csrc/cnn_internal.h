// Internal declarations of the warm-start network: bf16 MFMA convolution
// kernels, the element-wise passes between them and the network runner.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

struct ebsd_cnn;

namespace ebsd {

typedef uint16_t bf16_t;  // bfloat16 storage (upper half of an IEEE float)

// 3x3 convolution, zero padding 1, NHWC, as an implicit GEMM on the matrix
// cores: M = output pixels, N = output channels, K = 9 * Cin with
// k = (ky * 3 + kx) * Cin + ci.  Weights are bf16 [Cout][9][Cin].
struct ConvArgs {
    const bf16_t* x;   // input [n][H][W][Cin] bf16
    const bf16_t* w;   // [Cout][9][Cin] bf16
    const float* bias; // [Cout] (mode 0)
    void* out;         // mode 0: bf16, mode 1: fp32
    int32_t n, H, W, Cin, Cout;
    int32_t mode;      // 0: bf16(relu(acc + bias)); 1: fp32 acc (input gradients); 2: as 0, then the
                       // 2 x 2 max-pool (out is [n][H/2][W/2][out_cs], the result of k_maxpool);
                       // 3: as 0, and also the pooled result into out2
    int32_t out_cs;    // channels per output pixel (>= Cout)
    int32_t out_co;    // channel offset of this output inside the output pixel
    // mode 3: pooled output [n][H/2][W/2][out2_cs], channels [0, Cout)
    bf16_t* out2 = nullptr;
    int32_t out2_cs = 0;
    // input channels [0, c2) read from x2 [n][H/2][W/2][c2] upsampled x2 (nearest) instead of x
    // (whose channels [0, c2) are then not read); c2 a multiple of 32, 0: not used
    const bf16_t* x2 = nullptr;
    int32_t c2 = 0;
    // bf16-output modes: k_conv3x3_lds (input chunks moved into LDS by the buffer unit, 16-row
    // tiles, the same sums in the same order, so the same outputs) for layers with at least 256
    // input channels (and H % 16 == 0); 0: k_conv3x3 throughout
    int32_t lds_dma = 0;
};
// Requirements: W % 32 == 0, H % 8 == 0, Cin % 32 == 0 or Cin == 8, Cout % 32 == 0.
bool conv3x3_supported(int H, int W, int Cin, int Cout);
hipError_t launch_conv3x3(const ConvArgs& a, hipStream_t s);

// The network's first block for inference in one pass: c1a (input packed as
// 8 bf16 channels [n][H][W][8], weights w1a [32][9][8]) and c1b (w1b
// [32][9][32]), each with bias and ReLU, then the 2 x 2 max-pool into p1
// [n][H/2][W/2][32]; equal bit for bit to the two convolutions (mode 0, then
// mode 2).  H % 16 == 0, W % 32 == 0.
hipError_t launch_conv_stem(const bf16_t* x0, const bf16_t* w1a, const float* b1a, const bf16_t* w1b,
                            const float* b1b, int n, int H, int W, bf16_t* p1, hipStream_t s);

// Weight gradient of a 3x3 convolution: dW[t][ci][co] = sum over pixels of
// x[p + off(t)][ci] * dz[p][co], split over pixel ranges into fp32 partial
// sums part[split][9][cin_keep][Cout] (then reduced in a fixed order).
struct WgradArgs {
    const bf16_t* x;   // [n][H][W][Cin] bf16
    const bf16_t* dz;  // [n][H][W][Cout] bf16
    float* part;       // [splits][9 * cin_keep * Cout]
    int32_t n, H, W, Cin, Cout;
    int32_t cin_keep;  // input channels whose gradient is kept (<= Cin)
    int32_t splits, tiles_per_split;
};
int wgrad_splits(int n, int H, int W, int Cin, int Cout, int* tiles_per_split);
hipError_t launch_wgrad3x3(const WgradArgs& a, hipStream_t s);

// out[c] = sum_{b < nb} part[b * ncols + c] in a fixed order: rows are
// summed in chunks of 512 (partial sums in tmp, ceil(nb / 512) * ncols
// floats) and the chunk sums in increasing chunk order; tmp is not used
// when nb <= 512.
hipError_t launch_colsum(const float* part, int64_t nb, int64_t ncols, float* out, float* tmp, int64_t tmp_floats,
                         hipStream_t s);

// Packed network input: x[i][y][x][0..7] = bf16(ref_i, test_i, 0, ..., 0) from
// normalised fp32 images ref = ref_base + slot(i) * ref_stride, test likewise.
hipError_t launch_pack_input(const float* ref_base, int64_t ref_stride, const int32_t* ref_slot,
                             const float* test_base, int64_t test_stride, int n, int H, int W,
                             bf16_t* x, hipStream_t s);
// Same from h x w images upsampled x2 to 2h x 2w (bilinear, clamped, source
// coordinate (i - 0.5) / 2).
hipError_t launch_pack_input_up2(const float* ref_base, int64_t ref_stride, const int32_t* ref_slot,
                                 const float* test_base, int64_t test_stride, int n, int h, int w,
                                 bf16_t* x, hipStream_t s);
// 2x2 max pooling of bf16 [n][H][W][cs] (channels [co, co + C)) -> [n][H/2][W/2][C].
hipError_t launch_maxpool(const bf16_t* in, int n, int H, int W, int C, int cs, int co, bf16_t* out,
                          hipStream_t s);
// Gradient through the pooling: g_in[p][c] = (first maximum of p's window ? g[p/2][c] : 0)
// (+ add[p * add_cs + add_co + c] when add != NULL).  fp32.
hipError_t launch_maxpool_back(const float* g, const bf16_t* act, int n, int H, int W, int C, int cs,
                               int co, const float* add, int add_cs, int add_co, float* g_in,
                               hipStream_t s);
// Nearest 2x upsampling of bf16 [n][h][w][C] into channels [0, C) of [n][2h][2w][cs].
hipError_t launch_upsample_into(const bf16_t* in, int n, int h, int w, int C, bf16_t* out, int cs,
                                hipStream_t s);
// Gradient of the upsampling: g[n][h][w][c] = sum of the 4 copies in gout[n][2h][2w][cs] channel c.
hipError_t launch_upsample_back(const float* gout, int n, int h, int w, int C, int cs, float* g,
                                hipStream_t s);
// dz = g * (act > 0) rounded to bf16; per-block partial bias sums of the fp32
// dz (mask_blocks(P, C) rows of C).  C in {32, 64, 128, 256}.
int mask_blocks(int64_t P, int C);
hipError_t launch_mask_round(const float* g, const bf16_t* act, int64_t P, int C, int act_cs,
                             int act_co, bf16_t* dz, float* bias_part, hipStream_t s);
// 1x1 head: out[p][o] = sum_c act[p][c] * hw[c][o] + hb[o], o < 2, fp32.
hipError_t launch_head_fwd(const bf16_t* act, int64_t P, int C, const float* hw, const float* hb,
                           float* out, hipStream_t s);
// Loss (mean squared endpoint error): gout = 2 (out - label) / P and per-block partial sums.
int loss_blocks(int64_t P);
hipError_t launch_loss(const float* out, const float* label, int64_t P, float* gout, float* loss_part,
                       hipStream_t s);
// Head backward: gact[p][c] = sum_o gout[p][o] hw[c][o]; per-block partials of
// dhw[c][o] = sum_p act[p][c] gout[p][o] and dhb[o] = sum_p gout[p][o].
int head_blocks(int64_t P);
hipError_t launch_head_back(const bf16_t* act, const float* gout, int64_t P, int C, const float* hw,
                            float* gact, float* part, hipStream_t s);
// Weight packing from fp32 HWIO masters [3][3][cin][cout]:
// fwd[co][t][ci] (ci < cin_pad, zero beyond cin) and, if dgr != NULL, the
// flipped transpose dgr[ci][t][co] = w[8 - t][ci][co].
hipError_t launch_pack_weights(const float* w, int cin, int cin_pad, int cout, bf16_t* fwd,
                               bf16_t* dgr, hipStream_t s);
// Adam (fp32): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2; p -= lr mhat / (sqrt(vhat) + eps).
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, float bc1, float bc2, hipStream_t s);
// Warm-start fallback: fit the Eq. (2) model to each predicted field (net_res
// / 4 square grid, px of the net_res x net_res image; geometry xs, ys, zs) at
// the grid points within `radius` px of the pattern centre (FP64 Eq. (3)
// solve); use = misfit / 4 <= threshold (px of that grid).  u_init
// [n][2][N/4][N/4] (px of the N x N pattern, geometry xsN, ysN, zsN) = 0 if
// not use, else the fitted model's field (model_field = 1) or the predicted
// field resampled to the N / 4 grid (N = net_res: copy; 2 net_res:
// prolongation; net_res / 2: restriction); misfit[i] = RMS endpoint misfit
// (px of the network's image), flag[i] = use ? 4 : 8.
hipError_t launch_warm_fit(const float* field, int n, int net_res, double xs, double ys, double zs, double radius,
                           double threshold, int model_field, int N, double xsN, double ysN, double zsN,
                           float* u_init, float* misfit, uint32_t* flag, hipStream_t s);

// Network runner (cnn.hip), for the registration's warm start.
int cnn_max_batch(const ebsd_cnn* c);
bool cnn_ready(const ebsd_cnn* c);
// Pack n <= max_batch normalised pairs and run the forward pass into out
// [n][64][64][2] (x, y) px of the 256 x 256 input, on stream s.  up2 != 0:
// the images are 128 x 128 and are upsampled x2 (bilinear, pixel centres at
// (i - 0.5) / 2) on the way in.
int cnn_forward_from(ebsd_cnn* c, const float* ref_base, int64_t ref_stride, const int32_t* ref_slot,
                     const float* test_base, int64_t test_stride, int n, int up2, float* out, hipStream_t s);

}  // namespace ebsd
