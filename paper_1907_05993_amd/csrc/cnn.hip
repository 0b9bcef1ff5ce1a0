// Warm-start network runner: parameters, activations, the forward and
// backward launch sequences, Adam, parameter files, and the ebsd_cnn_* C ABI.
//
// The network predicts the demons field at the coarsest pyramid level from a
// (reference, test) pair, so that the multi-resolution iteration of section 1
// of arXiv:1907.05993 can start from it instead of from zero.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/ebsd.h"
#include "cnn_internal.h"
#include "ebsd_internal.h"

using namespace ebsd;

namespace {

struct LayerDef {
    int cin, cinp, cout, lvl;  // lvl: resolution level (input size / 2^lvl)
};
// c1a c1b c2a c2b c3a c3b c4a c4b d1 d2
constexpr LayerDef kLayers[10] = {{2, 8, 32, 0},    {32, 32, 32, 0},    {32, 32, 64, 1},
                                  {64, 64, 64, 1},  {64, 64, 128, 2},   {128, 128, 128, 2},
                                  {128, 128, 256, 3}, {256, 256, 256, 3}, {384, 384, 128, 2},
                                  {128, 128, 128, 2}};
constexpr int64_t kNumParams = EBSD_CNN_PARAMS;
constexpr int kRes = 256, kHeadC = 128, kCatC = 384;
constexpr int64_t kPixPerPair = (int64_t)kRes * kRes;  // buffers hold up to 256 x 256 per pair
constexpr int kMaxBatch = 4096;

}  // namespace

struct ebsd_cnn {
    int device = 0;
    int max_batch = 0;
    float* params = nullptr;  // fp32 masters, flat
    float* grads = nullptr;
    float* adam_m = nullptr;
    float* adam_v = nullptr;
    int64_t step = 0;
    bool have_params = false;
    bool packed = false;
    bool fused = true;  // inference: fused kernels (equal bit for bit to the per-layer ones)
    int64_t off_w[10], off_b[10], off_hw, off_hb;
    bf16_t* wf[10] = {};
    bf16_t* wd[10] = {};
    // activations (bf16 NHWC)
    bf16_t *x0 = nullptr, *a1a = nullptr, *e1 = nullptr, *p1 = nullptr, *a2a = nullptr, *e2 = nullptr,
           *p2 = nullptr, *a3a = nullptr, *cat = nullptr, *p3 = nullptr, *a4a = nullptr, *e4 = nullptr,
           *a5 = nullptr, *a6 = nullptr;
    float* out = nullptr;   // [max_batch][64][64][2]
    float* norm = nullptr;  // [2][max_batch][256 * 256] normalised inputs of the standalone entries
    // backward (allocated by the first training step)
    bool have_bwd = false;
    float *gA = nullptr, *gB = nullptr, *gC = nullptr;
    bf16_t* dz = nullptr;
    float* part = nullptr;   // weight-gradient partial sums
    float* bpart = nullptr;  // bias / head / loss partial sums
    float* part2 = nullptr;  // chunk sums of the column reductions
    int64_t part2_floats = 0;
    float* dloss = nullptr;
    std::vector<void*> allocs;
};

namespace {

struct DevGuard {
    int prev = -1;
    bool ok = false;
    explicit DevGuard(int d)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(d) == hipSuccess;
    }
    ~DevGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

template <class T>
bool dalloc(ebsd_cnn* c, T** p, int64_t elems)
{
    void* q = nullptr;
    if (hipMalloc(&q, (size_t)elems * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    try {
        c->allocs.push_back(q);
    } catch (const std::bad_alloc&) {
        (void)hipFree(q);
        return false;
    }
    *p = static_cast<T*>(q);
    return true;
}

void free_all(ebsd_cnn* c)
{
    for (void* p : c->allocs) (void)hipFree(p);
    c->allocs.clear();
}

void layout(ebsd_cnn* c)
{
    int64_t o = 0;
    for (int l = 0; l < 10; l++) {
        c->off_w[l] = o;
        o += 9LL * kLayers[l].cin * kLayers[l].cout;
        c->off_b[l] = o;
        o += kLayers[l].cout;
    }
    c->off_hw = o;
    o += 2 * kHeadC;
    c->off_hb = o;
}

int64_t px(int res) { return (int64_t)res * res; }

bool alloc_forward(ebsd_cnn* c)
{
    const int64_t n = c->max_batch;
    bool ok = dalloc(c, &c->params, kNumParams) && dalloc(c, &c->x0, n * px(256) * 8) &&
              dalloc(c, &c->a1a, n * px(256) * 32) && dalloc(c, &c->e1, n * px(256) * 32) &&
              dalloc(c, &c->p1, n * px(128) * 32) && dalloc(c, &c->a2a, n * px(128) * 64) &&
              dalloc(c, &c->e2, n * px(128) * 64) && dalloc(c, &c->p2, n * px(64) * 64) &&
              dalloc(c, &c->a3a, n * px(64) * 128) && dalloc(c, &c->cat, n * px(64) * kCatC) &&
              dalloc(c, &c->p3, n * px(32) * 128) && dalloc(c, &c->a4a, n * px(32) * 256) &&
              dalloc(c, &c->e4, n * px(32) * 256) && dalloc(c, &c->a5, n * px(64) * 128) &&
              dalloc(c, &c->a6, n * px(64) * 128) && dalloc(c, &c->out, n * px(64) * 2) &&
              dalloc(c, &c->norm, 2 * n * px(256));
    for (int l = 0; ok && l < 10; l++) {
        ok = dalloc(c, &c->wf[l], 9LL * kLayers[l].cinp * kLayers[l].cout);
        if (ok && l > 0) ok = dalloc(c, &c->wd[l], 9LL * kLayers[l].cin * kLayers[l].cout);
    }
    if (ok) ok = hipMemset(c->params, 0, kNumParams * sizeof(float)) == hipSuccess;
    return ok;
}

int64_t wgrad_part_floats(int n)
{
    int64_t mx = 0;
    for (int l = 0; l < 10; l++) {
        const LayerDef& d = kLayers[l];
        int tps;
        const int sp = wgrad_splits(n, kRes >> d.lvl, kRes >> d.lvl, d.cinp, d.cout, &tps);
        const int64_t f = (int64_t)sp * 9 * d.cin * d.cout;
        if (f > mx) mx = f;
    }
    return mx;
}

bool alloc_backward(ebsd_cnn* c)
{
    if (c->have_bwd) return true;
    DeviceWideLock lk(capture_mutex());
    const int64_t n = c->max_batch;
    const int64_t g = n * px(256) * 32;  // largest gradient tensor
    const int64_t bp = (int64_t)mask_blocks(n * px(256), 32) * 32;
    c->part2_floats = 1600000 + 128 * n;
    bool ok = dalloc(c, &c->grads, kNumParams) && dalloc(c, &c->adam_m, kNumParams) &&
              dalloc(c, &c->adam_v, kNumParams) && dalloc(c, &c->gA, g) && dalloc(c, &c->gB, g) &&
              dalloc(c, &c->gC, n * px(64) * 128) && dalloc(c, &c->dz, g) &&
              dalloc(c, &c->part, wgrad_part_floats(c->max_batch)) &&
              dalloc(c, &c->bpart, bp > (int64_t)head_blocks(n * px(64)) * 258 ? bp
                                                                               : (int64_t)head_blocks(n * px(64)) * 258) &&
              dalloc(c, &c->dloss, 1) && dalloc(c, &c->part2, c->part2_floats);
    if (ok) ok = hipMemset(c->grads, 0, kNumParams * sizeof(float)) == hipSuccess &&
                 hipMemset(c->adam_m, 0, kNumParams * sizeof(float)) == hipSuccess &&
                 hipMemset(c->adam_v, 0, kNumParams * sizeof(float)) == hipSuccess;
    c->have_bwd = ok;
    return ok;
}

hipError_t pack_weights(ebsd_cnn* c, hipStream_t s)
{
    if (c->packed) return hipSuccess;
    for (int l = 0; l < 10; l++) {
        const LayerDef& d = kLayers[l];
        hipError_t e = launch_pack_weights(c->params + c->off_w[l], d.cin, d.cinp, d.cout, c->wf[l], c->wd[l], s);
        if (e != hipSuccess) return e;
    }
    c->packed = true;
    return hipSuccess;
}

hipError_t conv_fwd(ebsd_cnn* c, int l, int n, int H, int W, const bf16_t* x, bf16_t* out, int out_cs,
                    int out_co, hipStream_t s, int mode = 0, bf16_t* out2 = nullptr, int out2_cs = 0,
                    const bf16_t* x2 = nullptr, int c2 = 0)
{
    const LayerDef& d = kLayers[l];
    ConvArgs a;
    a.x = x;
    a.w = c->wf[l];
    a.bias = c->params + c->off_b[l];
    a.out = out;
    a.n = n;
    a.H = H >> d.lvl;
    a.W = W >> d.lvl;
    a.Cin = d.cinp;
    a.Cout = d.cout;
    a.mode = mode;
    a.out_cs = out_cs;
    a.out_co = out_co;
    a.out2 = out2;
    a.out2_cs = out2_cs;
    a.x2 = x2;
    a.c2 = c2;
    a.lds_dma = c->fused ? 1 : 0;  // the per-layer setting (tests) keeps k_conv3x3 throughout
    return launch_conv3x3(a, s);
}

// Forward from the packed input x0 (n <= max_batch pairs of H x W) to out
// [n][H/4][W/4][2].  infer: the two encoder convolutions whose outputs are
// only pooled write the pooled activations directly (the training step keeps
// them for the pooling's backward pass).
hipError_t forward(ebsd_cnn* c, int n, int H, int W, float* out, hipStream_t s, bool infer = false)
{
    hipError_t e = pack_weights(c, s);
#define CK(x)                          \
    do {                               \
        if (e != hipSuccess) return e; \
        e = (x);                       \
    } while (0)
    const int H1 = H / 2, W1 = W / 2, H2 = H / 4, W2 = W / 4, H3 = H / 8, W3 = W / 8;
    if (infer && c->fused) {
        CK(launch_conv_stem(c->x0, c->wf[0], c->params + c->off_b[0], c->wf[1], c->params + c->off_b[1], n, H, W,
                            c->p1, s));
    } else if (infer) {
        CK(conv_fwd(c, 0, n, H, W, c->x0, c->a1a, 32, 0, s));
        CK(conv_fwd(c, 1, n, H, W, c->a1a, c->p1, 32, 0, s, 2));
    } else {
        CK(conv_fwd(c, 0, n, H, W, c->x0, c->a1a, 32, 0, s));
        CK(conv_fwd(c, 1, n, H, W, c->a1a, c->e1, 32, 0, s));
        CK(launch_maxpool(c->e1, n, H, W, 32, 32, 0, c->p1, s));
    }
    CK(conv_fwd(c, 2, n, H, W, c->p1, c->a2a, 64, 0, s));
    if (infer) {
        CK(conv_fwd(c, 3, n, H, W, c->a2a, c->p2, 64, 0, s, 2));
    } else {
        CK(conv_fwd(c, 3, n, H, W, c->a2a, c->e2, 64, 0, s));
        CK(launch_maxpool(c->e2, n, H1, W1, 64, 64, 0, c->p2, s));
    }
    CK(conv_fwd(c, 4, n, H, W, c->p2, c->a3a, 128, 0, s));
    const bool fuse = infer && c->fused;
    if (fuse) {  // e3 into channels 256..383 of cat and, pooled, into p3
        CK(conv_fwd(c, 5, n, H, W, c->a3a, c->cat, kCatC, 256, s, 3, c->p3, 128));
    } else {
        CK(conv_fwd(c, 5, n, H, W, c->a3a, c->cat, kCatC, 256, s));  // e3 = channels 256..383 of cat
        CK(launch_maxpool(c->cat, n, H2, W2, 128, kCatC, 256, c->p3, s));
    }
    CK(conv_fwd(c, 6, n, H, W, c->p3, c->a4a, 256, 0, s));
    CK(conv_fwd(c, 7, n, H, W, c->a4a, c->e4, 256, 0, s));
    if (fuse) {  // d1 reads channels 0..255 (e4 upsampled) from e4 itself
        CK(conv_fwd(c, 8, n, H, W, c->cat, c->a5, 128, 0, s, 0, nullptr, 0, c->e4, 256));
    } else {
        CK(launch_upsample_into(c->e4, n, H3, W3, 256, c->cat, kCatC, s));
        CK(conv_fwd(c, 8, n, H, W, c->cat, c->a5, 128, 0, s));
    }
    CK(conv_fwd(c, 9, n, H, W, c->a5, c->a6, 128, 0, s));
    CK(launch_head_fwd(c->a6, (int64_t)n * H2 * W2, kHeadC, c->params + c->off_hw, c->params + c->off_hb, out,
                       s));
    return e;
}

// Gradient through layer l given the fp32 gradient g of its output activation
// act (channel stride act_cs, offset act_co): bias and weight gradients into
// c->grads and, if gin != NULL, the fp32 gradient of its input.
hipError_t layer_back(ebsd_cnn* c, int l, int n, int H0, int W0, const float* g, const bf16_t* act,
                      int act_cs, int act_co, const bf16_t* x, float* gin, hipStream_t s)
{
    const LayerDef& d = kLayers[l];
    const int H = H0 >> d.lvl, W = W0 >> d.lvl;
    const int64_t P = (int64_t)n * H * W;
    hipError_t e = launch_mask_round(g, act, P, d.cout, act_cs, act_co, c->dz, c->bpart, s);
    CK(launch_colsum(c->bpart, mask_blocks(P, d.cout), d.cout, c->grads + c->off_b[l], c->part2, c->part2_floats, s));
    WgradArgs w;
    w.x = x;
    w.dz = c->dz;
    w.part = c->part;
    w.n = n;
    w.H = H;
    w.W = W;
    w.Cin = d.cinp;
    w.Cout = d.cout;
    w.cin_keep = d.cin;
    w.splits = wgrad_splits(n, H, W, d.cinp, d.cout, &w.tiles_per_split);
    CK(launch_wgrad3x3(w, s));
    CK(launch_colsum(c->part, w.splits, 9LL * d.cin * d.cout, c->grads + c->off_w[l], c->part2, c->part2_floats,
                     s));
    if (gin) {
        ConvArgs a;
        a.x = c->dz;
        a.w = c->wd[l];
        a.bias = nullptr;
        a.out = gin;
        a.n = n;
        a.H = H;
        a.W = W;
        a.Cin = d.cout;
        a.Cout = d.cin;
        a.mode = 1;
        a.out_cs = d.cin;
        a.out_co = 0;
        CK(launch_conv3x3(a, s));
    }
    return e;
}

// Backward of the whole network from d(loss)/d(out) = gout [n][64][64][2]:
// every parameter gradient into c->grads.  Gradients of activations move
// through gA, gB and gC (fp32); dz holds the bf16 pre-activation gradient.
hipError_t backward(ebsd_cnn* c, int n, int H, int W, const float* gout, hipStream_t s)
{
    const int H1 = H / 2, W1 = W / 2, H2 = H / 4, W2 = W / 4, H3 = H / 8, W3 = W / 8;
    const int64_t P2 = (int64_t)n * H2 * W2;
    hipError_t e = launch_head_back(c->a6, gout, P2, kHeadC, c->params + c->off_hw, c->gA, c->bpart, s);
    CK(launch_colsum(c->bpart, head_blocks(P2), 2 * kHeadC + 2, c->grads + c->off_hw, c->part2, c->part2_floats, s));
    CK(layer_back(c, 9, n, H, W, c->gA, c->a6, 128, 0, c->a5, c->gB, s));         // d2 -> g(a5)
    CK(layer_back(c, 8, n, H, W, c->gB, c->a5, 128, 0, c->cat, c->gA, s));        // d1 -> g(cat)
    CK(launch_upsample_back(c->gA, n, H3, W3, 256, kCatC, c->gB, s));             // g(e4)
    CK(layer_back(c, 7, n, H, W, c->gB, c->e4, 256, 0, c->a4a, c->gC, s));        // c4b -> g(a4a)
    CK(layer_back(c, 6, n, H, W, c->gC, c->a4a, 256, 0, c->p3, c->gB, s));        // c4a -> g(p3)
    CK(launch_maxpool_back(c->gB, c->cat, n, H2, W2, 128, kCatC, 256, c->gA, kCatC, 256, c->gC, s));  // g(e3)
    CK(layer_back(c, 5, n, H, W, c->gC, c->cat, kCatC, 256, c->a3a, c->gA, s));   // c3b -> g(a3a)
    CK(layer_back(c, 4, n, H, W, c->gA, c->a3a, 128, 0, c->p2, c->gB, s));        // c3a -> g(p2)
    CK(launch_maxpool_back(c->gB, c->e2, n, H1, W1, 64, 64, 0, nullptr, 0, 0, c->gA, s));  // g(e2)
    CK(layer_back(c, 3, n, H, W, c->gA, c->e2, 64, 0, c->a2a, c->gB, s));         // c2b -> g(a2a)
    CK(layer_back(c, 2, n, H, W, c->gB, c->a2a, 64, 0, c->p1, c->gA, s));         // c2a -> g(p1)
    CK(launch_maxpool_back(c->gA, c->e1, n, H, W, 32, 32, 0, nullptr, 0, 0, c->gB, s));  // g(e1)
    CK(layer_back(c, 1, n, H, W, c->gB, c->e1, 32, 0, c->a1a, c->gA, s));         // c1b -> g(a1a)
    CK(layer_back(c, 0, n, H, W, c->gA, c->a1a, 32, 0, c->x0, nullptr, s));       // c1a
    return e;
}
#undef CK

int check_net(const ebsd_cnn* c) { return c ? EBSD_OK : EBSD_EINVAL; }

// Network input sizes: H a multiple of 64 and W a multiple of 256 (the
// convolution tiles at 1/8 resolution), at most 256 x 256 px per pair.
bool shape_ok(int H, int W) { return H > 0 && W > 0 && H % 64 == 0 && W % 256 == 0 && (int64_t)H * W <= kPixPerPair; }

int normalize_pack(ebsd_cnn* c, const float* ref, const float* test, int n, int H, int W, hipStream_t s)
{
    const int64_t hw = (int64_t)H * W;
    float* nr = c->norm;
    float* nt = c->norm + (int64_t)c->max_batch * kPixPerPair;
    if (launch_stage_normalize(ref, n, hw, nr, nullptr, s) != hipSuccess) return EBSD_EDEVICE;
    if (launch_stage_normalize(test, n, hw, nt, nullptr, s) != hipSuccess) return EBSD_EDEVICE;
    if (launch_pack_input(nr, hw, nullptr, nt, hw, n, H, W, c->x0, s) != hipSuccess) return EBSD_EDEVICE;
    return EBSD_OK;
}

}  // namespace

// ---- internal interface used by the registration entry points ---------------------

namespace ebsd {

int cnn_max_batch(const ebsd_cnn* c) { return c ? c->max_batch : 0; }
bool cnn_ready(const ebsd_cnn* c) { return c && c->have_params; }

// Pack n <= max_batch normalised pairs (see launch_pack_input) and run the
// forward pass into out [n][64][64][2].
int cnn_forward_from(ebsd_cnn* c, const float* ref_base, int64_t ref_stride, const int32_t* ref_slot,
                     const float* test_base, int64_t test_stride, int n, int up2, float* out, hipStream_t s)
{
    DevGuard g(c->device);
    if (!g.ok) return EBSD_EDEVICE;
    const hipError_t e = up2 ? launch_pack_input_up2(ref_base, ref_stride, ref_slot, test_base, test_stride, n,
                                                     kRes / 2, kRes / 2, c->x0, s)
                             : launch_pack_input(ref_base, ref_stride, ref_slot, test_base, test_stride, n, kRes,
                                                 kRes, c->x0, s);
    if (e != hipSuccess) return EBSD_EDEVICE;
    return forward(c, n, kRes, kRes, out, s, true) == hipSuccess ? EBSD_OK : EBSD_EDEVICE;
}

}  // namespace ebsd

// ---- C ABI --------------------------------------------------------------------------

extern "C" {

int64_t ebsd_cnn_num_params(void) { return kNumParams; }

int ebsd_cnn_create(int device, int32_t max_batch, ebsd_cnn** out)
{
    if (!out || max_batch < 1 || max_batch > kMaxBatch) return EBSD_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        return EBSD_EDEVICE;
    }
    DevGuard g(device);
    if (!g.ok) return EBSD_EDEVICE;
    DeviceWideLock lk(capture_mutex());
    ebsd_cnn* c = new (std::nothrow) ebsd_cnn();
    if (!c) return EBSD_ENOMEM;
    c->device = device;
    c->max_batch = max_batch;
    layout(c);
    if (!alloc_forward(c)) {
        free_all(c);
        delete c;
        return EBSD_ENOMEM;
    }
    *out = c;
    return EBSD_OK;
}

int ebsd_cnn_destroy(ebsd_cnn* c)
{
    if (!c) return EBSD_OK;
    {
        DevGuard g(c->device);
        DeviceWideLock lk(capture_mutex());
        (void)hipDeviceSynchronize();
        free_all(c);
    }
    delete c;
    return EBSD_OK;
}

int ebsd_cnn_set_params(ebsd_cnn* c, const float* host, int64_t n)
{
    if (!c || !host || n != kNumParams) return EBSD_EINVAL;
    DevGuard g(c->device);
    DeviceWideLock lk(capture_mutex());
    if (!g.ok) return EBSD_EDEVICE;
    if (hipDeviceSynchronize() != hipSuccess) return EBSD_EDEVICE;
    if (hipMemcpy(c->params, host, kNumParams * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
        return EBSD_EDEVICE;
    c->have_params = true;
    c->packed = false;
    c->step = 0;
    if (c->have_bwd) {
        if (hipMemset(c->adam_m, 0, kNumParams * sizeof(float)) != hipSuccess ||
            hipMemset(c->adam_v, 0, kNumParams * sizeof(float)) != hipSuccess)
            return EBSD_EDEVICE;
    }
    return EBSD_OK;
}

int ebsd_cnn_get_params(const ebsd_cnn* c, float* host, int64_t n)
{
    if (!c || !host || n != kNumParams) return EBSD_EINVAL;
    DevGuard g(c->device);
    DeviceWideLock lk(capture_mutex());
    if (!g.ok || hipDeviceSynchronize() != hipSuccess) return EBSD_EDEVICE;
    return hipMemcpy(host, c->params, kNumParams * sizeof(float), hipMemcpyDeviceToHost) == hipSuccess
               ? EBSD_OK
               : EBSD_EDEVICE;
}

int ebsd_cnn_get_grads(const ebsd_cnn* c, float* host, int64_t n)
{
    if (!c || !host || n != kNumParams || !c->have_bwd) return EBSD_EINVAL;
    DevGuard g(c->device);
    DeviceWideLock lk(capture_mutex());
    if (!g.ok || hipDeviceSynchronize() != hipSuccess) return EBSD_EDEVICE;
    return hipMemcpy(host, c->grads, kNumParams * sizeof(float), hipMemcpyDeviceToHost) == hipSuccess
               ? EBSD_OK
               : EBSD_EDEVICE;
}

int ebsd_cnn_load(ebsd_cnn* c, const char* path)
{
    if (!c || !path) return EBSD_EINVAL;
    std::vector<float> buf;
    try {
        buf.resize((size_t)kNumParams);
    } catch (const std::bad_alloc&) {
        return EBSD_ENOMEM;
    }
    FILE* f = fopen(path, "rb");
    if (!f) return EBSD_EIO;
    char magic[8];
    int64_t cnt = 0;
    bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, "EBSDCNN1", 8) == 0 &&
              fread(&cnt, sizeof(cnt), 1, f) == 1 && cnt == kNumParams;
    if (ok) {
        ok = fread(buf.data(), sizeof(float), (size_t)kNumParams, f) == (size_t)kNumParams;
    }
    fclose(f);
    if (!ok) return EBSD_EIO;
    for (float v : buf)
        if (!std::isfinite(v)) return EBSD_EIO;
    return ebsd_cnn_set_params(c, buf.data(), kNumParams);
}

int ebsd_cnn_save(const ebsd_cnn* c, const char* path)
{
    if (!c || !path) return EBSD_EINVAL;
    std::vector<float> buf;
    try {
        buf.resize((size_t)kNumParams);
    } catch (const std::bad_alloc&) {
        return EBSD_ENOMEM;
    }
    int e = ebsd_cnn_get_params(c, buf.data(), kNumParams);
    if (e != EBSD_OK) return e;
    FILE* f = fopen(path, "wb");
    if (!f) return EBSD_EIO;
    const int64_t cnt = kNumParams;
    bool ok = fwrite("EBSDCNN1", 1, 8, f) == 8 && fwrite(&cnt, sizeof(cnt), 1, f) == 1 &&
              fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    ok = (fclose(f) == 0) && ok;
    return ok ? EBSD_OK : EBSD_EIO;
}

int ebsd_cnn_forward(ebsd_cnn* c, const float* ref, const float* test, int32_t n, int32_t H, int32_t W,
                     float* out, void* stream)
{
    if (!c || !ref || !test || !out || n < 0 || n > c->max_batch) return EBSD_EINVAL;
    if (!shape_ok(H, W)) return EBSD_ESHAPE;
    if (!c->have_params) return EBSD_ENOMODEL;
    if (n == 0) return EBSD_OK;
    DevGuard g(c->device);
    if (!g.ok) return EBSD_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int e = normalize_pack(c, ref, test, n, H, W, s);
    if (e != EBSD_OK) return e;
    return forward(c, n, H, W, out, s, true) == hipSuccess ? EBSD_OK : EBSD_EDEVICE;
}

int ebsd_cnn_train_step(ebsd_cnn* c, const float* ref, const float* test, const float* label, int32_t n,
                        int32_t H, int32_t W, float lr, int32_t update, float* loss, void* stream)
{
    if (!c || !ref || !test || !label || n < 1 || n > c->max_batch) return EBSD_EINVAL;
    if (!(lr >= 0.0f) || !std::isfinite(lr)) return EBSD_EINVAL;
    if (!shape_ok(H, W)) return EBSD_ESHAPE;
    if (!c->have_params) return EBSD_ENOMODEL;
    DevGuard g(c->device);
    if (!g.ok) return EBSD_EDEVICE;
    if (!alloc_backward(c)) return EBSD_ENOMEM;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int e = normalize_pack(c, ref, test, n, H, W, s);
    if (e != EBSD_OK) return e;
    const int64_t P64 = (int64_t)n * (H / 4) * (W / 4);
    if (forward(c, n, H, W, c->out, s) != hipSuccess) return EBSD_EDEVICE;
    // the loss gradient replaces the output in place
    if (launch_loss(c->out, label, P64, c->out, c->bpart, s) != hipSuccess) return EBSD_EDEVICE;
    if (launch_colsum(c->bpart, loss_blocks(P64), 1, c->dloss, c->part2, c->part2_floats, s) != hipSuccess)
        return EBSD_EDEVICE;
    // read the loss before the backward pass reuses bpart
    float lsum = 0.0f;
    if (hipMemcpyAsync(&lsum, c->dloss, sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return EBSD_EDEVICE;
    if (backward(c, n, H, W, c->out, s) != hipSuccess) return EBSD_EDEVICE;
    if (update) {
        c->step++;
        const double b1 = 0.9, b2 = 0.999;
        const float bc1 = (float)(1.0 - std::pow(b1, (double)c->step));
        const float bc2 = (float)(1.0 - std::pow(b2, (double)c->step));
        if (launch_adam(c->params, c->grads, c->adam_m, c->adam_v, kNumParams, lr, (float)b1, (float)b2, 1e-8f,
                        bc1, bc2, s) != hipSuccess)
            return EBSD_EDEVICE;
        c->packed = false;
    }
    if (hipStreamSynchronize(s) != hipSuccess) return EBSD_EDEVICE;
    if (loss) *loss = lsum / (float)P64;
    return EBSD_OK;
}

int ebsd_cnn_get_optimizer(const ebsd_cnn* c, float* m, float* v, int64_t n, int64_t* step)
{
    if (!c || n != kNumParams) return EBSD_EINVAL;
    if (step) *step = c->step;
    DevGuard g(c->device);
    DeviceWideLock lk(capture_mutex());
    if (!g.ok || hipDeviceSynchronize() != hipSuccess) return EBSD_EDEVICE;
    for (int k = 0; k < 2; k++) {
        float* dst = k == 0 ? m : v;
        if (!dst) continue;
        const float* src = k == 0 ? c->adam_m : c->adam_v;
        if (!c->have_bwd) {
            std::memset(dst, 0, kNumParams * sizeof(float));
        } else if (hipMemcpy(dst, src, kNumParams * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess) {
            return EBSD_EDEVICE;
        }
    }
    return EBSD_OK;
}

int ebsd_cnn_set_optimizer(ebsd_cnn* c, const float* m, const float* v, int64_t n, int64_t step)
{
    if (!c || !m || !v || n != kNumParams || step < 0) return EBSD_EINVAL;
    DevGuard g(c->device);
    if (!g.ok) return EBSD_EDEVICE;
    if (!alloc_backward(c)) return EBSD_ENOMEM;
    DeviceWideLock lk(capture_mutex());
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(c->adam_m, m, kNumParams * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->adam_v, v, kNumParams * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
        return EBSD_EDEVICE;
    c->step = step;
    return EBSD_OK;
}

int ebsd_cnn_set_fusion(ebsd_cnn* c, int32_t on)
{
    if (!c || (on != 0 && on != 1)) return EBSD_EINVAL;
    c->fused = on != 0;
    return EBSD_OK;
}

int ebsd_cnn_reset_optimizer(ebsd_cnn* c)
{
    if (!c) return EBSD_EINVAL;
    c->step = 0;
    if (!c->have_bwd) return EBSD_OK;
    DevGuard g(c->device);
    DeviceWideLock lk(capture_mutex());
    if (!g.ok || hipDeviceSynchronize() != hipSuccess) return EBSD_EDEVICE;
    if (hipMemset(c->adam_m, 0, kNumParams * sizeof(float)) != hipSuccess ||
        hipMemset(c->adam_v, 0, kNumParams * sizeof(float)) != hipSuccess)
        return EBSD_EDEVICE;
    return EBSD_OK;
}

}  // extern "C"

// ---- single-kernel entry points (convolution kernels in isolation) -----------------

namespace {

struct TempBuf {
    void* p = nullptr;
    ~TempBuf()
    {
        if (p) (void)hipFree(p);
    }
};

bool conv_shape_ok(int n, int H, int W, int Cin, int Cout)
{
    return n > 0 && n <= kMaxBatch && conv3x3_supported(H, W, Cin, Cout) && Cin <= 512 && Cout <= 512 &&
           (int64_t)H * W <= 1 << 20;
}

}  // namespace

extern "C" {

int ebsd_stage_conv3x3(const uint16_t* x, int32_t n, int32_t H, int32_t W, int32_t Cin, const float* w,
                       const float* bias, int32_t Cout, int32_t mode, void* out, void* stream)
{
    if (!x || !w || !out || (mode != 0 && mode != 1) || (mode == 0 && !bias)) return EBSD_EINVAL;
    if (!conv_shape_ok(n, H, W, Cin, Cout)) return EBSD_ESHAPE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    DeviceWideLock lk(capture_mutex());
    TempBuf wf;
    if (hipMalloc(&wf.p, sizeof(bf16_t) * 9 * Cin * Cout) != hipSuccess) return EBSD_ENOMEM;
    if (launch_pack_weights(w, Cin, Cin, Cout, static_cast<bf16_t*>(wf.p), nullptr, s) != hipSuccess)
        return EBSD_EDEVICE;
    ConvArgs a;
    a.x = x;
    a.w = static_cast<bf16_t*>(wf.p);
    a.bias = bias;
    a.out = out;
    a.n = n;
    a.H = H;
    a.W = W;
    a.Cin = Cin;
    a.Cout = Cout;
    a.mode = mode;
    a.out_cs = Cout;
    a.out_co = 0;
    if (launch_conv3x3(a, s) != hipSuccess) return EBSD_EDEVICE;
    return hipStreamSynchronize(s) == hipSuccess ? EBSD_OK : EBSD_EDEVICE;
}

int ebsd_stage_conv3x3_dgrad(const uint16_t* dz, int32_t n, int32_t H, int32_t W, int32_t Cout, const float* w,
                             int32_t Cin, float* dx, void* stream)
{
    if (!dz || !w || !dx) return EBSD_EINVAL;
    if (!conv_shape_ok(n, H, W, Cout, Cin)) return EBSD_ESHAPE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    DeviceWideLock lk(capture_mutex());
    TempBuf wf, wd;
    if (hipMalloc(&wf.p, sizeof(bf16_t) * 9 * Cin * Cout) != hipSuccess ||
        hipMalloc(&wd.p, sizeof(bf16_t) * 9 * Cin * Cout) != hipSuccess)
        return EBSD_ENOMEM;
    if (launch_pack_weights(w, Cin, Cin, Cout, static_cast<bf16_t*>(wf.p), static_cast<bf16_t*>(wd.p), s) !=
        hipSuccess)
        return EBSD_EDEVICE;
    ConvArgs a;
    a.x = dz;
    a.w = static_cast<bf16_t*>(wd.p);
    a.bias = nullptr;
    a.out = dx;
    a.n = n;
    a.H = H;
    a.W = W;
    a.Cin = Cout;
    a.Cout = Cin;
    a.mode = 1;
    a.out_cs = Cin;
    a.out_co = 0;
    if (launch_conv3x3(a, s) != hipSuccess) return EBSD_EDEVICE;
    return hipStreamSynchronize(s) == hipSuccess ? EBSD_OK : EBSD_EDEVICE;
}

int ebsd_stage_conv3x3_wgrad(const uint16_t* x, const uint16_t* dz, int32_t n, int32_t H, int32_t W, int32_t Cin,
                             int32_t Cout, float* dw, void* stream)
{
    if (!x || !dz || !dw) return EBSD_EINVAL;
    if (!conv_shape_ok(n, H, W, Cin, Cout) || H % 4 != 0) return EBSD_ESHAPE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    WgradArgs a;
    a.x = x;
    a.dz = dz;
    a.n = n;
    a.H = H;
    a.W = W;
    a.Cin = Cin;
    a.Cout = Cout;
    a.cin_keep = Cin;
    a.splits = wgrad_splits(n, H, W, Cin, Cout, &a.tiles_per_split);
    DeviceWideLock lk(capture_mutex());
    TempBuf part, tmp;
    const int64_t tmp_floats = (int64_t)((a.splits + 511) / 512) * 9 * Cin * Cout;
    if (hipMalloc(&part.p, sizeof(float) * (size_t)a.splits * 9 * Cin * Cout) != hipSuccess ||
        hipMalloc(&tmp.p, sizeof(float) * (size_t)tmp_floats) != hipSuccess)
        return EBSD_ENOMEM;
    a.part = static_cast<float*>(part.p);
    if (launch_wgrad3x3(a, s) != hipSuccess) return EBSD_EDEVICE;
    if (launch_colsum(a.part, a.splits, 9LL * Cin * Cout, dw, static_cast<float*>(tmp.p), tmp_floats, s) != hipSuccess)
        return EBSD_EDEVICE;
    return hipStreamSynchronize(s) == hipSuccess ? EBSD_OK : EBSD_EDEVICE;
}

}  // extern "C"
