// C ABI of the gfx950 demons-based HR-EBSD library (declared in include/ebsd.h).
//
// Host side: argument validation (before anything is enqueued), size
// bucketing, workspace management and the launch sequence of the whole path
// (arXiv:1907.05993: multi-resolution demons of section 1 / Eq. (1), shifts at
// the ROI centres and the Eq. (2)-(3) solve of section 2, polar rotation of
// Eq. (4)-(5), remap and second-pass cross-correlation, Eq. (12)).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <fstream>
#include <sstream>
#include <string>
#include <new>
#include <utility>
#include <vector>

#include <unistd.h>

#include "../../include/ebsd.h"
#include "ebsd_internal.h"
#include "cnn_internal.h"

using namespace ebsd;

struct ebsd_handle {
    ebsd_params p;
    int device;
    float taps[2 * kMaxRadius + 1];
    int radius;
    char* ws = nullptr;  // device workspace
    size_t ws_bytes = 0;
    char* pin = nullptr;  // pinned staging for descriptors
    size_t pin_bytes = 0;
    hipEvent_t pin_free = nullptr;  // recorded after the last upload from `pin`
    bool pin_pending = false;
    // timing: ev[0] call start, ev[1] call end, ev[2 + 2l] / ev[3 + 2l] level l
    bool timing = false;
    bool timed_call = false;
    int timed_levels = 0;
    hipEvent_t ev[2 + 2 * EBSD_MAX_LEVELS] = {};
    // strip height of the row-marching demons kernel per level size (h, w),
    // from ebsd_autotune or the tuning cache file; default kDefaultStripTY
    std::map<std::pair<int, int>, int> strip_ty;
    // strip height of the two-iterations-per-launch kernel per level size; a
    // level size absent here (or 0) runs one iteration per launch
    std::map<std::pair<int, int>, int> fused_ty;
    // batch size each level size's strip height and two-iteration strip
    // height were tuned on (absent: forced or read from the cache file); kept
    // apart so that forcing one of them leaves the other's record in place
    std::map<std::pair<int, int>, int> tuned_nb_strip, tuned_nb_fused;
    std::string tune_cache;  // EBSD_TUNE_CACHE at create time (may be empty)
    // captured launch sequences per bucket configuration (replayed with
    // hipGraphLaunch); the capture itself runs on a private stream
    bool graphs = true;
    bool resident = true;  // levels of at most 64 x 64 px iterate in one launch
    hipStream_t cap_stream = nullptr;
    std::map<std::string, hipGraphExec_t> graph_cache;
    // With a tolerance, a level's launches go out in chunks of gate_chunk; after
    // each chunk a kernel writes the number of pairs still iterating into
    // pinned host memory, and the host stops issuing chunks once a chunk has
    // left none.  It reads chunk c - 2's count while chunks c - 1 and c are
    // queued, so the device never waits for the host.  0: every launch of
    // every level is issued and the call never waits on the stream.
    int gate_chunk = 8;
    int32_t* gate_host = nullptr;  // pinned, device-visible [4]
    int32_t* gate_dev = nullptr;   // the same memory as the device addresses it
    hipEvent_t gate_ev[4] = {};
    // launches of the last call per level (summed over size buckets): issued,
    // and the full sequence up to the cap
    int32_t launches_issued[EBSD_MAX_LEVELS] = {};
    int32_t launches_planned[EBSD_MAX_LEVELS] = {};
    // warm-start network (created by ebsd_load_model / ebsd_set_model)
    ebsd_cnn* cnn = nullptr;
};

namespace {

// Strip height of the row-marching kernel for a level: the tuned or forced
// value, else kDefaultStripTY when the batch has enough strips to fill the
// device (>= 2 per compute unit), else the tallest of 32, 16 rows that does,
// or 16 (a small batch is latency-bound: shorter strips, more workgroups).
// A tuned entry is not used for a batch under a quarter of the one it was
// tuned on: the fastest decomposition of a large batch starves a small one
// of workgroups.
bool tuned_applies(const std::map<std::pair<int, int>, int>& rec, int lh, int lw, int nb)
{
    auto it = rec.find(std::make_pair(lh, lw));
    return it == rec.end() || 4 * (int64_t)nb >= it->second;
}

int strip_ty_for(const ebsd_handle* h, int lh, int lw, int nb = 1 << 20)
{
    auto it = h->strip_ty.find(std::make_pair(lh, lw));
    if (it != h->strip_ty.end() && tuned_applies(h->tuned_nb_strip, lh, lw, nb)) return it->second;
    constexpr int kFill = 512;
    for (int ty = kDefaultStripTY; ty > kMinStripTY; ty /= 2)
        if ((int64_t)nb * ((lh + ty - 1) / ty) >= kFill) return ty;
    return kMinStripTY;
}

int fused_ty_for(const ebsd_handle* h, int lh, int lw, int nb = 1 << 20)
{
    if (!rows_cpl(lw) || !tuned_applies(h->tuned_nb_fused, lh, lw, nb)) return 0;
    auto it = h->fused_ty.find(std::make_pair(lh, lw));
    return it == h->fused_ty.end() ? 0 : it->second;
}

// Tuning cache: one line "gfx950 <level h> <level w> <strip height>" per entry.
// Tuning cache: one line "gfx950 <level h> <level w> <strip height> <fused strip height>"
// per level size (fused strip height 0: one iteration per launch).
void load_tune_cache(ebsd_handle* h)
{
    if (h->tune_cache.empty()) return;
    std::ifstream f(h->tune_cache);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string arch;
        int lh = 0, lw = 0, ty = 0, fty = 0;
        if (!(is >> arch >> lh >> lw >> ty) || arch != "gfx950") continue;
        if (!(is >> fty)) fty = 0;
        const auto key = std::make_pair(lh, lw);
        if (strip_ty_ok(lw, ty)) h->strip_ty[key] = ty;
        if (rows2_ty_ok(lw, fty)) h->fused_ty[key] = fty;
        else h->fused_ty.erase(key);
    }
}

// Written to a temporary file in the same folder and renamed over the cache, so
// a handle created meanwhile (here or in another process) reads either the old
// table or the new one, never a partial file; writers in this process take
// turns.  Best effort: a cache that cannot be written is left as it was.
void save_tune_cache(const ebsd_handle* h)
{
    if (h->tune_cache.empty()) return;
    static std::mutex mu;
    std::lock_guard<std::mutex> lk(mu);
    std::ostringstream tmp;
    tmp << h->tune_cache << ".tmp." << (unsigned long)getpid();
    {
        std::ofstream f(tmp.str(), std::ios::trunc);
        for (auto& kv : h->strip_ty)
            f << "gfx950 " << kv.first.first << " " << kv.first.second << " " << kv.second << " "
              << fused_ty_for(h, kv.first.first, kv.first.second) << "\n";
        f.flush();
        if (!f) {
            f.close();
            std::remove(tmp.str().c_str());
            return;
        }
    }
    if (std::rename(tmp.str().c_str(), h->tune_cache.c_str()) != 0) std::remove(tmp.str().c_str());
}

struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Sub-allocation plan inside one buffer.
struct Plan {
    size_t off = 0;
    size_t take(size_t bytes)
    {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    }
};

// A device temporary released when it goes out of scope.
struct DevBuf {
    void* p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
};

int check_params(const ebsd_params* p)
{
    if (!p) return EBSD_EINVAL;
    if (p->struct_size != sizeof(ebsd_params)) return EBSD_EVERSION;
    if (p->levels < 1 || p->levels > EBSD_MAX_LEVELS) return EBSD_EINVAL;
    for (int l = 0; l < p->levels; l++)
        if (p->max_iters[l] < 0 || p->max_iters[l] > 1000000) return EBSD_EINVAL;
    if (!(p->sigma_px >= 0.0f) || !(p->sigma_px <= 1.3f)) return EBSD_EINVAL;
    if (!(p->tol_px >= 0.0f) || !std::isfinite(p->tol_px)) return EBSD_EINVAL;
    if (!std::isfinite(p->pc_x) || !std::isfinite(p->pc_y) || !(p->pc_z > 0.0) ||
        !std::isfinite(p->pc_z))
        return EBSD_EINVAL;
    if (p->n_roi < 5 || p->n_roi > 256) return EBSD_EINVAL;
    if (p->roi_size != 32 && p->roi_size != 64 && p->roi_size != 128 && p->roi_size != 256) return EBSD_EROI;
    if (!(p->roi_radius_frac >= 0.0) || !std::isfinite(p->roi_radius_frac)) return EBSD_EINVAL;
    if (p->window != 0 && p->window != 1) return EBSD_EINVAL;
    if (p->second_pass != 0 && p->second_pass != 1) return EBSD_EINVAL;
    if (p->warm_start < 0 || p->warm_start > 2) return EBSD_EINVAL;
    if (!(p->fallback_residual_px >= 0.0f) || !std::isfinite(p->fallback_residual_px)) return EBSD_EINVAL;
    if (p->remap_interp != 1 && p->remap_interp != 3) return EBSD_EINVAL;
    if (p->xcf_passes < 1 || p->xcf_passes > 16) return EBSD_EINVAL;
    if (p->first_pass != 0 && p->first_pass != 1) return EBSD_EINVAL;
    if (p->first_pass == 1 && p->warm_start != 0) return EBSD_EINVAL;
    if (!(p->bandpass_lo_px >= 0.0f && p->bandpass_lo_px <= 32.0f)) return EBSD_EINVAL;
    if (!(p->bandpass_hi_px >= 0.0f && p->bandpass_hi_px <= 32.0f)) return EBSD_EINVAL;
    if (p->background_static != 0 && p->background_static != 1) return EBSD_EINVAL;
    if (!(p->background_dynamic_px >= 0.0f && p->background_dynamic_px <= 32.0f)) return EBSD_EINVAL;
    return EBSD_OK;
}

// Largest size bucket whose coarse levels run level-resident (one workgroup per
// pair; 256 compute units).
constexpr int kResidentMaxPairs = 256;

// The network's input and output grid: 256 x 256 patterns, 3 pyramid levels.
constexpr int kWarmRes = 256, kWarmLevels = 3;
constexpr int kWarmBatch = 256;  // pairs per network launch sequence

// ROI layout for an H x W pattern (see ebsd_roi_layout in the header).
int roi_layout(const ebsd_params& p, int H, int W, double* cx, double* cy, int32_t* x0, int32_t* y0)
{
    const double xs = p.pc_x * W - 0.5, ys = p.pc_y * H - 0.5;
    const double rho = p.roi_radius_frac * W;
    const int N = p.roi_size;
    const double pi = 3.14159265358979323846;
    int bad = 0;
    for (int j = 0; j < p.n_roi; j++) {
        double px = xs, py = ys;
        if (j > 0) {
            const double a = 2.0 * pi * (double)(j - 1) / (double)(p.n_roi - 1);
            px += rho * std::cos(a);
            py += rho * std::sin(a);
        }
        const int ix = (int)std::floor(px - (N - 1) / 2.0 + 0.5);
        const int iy = (int)std::floor(py - (N - 1) / 2.0 + 0.5);
        if (x0) x0[j] = ix;
        if (y0) y0[j] = iy;
        if (cx) cx[j] = ix + (N - 1) / 2.0;
        if (cy) cy[j] = iy + (N - 1) / 2.0;
        if (ix < 0 || iy < 0 || ix + N > W || iy + N > H) bad = 1;
    }
    return bad ? EBSD_EROI : EBSD_OK;
}

int check_shape(const ebsd_params& p, int H, int W)
{
    if (H <= 0 || W <= 0 || H > 16384 || W > 16384) return EBSD_ESHAPE;
    // the coarsest level (sizes halved, rounding up) must keep 4 x 4 pixels
    int hc = H, wc = W;
    for (int l = 1; l < p.levels; l++) {
        hc = (hc + 1) / 2;
        wc = (wc + 1) / 2;
    }
    if (hc < 4 || wc < 4) return EBSD_ESHAPE;
    if (H < p.roi_size || W < p.roi_size) return EBSD_EROI;
    return roi_layout(p, H, W, nullptr, nullptr, nullptr, nullptr);
}

int check_pairs(const ebsd_params& p, const ebsd_pair* pairs, int n)
{
    if (n < 0 || n > (1 << 24)) return EBSD_EINVAL;
    if (n > 0 && !pairs) return EBSD_EINVAL;
    std::map<int, std::pair<const float*, std::pair<int, int>>> refs;
    for (int i = 0; i < n; i++) {
        const ebsd_pair& q = pairs[i];
        if (!q.ref || !q.test) return EBSD_EINVAL;
        int e = check_shape(p, q.H, q.W);
        if (e) return e;
        if (q.ref_id >= 0) {
            auto it = refs.find(q.ref_id);
            if (it == refs.end())
                refs[q.ref_id] = {q.ref, {q.H, q.W}};
            else if (it->second.first != q.ref || it->second.second.first != q.H ||
                     it->second.second.second != q.W)
                return EBSD_EINVAL;
        }
    }
    return EBSD_OK;
}

int map_err(hipError_t e)
{
    if (e == hipSuccess) return EBSD_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return EBSD_ENOMEM;
    return EBSD_EDEVICE;
}

// Make sure the handle's workspace holds `bytes`.  Growing waits for all
// work on the device, since earlier calls may still be using the old buffer.
void clear_graphs(ebsd_handle* h)
{
    for (auto& kv : h->graph_cache)
        if (kv.second) (void)hipGraphExecDestroy(kv.second);
    h->graph_cache.clear();
}

int ensure_ws(ebsd_handle* h, size_t bytes)
{
    if (bytes <= h->ws_bytes) return EBSD_OK;
    DeviceWideLock lk(capture_mutex());
    if (hipDeviceSynchronize() != hipSuccess) return EBSD_EDEVICE;
    clear_graphs(h);  // captured kernels point into the old workspace
    if (h->ws) (void)hipFree(h->ws);
    h->ws = nullptr;
    h->ws_bytes = 0;
    size_t want = align_up(bytes + bytes / 8, 1 << 20);
    if (hipMalloc(&h->ws, want) != hipSuccess) {
        h->ws = nullptr;
        (void)hipGetLastError();
        return EBSD_ENOMEM;
    }
    h->ws_bytes = want;
    return EBSD_OK;
}

// Pinned staging for descriptor uploads; waits until the previous upload has
// been consumed before the buffer is rewritten.
int ensure_pin(ebsd_handle* h, size_t bytes)
{
    if (h->pin_pending) {
        if (hipEventSynchronize(h->pin_free) != hipSuccess) return EBSD_EDEVICE;
        h->pin_pending = false;
    }
    if (bytes <= h->pin_bytes) return EBSD_OK;
    DeviceWideLock lk(capture_mutex());
    if (h->pin) (void)hipHostFree(h->pin);
    h->pin = nullptr;
    h->pin_bytes = 0;
    size_t want = align_up(bytes * 2, 1 << 16);
    if (hipHostMalloc((void**)&h->pin, want, hipHostMallocDefault) != hipSuccess) {
        h->pin = nullptr;
        (void)hipGetLastError();
        return EBSD_ENOMEM;
    }
    h->pin_bytes = want;
    return EBSD_OK;
}

// Host-side description of one size bucket.
struct HostBucket {
    int H, W;
    std::vector<int> idx;        // caller pair indices
    std::vector<const float*> test_in, ref_in;
    std::vector<int32_t> ref_slot, pair_index;
};

std::vector<HostBucket> make_buckets(const ebsd_pair* pairs, int n)
{
    std::vector<HostBucket> out;
    std::map<std::pair<int, int>, size_t> where;
    for (int i = 0; i < n; i++) {
        auto key = std::make_pair(pairs[i].H, pairs[i].W);
        auto it = where.find(key);
        size_t k;
        if (it == where.end() || out[it->second].idx.size() >= 32000) {
            k = out.size();
            where[key] = k;
            HostBucket hb;
            hb.H = pairs[i].H;
            hb.W = pairs[i].W;
            out.push_back(hb);
        } else {
            k = it->second;
        }
        out[k].idx.push_back(i);
    }
    for (auto& hb : out) {
        std::map<int, int> slot_of_id;
        for (int i : hb.idx) {
            const ebsd_pair& q = pairs[i];
            int slot;
            if (q.ref_id >= 0) {
                auto it = slot_of_id.find(q.ref_id);
                if (it == slot_of_id.end()) {
                    slot = (int)hb.ref_in.size();
                    slot_of_id[q.ref_id] = slot;
                    hb.ref_in.push_back(q.ref);
                } else {
                    slot = it->second;
                }
            } else {
                slot = (int)hb.ref_in.size();
                hb.ref_in.push_back(q.ref);
            }
            hb.test_in.push_back(q.test);
            hb.ref_slot.push_back(slot);
            hb.pair_index.push_back(i);
        }
    }
    return out;
}

enum class Mode { Full, SecondPassOnly };

// Lay out, upload and run one bucket.  `pin_off` is this bucket's slice of
// the pinned staging buffer.
int run_bucket(ebsd_handle* h, const HostBucket& hbk, Mode mode, const float* u_init,
               const double* rfin_in, const ebsd_outputs* out, hipStream_t s, size_t pin_off,
               size_t* pin_used, bool tune_only = false)
{
    const ebsd_params& p = h->p;
    const int nb = (int)hbk.idx.size();
    const int nref = (int)hbk.ref_in.size();
    const int L = mode == Mode::Full ? p.levels : 1;
    const int H = hbk.H, W = hbk.W;
    const int nr = p.n_roi;

    Bucket b;
    std::memset(&b, 0, sizeof b);
    b.nb = nb;
    b.nref = nref;
    b.H = H;
    b.W = W;
    b.L = L;
    int64_t pe = 0;
    int max_units = 1;
    for (int l = 0; l < L; l++) {
        // level sizes halve rounding up (odd sizes keep their last pixel)
        b.lh[l] = l == 0 ? H : (b.lh[l - 1] + 1) / 2;
        b.lw[l] = l == 0 ? W : (b.lw[l - 1] + 1) / 2;
        b.lvl_off[l] = (int32_t)pe;
        pe += (int64_t)b.lh[l] * b.lw[l];
        pe = (pe + 63) / 64 * 64;  // every level 256 B aligned
        max_units = std::max(max_units, demons_units(b.lh[l], b.lw[l], kMinStripTY2));
        if (b.lw[l] > 512) max_units = std::max(max_units, demons_tiles(b.lh[l], b.lw[l]));
    }
    b.pyr_elems = pe;
    b.max_tiles = max_units;
    b.n_roi = nr;
    b.roi_N = p.roi_size;
    b.xs = p.pc_x * W - 0.5;
    b.ys = p.pc_y * H - 0.5;
    b.zs = p.pc_z * W;

    // workspace plan
    const int max_tiles = b.max_tiles;
    Plan w;
    const size_t o_desc = w.take(sizeof(Bucket));
    const size_t o_test_in = w.take(sizeof(void*) * nb);
    const size_t o_ref_in = w.take(sizeof(void*) * nref);
    const size_t o_ref_slot = w.take(sizeof(int32_t) * nb);
    const size_t o_pair_index = w.take(sizeof(int32_t) * nb);
    const size_t o_roi_c = w.take(sizeof(double) * 2 * nr);
    const size_t o_roi_xy = w.take(sizeof(int32_t) * 2 * nr);
    const size_t o_dst = w.take(sizeof(float*) * nb);
    const size_t desc_bytes = w.off;
    const size_t o_test_pyr = w.take(sizeof(float) * (size_t)nb * pe);
    const size_t o_ref_pyr = w.take(sizeof(float) * (size_t)nref * pe);
    const size_t o_tstat = w.take(sizeof(PatStat) * nb);
    const size_t o_rstat = w.take(sizeof(PatStat) * nref);
    const size_t field_bytes = mode == Mode::Full ? sizeof(float) * 2 * (size_t)nb * H * W : 0;
    const size_t o_f0 = w.take(field_bytes);
    const size_t o_f1 = w.take(field_bytes);
    const size_t o_state = w.take(sizeof(PairState) * nb);
    const size_t o_partial = w.take(sizeof(float) * 4 * (size_t)nb * max_tiles);
    const size_t o_iters = w.take(sizeof(int32_t) * (size_t)nb * L);
    const size_t o_q1 = w.take(sizeof(float) * 2 * (size_t)nb * nr);
    const size_t o_q2 = w.take(sizeof(float) * 2 * (size_t)nb * nr);
    const size_t o_ph = w.take(sizeof(float) * (size_t)nb * nr);
    const size_t o_F1 = w.take(sizeof(double) * 9 * nb);
    const size_t o_Rfin = w.take(sizeof(double) * 9 * nb);
    const size_t o_F = w.take(sizeof(double) * 9 * nb);
    const size_t o_R = w.take(sizeof(double) * 9 * nb);
    const size_t o_rv = w.take(sizeof(double) * 3 * nb);
    const size_t o_st = w.take(sizeof(uint32_t) * nb);
    const size_t o_mae = w.take(sizeof(double) * 2 * nb);
    const bool bandpass = p.bandpass_lo_px > 0.0f || p.bandpass_hi_px > 0.0f;
    const bool bg_static = p.background_static != 0, bg_dyn = p.background_dynamic_px > 0.0f;
    const bool prefilter = bandpass || bg_static || bg_dyn;
    const size_t npat_hw = (size_t)(nb + nref) * H * W;
    const size_t o_pf = w.take(prefilter ? sizeof(float) * 2 * npat_hw : 0);  // band row sums
    const size_t o_blur = w.take(bg_dyn ? sizeof(float) * npat_hw : 0);       // dynamic background
    const size_t o_bgs = w.take(bg_static ? sizeof(float) * (size_t)H * W : 0);  // static background
    const bool want_ssim = mode == Mode::Full && p.first_pass == 0 && out->ssim && !tune_only &&
                           ssim_tiles(H, W) > 0;
    const size_t o_ssim = w.take(want_ssim ? sizeof(double) * (size_t)nb * (1 + ssim_tiles(H, W)) : 0);
    const bool xcf = mode == Mode::SecondPassOnly || p.second_pass;
    const bool cubic = xcf && p.remap_interp == 3 && !tune_only;
    const size_t o_coef = w.take(cubic ? sizeof(float) * (size_t)nref * H * W : 0);
    const size_t o_coef_tmp = w.take(cubic ? sizeof(float) * (size_t)nref * H * W : 0);
    const bool xcf_any = (xcf || (mode == Mode::Full && p.first_pass == 1)) && !tune_only;
    const size_t o_xscr = w.take(xcf_any ? sizeof(float) * (size_t)xcf_scratch_floats(p.roi_size, (int64_t)nb * nr)
                                         : 0);
    const bool warm = mode == Mode::Full && !tune_only && !u_init && p.warm_start;
    const int64_t gcell = (int64_t)(H >> 2) * (W >> 2);  // coarse grid of the pattern
    const int64_t ncell = (int64_t)(kWarmRes / 4) * (kWarmRes / 4);  // the network's output grid
    const size_t o_wfield = w.take(warm ? sizeof(float) * 2 * (size_t)nb * ncell : 0);
    const size_t o_uinit = w.take(warm ? sizeof(float) * 2 * (size_t)nb * gcell : 0);
    const size_t o_wmis = w.take(warm ? sizeof(float) * (size_t)nb : 0);
    const size_t o_wflag = w.take(warm ? sizeof(uint32_t) * (size_t)nb : 0);
    int e = ensure_ws(h, w.off);
    if (e) return e;
    char* base = h->ws;

    b.test_in = reinterpret_cast<const float* const*>(base + o_test_in);
    b.ref_in = reinterpret_cast<const float* const*>(base + o_ref_in);
    b.ref_slot = reinterpret_cast<const int32_t*>(base + o_ref_slot);
    b.pair_index = reinterpret_cast<const int32_t*>(base + o_pair_index);
    b.roi_c = reinterpret_cast<const double*>(base + o_roi_c);
    b.roi_xy = reinterpret_cast<const int32_t*>(base + o_roi_xy);
    b.test_pyr = reinterpret_cast<float*>(base + o_test_pyr);
    b.ref_pyr = reinterpret_cast<float*>(base + o_ref_pyr);
    b.test_stat = reinterpret_cast<PatStat*>(base + o_tstat);
    b.ref_stat = reinterpret_cast<PatStat*>(base + o_rstat);
    b.field[0] = reinterpret_cast<float*>(base + o_f0);
    b.field[1] = reinterpret_cast<float*>(base + o_f1);
    b.state = reinterpret_cast<PairState*>(base + o_state);
    b.partial = reinterpret_cast<float*>(base + o_partial);
    b.iters = reinterpret_cast<int32_t*>(base + o_iters);
    b.q1 = reinterpret_cast<float*>(base + o_q1);
    b.q2 = reinterpret_cast<float*>(base + o_q2);
    b.ph = reinterpret_cast<float*>(base + o_ph);
    b.F1 = reinterpret_cast<double*>(base + o_F1);
    b.Rfin = reinterpret_cast<double*>(base + o_Rfin);
    b.F = reinterpret_cast<double*>(base + o_F);
    b.R = reinterpret_cast<double*>(base + o_R);
    b.rotvec = reinterpret_cast<double*>(base + o_rv);
    b.status = reinterpret_cast<uint32_t*>(base + o_st);
    b.mae1 = reinterpret_cast<double*>(base + o_mae);
    b.mae = b.mae1 + nb;
    b.prefilter = prefilter ? 1 : 0;
    b.ssim = want_ssim ? reinterpret_cast<double*>(base + o_ssim) : nullptr;
    b.ssim_part = want_ssim ? b.ssim + nb : nullptr;
    b.ref_coef = cubic ? reinterpret_cast<float*>(base + o_coef) : nullptr;
    b.coef_tmp = cubic ? reinterpret_cast<float*>(base + o_coef_tmp) : nullptr;
    b.xcf_scratch = xcf_any && p.roi_size == 256 ? reinterpret_cast<float*>(base + o_xscr) : nullptr;

    const bool xcf_first = mode == Mode::Full && p.first_pass == 1;
    bool want_field = mode == Mode::Full && out->field && !xcf_first;
    b.out.F = out->F;
    b.out.R = out->R;
    b.out.rotvec = out->rotvec;
    b.out.Rfin = out->R_finite;
    b.out.F1 = mode == Mode::Full ? out->F_first : nullptr;
    b.out.q1 = mode == Mode::Full ? out->q1 : nullptr;
    b.out.q2 = out->q2;
    b.out.ph = out->peak_height;
    b.out.iters = mode == Mode::Full ? out->iters : nullptr;
    b.out.status = out->status;
    b.out.mae1 = mode == Mode::Full ? out->mae_first : nullptr;
    b.out.mae = out->mae;
    b.out.ssim = mode == Mode::Full ? out->ssim : nullptr;
    b.out.omega = out->omega;
    b.u_init = warm ? reinterpret_cast<const float*>(base + o_uinit) : u_init;
    if (warm) {
        b.warm_field = reinterpret_cast<const float*>(base + o_wfield);
        b.warm_misfit = reinterpret_cast<const float*>(base + o_wmis);
        b.warm_flag = reinterpret_cast<const uint32_t*>(base + o_wflag);
        b.out.warm_field = out->warm_field;
        b.out.warm_misfit = out->warm_misfit;
    }
    b.field_dst = want_field ? reinterpret_cast<float* const*>(base + o_dst) : nullptr;
    b.rfin_in = rfin_in;

    // descriptor blob in pinned memory
    char* pin = h->pin + pin_off;
    std::memset(pin, 0, desc_bytes);
    std::memcpy(pin + o_desc, &b, sizeof b);
    std::memcpy(pin + o_test_in, hbk.test_in.data(), sizeof(void*) * nb);
    std::memcpy(pin + o_ref_in, hbk.ref_in.data(), sizeof(void*) * nref);
    std::memcpy(pin + o_ref_slot, hbk.ref_slot.data(), sizeof(int32_t) * nb);
    std::memcpy(pin + o_pair_index, hbk.pair_index.data(), sizeof(int32_t) * nb);
    {
        std::vector<double> cx(nr), cy(nr), c2(2 * nr);
        std::vector<int32_t> x0(nr), y0(nr), xy(2 * nr);
        roi_layout(p, H, W, cx.data(), cy.data(), x0.data(), y0.data());
        for (int j = 0; j < nr; j++) {
            c2[2 * j] = cx[j];
            c2[2 * j + 1] = cy[j];
            xy[2 * j] = x0[j];
            xy[2 * j + 1] = y0[j];
        }
        std::memcpy(pin + o_roi_c, c2.data(), sizeof(double) * 2 * nr);
        std::memcpy(pin + o_roi_xy, xy.data(), sizeof(int32_t) * 2 * nr);
    }
    if (want_field) {
        float** dst = reinterpret_cast<float**>(pin + o_dst);
        for (int k = 0; k < nb; k++) {
            const int i = hbk.idx[k];
            const int64_t off = out->field_offset ? out->field_offset[i] : (int64_t)i * 2 * H * W;
            dst[k] = out->field + off;
        }
    }
    *pin_used = desc_bytes;
    hipError_t he = hipMemcpyAsync(base, pin, desc_bytes, hipMemcpyHostToDevice, s);
    if (he != hipSuccess) return map_err(he);
    const Bucket* d_bk = reinterpret_cast<const Bucket*>(base + o_desc);

#define EBSD_TRY(x)                       \
    do {                                  \
        hipError_t err_ = (x);            \
        if (err_ != hipSuccess) return map_err(err_); \
    } while (0)

    const bool tm = h->timing && mode == Mode::Full;
    if (tm) EBSD_TRY(hipEventRecord(h->ev[0], s));
    if (prefilter) {
        // background-corrected, pre-filtered raw patterns into level 0, normalised
        // there in place: static background, dynamic background, band-pass
        BandIO io;
        std::memset(&io, 0, sizeof io);
        io.src_a = b.test_in;
        io.src_b = b.ref_in;
        io.dst_a = b.test_pyr;
        io.dst_b = b.ref_pyr;
        io.dst_stride = pe;
        io.na = nb;
        io.npat = nb + nref;
        io.H = H;
        io.W = W;
        io.tmp = reinterpret_cast<float*>(base + o_pf);
        float* bgs = bg_static ? reinterpret_cast<float*>(base + o_bgs) : nullptr;
        if (bg_static) EBSD_TRY(launch_mean_pattern(b.test_in, nb, (int64_t)H * W, bgs, s));
        EBSD_TRY(launch_bg_static(io, bgs, s));  // a copy into level 0 without the static step
        // from here on level 0 is the source
        BandIO lv = io;
        lv.src_a = nullptr;
        lv.src_b = nullptr;
        lv.srcb_a = b.test_pyr;
        lv.srcb_b = b.ref_pyr;
        lv.srcb_stride = pe;
        if (bg_dyn) {
            float* blur = reinterpret_cast<float*>(base + o_blur);
            BandIO bl = lv;  // the blur of every pattern into a contiguous buffer
            bl.dst_a = blur;
            bl.dst_b = blur + (size_t)nb * H * W;
            bl.dst_stride = (int64_t)H * W;
            EBSD_TRY(launch_bandpass(bl, make_band_taps(p.background_dynamic_px, 0.0), s));
            EBSD_TRY(launch_bg_dynamic(lv, blur, s));
        }
        if (bandpass) EBSD_TRY(launch_bandpass(lv, make_band_taps(p.bandpass_lo_px, p.bandpass_hi_px), s));
    }
    EBSD_TRY(launch_stats(d_bk, nb, nref, s));
    EBSD_TRY(launch_pyramids(d_bk, b, s));
    if (tune_only) {
        // time each supported strip height for every row-marching level
        EBSD_TRY(launch_demons_init(d_bk, b, s));
        hipEvent_t e0, e1;
        EBSD_TRY(hipEventCreate(&e0));
        EBSD_TRY(hipEventCreate(&e1));
        for (int l = L - 1; l >= 0; l--) {
            const int lh = b.lh[l], lw = b.lw[l];
            if (!rows_cpl(lw)) continue;
            float best = 1e30f;
            int best_ty = kDefaultStripTY;
            for (int ty : {0, 16, 32, 64, 128}) {
                if (!strip_ty_ok(lw, ty)) continue;  // 0: the 2-D tile kernel, levels wider than 512 px
                for (int it = 0; it < 2; it++)
                    EBSD_TRY(launch_demons_iter(d_bk, b, l, it, h->taps, h->radius, 0.0f, ty, s));
                EBSD_TRY(hipEventRecord(e0, s));
                for (int it = 0; it < 6; it++)
                    EBSD_TRY(launch_demons_iter(d_bk, b, l, it, h->taps, h->radius, 0.0f, ty, s));
                EBSD_TRY(hipEventRecord(e1, s));
                EBSD_TRY(hipEventSynchronize(e1));
                float ms = 0.0f;
                EBSD_TRY(hipEventElapsedTime(&ms, e0, e1));
                if (ms < best) {
                    best = ms;
                    best_ty = ty;
                }
            }
            h->strip_ty[std::make_pair(lh, lw)] = best_ty;
            h->tuned_nb_strip[std::make_pair(lh, lw)] = nb;
            // two iterations per launch: 3 launches (6 iterations) against the best 6 single launches
            int best_fty = 0;
            for (int fty : {8, 16, 32, 64, 128}) {
                if (!rows2_ty_ok(lw, fty)) continue;
                EBSD_TRY(launch_demons_iter2(d_bk, b, l, 0, h->taps, h->radius, 0.0f, 1 << 20, fty, s));
                EBSD_TRY(hipEventRecord(e0, s));
                for (int L2 = 1; L2 <= 3; L2++)
                    EBSD_TRY(launch_demons_iter2(d_bk, b, l, L2, h->taps, h->radius, 0.0f, 1 << 20, fty, s));
                EBSD_TRY(hipEventRecord(e1, s));
                EBSD_TRY(hipEventSynchronize(e1));
                float ms = 0.0f;
                EBSD_TRY(hipEventElapsedTime(&ms, e0, e1));
                if (ms < best) {
                    best = ms;
                    best_fty = fty;
                }
            }
            if (best_fty) h->fused_ty[std::make_pair(lh, lw)] = best_fty;
            else h->fused_ty.erase(std::make_pair(lh, lw));
            h->tuned_nb_fused[std::make_pair(lh, lw)] = nb;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return EBSD_OK;
    }
    // The demons iterations of one level (up to a few hundred launches) are a
    // static sequence for a given configuration: captured once into a graph
    // (per chunk of launches when the level is gated) and replayed; the few
    // other launches and the timing events stay on the stream.
    // fty > 0: two iterations per launch (ceil(cap / 2) launches, plus the
    // decision-only launch that follows an even cap when a tolerance is set)
    auto n_launches = [&](int l, int fty) -> int {
        const int cap = p.max_iters[l];
        if (fty) return (cap + 1) / 2 + ((p.tol_px > 0.0f && cap > 0 && cap % 2 == 0) ? 1 : 0);
        return cap;
    };
    auto launch_range = [&](int l, int ty, int fty, int a, int e, hipStream_t st) -> int {
        for (int k = a; k < e; k++) {
            if (fty)
                EBSD_TRY(launch_demons_iter2(d_bk, b, l, k, h->taps, h->radius, p.tol_px, p.max_iters[l], fty, st));
            else
                EBSD_TRY(launch_demons_iter(d_bk, b, l, k, h->taps, h->radius, p.tol_px, ty, st));
        }
        return EBSD_OK;
    };
    auto run_range = [&](int l, int ty, int fty, int a, int e) -> int {
        if (h->graphs && e > a) {
            std::ostringstream key;
            key << H << ' ' << W << ' ' << nb << ' ' << nref << ' ' << l << ' ' << p.max_iters[l]
                << ' ' << p.tol_px << ' ' << h->radius << ' ' << ty << ' ' << fty << ' ' << a << ' ' << e
                << ' ' << (void*)base;
            auto it = h->graph_cache.find(key.str());
            hipGraphExec_t exec = nullptr;
            if (it != h->graph_cache.end()) {
                exec = it->second;
            } else {
                if (!h->cap_stream &&
                    hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) != hipSuccess)
                    h->cap_stream = nullptr;
                hipGraph_t graph = nullptr;
                std::shared_lock<std::shared_mutex> cap_lk(capture_mutex());
                if (h->cap_stream &&
                    hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeRelaxed) == hipSuccess) {
                    const int e2 = launch_range(l, ty, fty, a, e, h->cap_stream);
                    const hipError_t ec = hipStreamEndCapture(h->cap_stream, &graph);
                    if (e2 == EBSD_OK && ec == hipSuccess && graph &&
                        hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
                        exec = nullptr;
                    if (graph) (void)hipGraphDestroy(graph);
                }
                (void)hipGetLastError();
                h->graph_cache[key.str()] = exec;  // nullptr: this configuration runs eagerly
            }
            if (exec) {
                EBSD_TRY(hipGraphLaunch(exec, s));
                return EBSD_OK;
            }
        }
        return launch_range(l, ty, fty, a, e, s);
    };
    // gating needs a stream the host may wait on: not while the caller captures it
    bool gate = p.tol_px > 0.0f && h->gate_chunk > 0 && mode == Mode::Full;
    if (gate) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) gate = false;
        (void)hipGetLastError();
    }
    if (gate && !h->gate_host) {
        DeviceWideLock lk(capture_mutex());
        if (hipHostMalloc((void**)&h->gate_host, sizeof(int32_t) * 4, hipHostMallocMapped) != hipSuccess ||
            hipHostGetDevicePointer((void**)&h->gate_dev, h->gate_host, 0) != hipSuccess) {
            if (h->gate_host) (void)hipHostFree(h->gate_host);
            h->gate_host = nullptr;
            h->gate_dev = nullptr;
            (void)hipGetLastError();
            return EBSD_ENOMEM;
        }
        for (auto& ev : h->gate_ev)
            EBSD_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    }
    auto run_level = [&](int l, int ty, int fty) -> int {
        const int nl = n_launches(l, fty);
        h->launches_planned[l] += nl;
        const int chunk = gate ? h->gate_chunk : 0;
        if (chunk <= 0 || nl <= chunk) {
            h->launches_issued[l] += nl;
            return run_range(l, ty, fty, 0, nl);
        }
        int done = 0;
        for (int c = 0, a = 0; a < nl; c++, a += chunk) {
            const int e = std::min(nl, a + chunk);
            const int r = run_range(l, ty, fty, a, e);
            if (r) return r;
            done = e;
            if (e == nl) break;
            EBSD_TRY(launch_count_active(d_bk, h->gate_dev + (c & 3), s));
            EBSD_TRY(hipEventRecord(h->gate_ev[c & 3], s));
            if (c >= 2) {
                // chunks c - 1 and c are queued behind chunk c - 2's count: the device
                // stays busy while the host waits for it and reads it
                EBSD_TRY(hipEventSynchronize(h->gate_ev[(c - 2) & 3]));
                if (reinterpret_cast<volatile int32_t*>(h->gate_host)[(c - 2) & 3] == 0) break;
            }
        }
        h->launches_issued[l] += done;
        return EBSD_OK;
    };
    if (warm) {
        // network field at the coarse grid, chunk by chunk, then the Eq. (2)
        // fit that decides between it and zero
        // The network sees 256 x 256 images: level 0 of a 256 px pattern, level
        // 1 of a 512 px pattern, level 0 of a 128 px pattern upsampled x2.
        float* wf = reinterpret_cast<float*>(base + o_wfield);
        const int in_lvl = H == 2 * kWarmRes ? 1 : 0;
        const int up2 = H * 2 == kWarmRes ? 1 : 0;
        const int cm = cnn_max_batch(h->cnn);
        for (int c0 = 0; c0 < nb; c0 += cm) {
            const int cnt = std::min(cm, nb - c0);
            const int ec = cnn_forward_from(h->cnn, b.ref_pyr + b.lvl_off[in_lvl], pe, b.ref_slot + c0,
                                            b.test_pyr + (int64_t)c0 * pe + b.lvl_off[in_lvl], pe, cnt, up2,
                                            wf + (int64_t)c0 * 2 * ncell, s);
            if (ec) return ec;
        }
        const double xn = p.pc_x * kWarmRes - 0.5, yn = p.pc_y * kWarmRes - 0.5, zn = p.pc_z * kWarmRes;
        EBSD_TRY(launch_warm_fit(wf, nb, kWarmRes, xn, yn, zn, p.roi_radius_frac * kWarmRes,
                                 (double)p.fallback_residual_px, p.warm_start == 2 ? 1 : 0, H, b.xs, b.ys, b.zs,
                                 reinterpret_cast<float*>(base + o_uinit),
                                 reinterpret_cast<float*>(base + o_wmis), reinterpret_cast<uint32_t*>(base + o_wflag),
                                 s));
    }
    if (xcf_first) {
        // the conventional first pass: ROI XCF of the unremapped patterns
        EBSD_TRY(launch_zero_iters(d_bk, b, s));
        EBSD_TRY(launch_xcf_first(d_bk, b, p.window, s));
        EBSD_TRY(launch_solve_first(d_bk, b, 0.0f, s));
    } else if (mode == Mode::Full) {
        EBSD_TRY(launch_demons_init(d_bk, b, s));
        for (int l = L - 1; l >= 0; l--) {
            const int ty = strip_ty_for(h, b.lh[l], b.lw[l], nb);
            const int fty = fused_ty_for(h, b.lh[l], b.lw[l], nb);
            // one workgroup per pair and CU: a win while the batch leaves CUs idle in the
            // per-iteration launches (measured: single pair 5.1 -> 3.6 ms; 1024 pairs at
            // 64 x 64 px 4.0 -> 4.5 ms, so large batches keep the row kernels)
            const bool res = h->resident && nb <= kResidentMaxPairs && demons_resident_ok(b.lh[l], b.lw[l]);
            if (tm) EBSD_TRY(hipEventRecord(h->ev[2 + 2 * l], s));
            if (res) {
                EBSD_TRY(launch_demons_resident(d_bk, b, l, h->taps, h->radius, p.tol_px, p.max_iters[l], s));
            } else {
                const int e = run_level(l, ty, fty);
                if (e) return e;
            }
            if (tm) EBSD_TRY(hipEventRecord(h->ev[3 + 2 * l], s));
            if (!res)
                EBSD_TRY(launch_level_end(d_bk, b, l, p.max_iters[l], p.tol_px, fty ? fty : ty, fty != 0, s));
            if (l > 0) EBSD_TRY(launch_prolong_level(d_bk, b, l, s));
        }
        EBSD_TRY(launch_sample_q1(d_bk, b, s));
        if (want_ssim) EBSD_TRY(launch_ssim(d_bk, b, s));
        if (want_field) EBSD_TRY(launch_copy_field(d_bk, b, s));
        EBSD_TRY(launch_solve_first(d_bk, b, p.tol_px, s));
    } else {
        EBSD_TRY(launch_gather_rfin(d_bk, b, s));
        EBSD_TRY(launch_status_inputs(d_bk, b, s));
    }
    if (xcf) {
        // remap + XCF + Eq. (12); pass k > 0 remaps by the rotation of pass k-1
        if (cubic) EBSD_TRY(launch_bspline_coef(d_bk, b, s));
        for (int pass = 0; pass < p.xcf_passes; pass++) {
            EBSD_TRY(launch_xcf_pairs(d_bk, b, p.window, p.remap_interp, pass, s));
            EBSD_TRY(launch_solve_second(d_bk, b, 1, pass, s));
        }
    } else {
        EBSD_TRY(launch_solve_second(d_bk, b, 0, 0, s));
    }
    EBSD_TRY(launch_scatter(d_bk, b, s));
    if (warm && out->warm_field) EBSD_TRY(launch_scatter_warm(d_bk, b, s));
    if (tm) {
        EBSD_TRY(hipEventRecord(h->ev[1], s));
        h->timed_call = true;
        h->timed_levels = xcf_first ? 0 : L;  // no demons levels with the XCF first pass
    }
#undef EBSD_TRY
    return EBSD_OK;
}

size_t desc_upper_bound(const HostBucket& hb, int nr)
{
    const size_t nb = hb.idx.size(), nref = hb.ref_in.size();
    return align_up(sizeof(Bucket), 256) + 8 * 256 + sizeof(void*) * (2 * nb + nref) +
           sizeof(int32_t) * 2 * nb + sizeof(double) * 2 * nr + sizeof(int32_t) * 2 * nr;
}

int run_body(ebsd_handle* h, const ebsd_pair* pairs, int n, Mode mode, const float* u_init,
             const double* rfin_in, const ebsd_outputs* out, void* stream, bool tune_only)
{
    if (!h || !out) return EBSD_EINVAL;
    int e = check_pairs(h->p, pairs, n);
    if (e) return e;
    if (n == 0) return EBSD_OK;
    if (mode == Mode::SecondPassOnly && !rfin_in) return EBSD_EINVAL;
    std::vector<HostBucket> buckets = make_buckets(pairs, n);
    if (u_init && buckets.size() != 1) return EBSD_EINVAL;
    if (u_init && h->p.first_pass == 1) return EBSD_EINVAL;
    if (mode == Mode::Full && !tune_only && !u_init && h->p.warm_start) {
        if (!cnn_ready(h->cnn)) return EBSD_ENOMODEL;
        if (h->p.levels != kWarmLevels) return EBSD_ESHAPE;
        for (auto& hb : buckets)
            if (hb.H != hb.W || (hb.H != kWarmRes && hb.H != kWarmRes / 2 && hb.H != 2 * kWarmRes))
                return EBSD_ESHAPE;
    }
    DeviceGuard g(h->device);
    if (!g.ok) return EBSD_EDEVICE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (!tune_only) {
        for (int l = 0; l < EBSD_MAX_LEVELS; l++) h->launches_issued[l] = h->launches_planned[l] = 0;
    }
    size_t need = 0;
    for (auto& hb : buckets) need += desc_upper_bound(hb, h->p.n_roi);
    e = ensure_pin(h, need);
    if (e) return e;
    size_t off = 0;
    for (auto& hb : buckets) {
        size_t used = 0;
        e = run_bucket(h, hb, mode, u_init, rfin_in, out, s, off, &used, tune_only);
        if (e) return e;
        off = align_up(off + used, 256);
    }
    if (hipEventRecord(h->pin_free, s) != hipSuccess) return EBSD_EDEVICE;
    h->pin_pending = true;
    if (tune_only) save_tune_cache(h);
    return EBSD_OK;
}

// A call's host-side containers (buckets, descriptors, the tuned tables) can
// throw std::bad_alloc; no exception leaves the C ABI or a pipeline's thread.
int run(ebsd_handle* h, const ebsd_pair* pairs, int n, Mode mode, const float* u_init,
        const double* rfin_in, const ebsd_outputs* out, void* stream, bool tune_only = false)
{
    try {
        return run_body(h, pairs, n, mode, u_init, rfin_in, out, stream, tune_only);
    } catch (const std::bad_alloc&) {
        return EBSD_ENOMEM;
    }
}

}  // namespace

extern "C" {

int ebsd_version(void) { return EBSD_ABI_VERSION; }

int ebsd_params_default(ebsd_params* p)
{
    if (!p) return EBSD_EINVAL;
    std::memset(p, 0, sizeof *p);
    p->struct_size = sizeof(ebsd_params);
    p->levels = 3;
    for (int l = 0; l < EBSD_MAX_LEVELS; l++) p->max_iters[l] = 150;
    p->sigma_px = 1.0f;
    p->tol_px = 0.0f;
    p->pc_x = 0.5;
    p->pc_y = 0.5;
    p->pc_z = 0.7;
    p->n_roi = 20;
    p->roi_size = 64;
    p->roi_radius_frac = 0.3;
    p->window = 1;
    p->second_pass = 1;
    p->warm_start = 0;
    p->fallback_residual_px = 0.5f;
    p->remap_interp = 3;
    p->xcf_passes = 1;
    p->first_pass = 0;
    p->bandpass_lo_px = 0.0f;
    p->bandpass_hi_px = 0.0f;
    p->background_static = 0;
    p->background_dynamic_px = 0.0f;
    return EBSD_OK;
}

const char* ebsd_strerror(int code)
{
    switch (code) {
    case EBSD_OK: return "ok";
    case EBSD_EINVAL: return "invalid argument";
    case EBSD_ESHAPE: return "unsupported pattern size";
    case EBSD_EROI: return "ROI outside the pattern or unsupported ROI size";
    case EBSD_ENOMEM: return "out of memory";
    case EBSD_EDEVICE: return "HIP runtime error";
    case EBSD_ENOTSUP: return "not supported";
    case EBSD_ENOMODEL: return "warm start requested but no network parameters loaded";
    case EBSD_EVERSION: return "ebsd_params.struct_size mismatch";
    case EBSD_EIO: return "parameter file could not be read or written";
    case EBSD_ETOOBIG: return "input larger than the fixed device buffer of an allocation-free entry point";
    default: return "unknown error";
    }
}

int ebsd_create(const ebsd_params* p, int device, ebsd_handle** out)
{
    if (!out) return EBSD_EINVAL;
    *out = nullptr;
    int e = check_params(p);
    if (e) return e;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return EBSD_EDEVICE;
    ebsd_handle* h = new (std::nothrow) ebsd_handle();
    if (!h) return EBSD_ENOMEM;
    h->p = *p;
    h->device = device;
    // Gaussian taps w_j ~ exp(-j^2 / (2 sigma^2)), j = -r..r, r = floor(3 sigma + 0.5)
    for (float& t : h->taps) t = 0.0f;
    if (p->sigma_px > 0.0f) {
        const double sg = p->sigma_px;
        h->radius = (int)std::floor(3.0 * sg + 0.5);
        if (h->radius > kMaxRadius) h->radius = kMaxRadius;
        double wsum = 0.0, wv[2 * kMaxRadius + 1];
        for (int j = -h->radius; j <= h->radius; j++) {
            wv[j + h->radius] = std::exp(-(double)(j * j) / (2.0 * sg * sg));
            wsum += wv[j + h->radius];
        }
        for (int j = 0; j <= 2 * h->radius; j++) h->taps[j] = (float)(wv[j] / wsum);
    } else {
        h->radius = 0;
        h->taps[0] = 1.0f;
    }
    DeviceGuard g(device);
    if (!g.ok || hipEventCreateWithFlags(&h->pin_free, hipEventDisableTiming) != hipSuccess) {
        delete h;
        return EBSD_EDEVICE;
    }
    try {
        if (const char* c = std::getenv("EBSD_TUNE_CACHE")) h->tune_cache = c;
        load_tune_cache(h);
    } catch (const std::bad_alloc&) {
        (void)ebsd_destroy(h);
        return EBSD_ENOMEM;
    }
    *out = h;
    return EBSD_OK;
}

int ebsd_autotune(ebsd_handle* h, const ebsd_pair* pairs, int32_t n, void* stream)
{
    if (!h) return EBSD_EINVAL;
    ebsd_outputs none;
    std::memset(&none, 0, sizeof none);
    int e = run(h, pairs, n, Mode::Full, nullptr, nullptr, &none, stream, true);
    if (e) return e;
    DeviceGuard g(h->device);
    return hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)) == hipSuccess ? EBSD_OK
                                                                                   : EBSD_EDEVICE;
}

int ebsd_set_graphs(ebsd_handle* h, int enable)
{
    if (!h) return EBSD_EINVAL;
    h->graphs = enable != 0;
    return EBSD_OK;
}

int ebsd_set_resident(ebsd_handle* h, int enable)
{
    if (!h) return EBSD_EINVAL;
    h->resident = enable != 0;
    return EBSD_OK;
}

int ebsd_tilt_rotation(double theta, double* S)
{
    if (!S || !std::isfinite(theta)) return EBSD_EINVAL;
    const double c = std::cos(theta), sn = std::sin(theta);
    const double m[9] = {c, sn, 0.0, -sn, c, 0.0, 0.0, 0.0, 1.0};
    for (int i = 0; i < 9; i++) S[i] = m[i];
    return EBSD_OK;
}

int ebsd_set_gating(ebsd_handle* h, int32_t chunk_launches)
{
    if (!h || chunk_launches < 0 || chunk_launches > 1000000) return EBSD_EINVAL;
    h->gate_chunk = chunk_launches;
    return EBSD_OK;
}

int ebsd_get_launch_counts(const ebsd_handle* h, int32_t* issued, int32_t* planned)
{
    if (!h) return EBSD_EINVAL;
    for (int l = 0; l < EBSD_MAX_LEVELS; l++) {
        if (issued) issued[l] = h->launches_issued[l];
        if (planned) planned[l] = h->launches_planned[l];
    }
    return EBSD_OK;
}

int ebsd_get_strip_height(const ebsd_handle* h, int32_t level_h, int32_t level_w)
{
    if (!h || level_h <= 0 || level_w <= 0) return EBSD_EINVAL;
    if (!rows_cpl(level_w)) return 0;
    return strip_ty_for(h, level_h, level_w);
}

int ebsd_set_strip_height(ebsd_handle* h, int32_t level_h, int32_t level_w, int32_t ty)
{
    if (!h || level_h <= 0 || level_w <= 0 || !strip_ty_ok(level_w, ty)) return EBSD_EINVAL;
    try {
        h->strip_ty[std::make_pair((int)level_h, (int)level_w)] = ty;
    } catch (const std::bad_alloc&) {
        return EBSD_ENOMEM;
    }
    h->tuned_nb_strip.erase(std::make_pair((int)level_h, (int)level_w));  // forced: applies to every batch
    return EBSD_OK;
}

int ebsd_get_fused_height(const ebsd_handle* h, int32_t level_h, int32_t level_w)
{
    if (!h || level_h <= 0 || level_w <= 0) return EBSD_EINVAL;
    return fused_ty_for(h, level_h, level_w);
}

int ebsd_set_fused_height(ebsd_handle* h, int32_t level_h, int32_t level_w, int32_t rows)
{
    if (!h || level_h <= 0 || level_w <= 0) return EBSD_EINVAL;
    if (rows != 0 && !rows2_ty_ok(level_w, rows)) return EBSD_EINVAL;
    const auto key = std::make_pair((int)level_h, (int)level_w);
    try {
        if (rows) h->fused_ty[key] = rows;
        else h->fused_ty.erase(key);
    } catch (const std::bad_alloc&) {
        return EBSD_ENOMEM;
    }
    h->tuned_nb_fused.erase(key);  // forced: applies to every batch
    return EBSD_OK;
}

int ebsd_destroy(ebsd_handle* h)
{
    if (!h) return EBSD_OK;
    {
        DeviceGuard g(h->device);
        DeviceWideLock lk(capture_mutex());
        (void)hipDeviceSynchronize();
        if (h->ws) (void)hipFree(h->ws);
        if (h->pin) (void)hipHostFree(h->pin);
        if (h->pin_free) (void)hipEventDestroy(h->pin_free);
        clear_graphs(h);
        if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
        if (h->gate_host) (void)hipHostFree(h->gate_host);
        for (auto& e : h->gate_ev)
            if (e) (void)hipEventDestroy(e);
        for (auto& e : h->ev)
            if (e) (void)hipEventDestroy(e);
    }
    if (h->cnn) (void)ebsd_cnn_destroy(h->cnn);
    delete h;
    return EBSD_OK;
}

int ebsd_set_timing(ebsd_handle* h, int enable)
{
    if (!h) return EBSD_EINVAL;
    DeviceGuard g(h->device);
    if (!g.ok) return EBSD_EDEVICE;
    if (enable && !h->ev[0]) {
        for (auto& e : h->ev)
            if (hipEventCreate(&e) != hipSuccess) return EBSD_EDEVICE;
    }
    h->timing = enable != 0;
    return EBSD_OK;
}

int ebsd_get_timing(ebsd_handle* h, double* level_ms, double* total_ms)
{
    if (!h || !h->timed_call) return EBSD_EINVAL;
    DeviceGuard g(h->device);
    if (hipEventSynchronize(h->ev[1]) != hipSuccess) return EBSD_EDEVICE;
    float ms = 0.0f;
    if (total_ms) {
        if (hipEventElapsedTime(&ms, h->ev[0], h->ev[1]) != hipSuccess) return EBSD_EDEVICE;
        *total_ms = ms;
    }
    if (level_ms)
        for (int l = 0; l < h->timed_levels; l++) {
            if (hipEventElapsedTime(&ms, h->ev[2 + 2 * l], h->ev[3 + 2 * l]) != hipSuccess)
                return EBSD_EDEVICE;
            level_ms[l] = ms;
        }
    return EBSD_OK;
}

int ebsd_get_params(const ebsd_handle* h, ebsd_params* out)
{
    if (!h || !out) return EBSD_EINVAL;
    *out = h->p;
    return EBSD_OK;
}

int ebsd_roi_layout(const ebsd_params* p, int32_t H, int32_t W, double* cx, double* cy,
                    int32_t* x0, int32_t* y0)
{
    int e = check_params(p);
    if (e) return e;
    if (H <= 0 || W <= 0) return EBSD_ESHAPE;
    return roi_layout(*p, H, W, cx, cy, x0, y0);
}

int ebsd_load_model(ebsd_handle* h, const char* path)
{
    if (!h || !path) return EBSD_EINVAL;
    if (!h->cnn) {
        const int e = ebsd_cnn_create(h->device, kWarmBatch, &h->cnn);
        if (e) return e;
    }
    return ebsd_cnn_load(h->cnn, path);
}

int ebsd_set_model(ebsd_handle* h, const ebsd_cnn* c)
{
    if (!h || !c) return EBSD_EINVAL;
    if (!h->cnn) {
        const int e = ebsd_cnn_create(h->device, kWarmBatch, &h->cnn);
        if (e) return e;
    }
    std::vector<float> buf;
    try {
        buf.resize((size_t)EBSD_CNN_PARAMS);
    } catch (const std::bad_alloc&) {
        return EBSD_ENOMEM;
    }
    int e = ebsd_cnn_get_params(c, buf.data(), EBSD_CNN_PARAMS);
    if (e) return e;
    return ebsd_cnn_set_params(h->cnn, buf.data(), EBSD_CNN_PARAMS);
}

int ebsd_register_batch(ebsd_handle* h, const ebsd_pair* pairs, int32_t n,
                        const ebsd_outputs* out, void* stream)
{
    return run(h, pairs, n, Mode::Full, nullptr, nullptr, out, stream);
}

int ebsd_register_batch_init(ebsd_handle* h, const ebsd_pair* pairs, int32_t n,
                             const float* u_init, const ebsd_outputs* out, void* stream)
{
    return run(h, pairs, n, Mode::Full, u_init, nullptr, out, stream);
}

int ebsd_second_pass_batch(ebsd_handle* h, const ebsd_pair* pairs, int32_t n,
                           const double* R_finite, const ebsd_outputs* out, void* stream)
{
    if (!R_finite && n > 0) return EBSD_EINVAL;
    return run(h, pairs, n, Mode::SecondPassOnly, nullptr, R_finite, out, stream);
}

int ebsd_stage_normalize(const float* in, int32_t n, int64_t elems, float* out, uint32_t* flags,
                         void* stream)
{
    if (n < 0 || elems <= 0 || (n > 0 && (!in || !out))) return EBSD_EINVAL;
    if (n == 0) return EBSD_OK;
    return map_err(launch_stage_normalize(in, n, elems, out, flags, (hipStream_t)stream));
}

int ebsd_stage_bandpass(const float* in, int32_t n, int32_t H, int32_t W, float lo_px, float hi_px, float* out,
                        void* stream)
{
    if (n < 0 || (n > 0 && (!in || !out))) return EBSD_EINVAL;
    if (!(lo_px >= 0.0f && lo_px <= 32.0f) || !(hi_px >= 0.0f && hi_px <= 32.0f)) return EBSD_EINVAL;
    if (H < 1 || W < 2 || W > 16384 || H > 65535 || n > 65535) return EBSD_ESHAPE;
    if (n == 0) return EBSD_OK;
    DeviceWideLock lk(capture_mutex());  // the temporary's free waits for the device
    DevBuf tmp;
    if (hipMalloc(&tmp.p, sizeof(float) * 2 * (size_t)n * H * W) != hipSuccess) return EBSD_ENOMEM;
    BandIO io;
    std::memset(&io, 0, sizeof io);
    io.src = in;
    io.src_stride = (int64_t)H * W;
    io.dst_a = out;
    io.dst_b = nullptr;
    io.dst_stride = (int64_t)H * W;
    io.na = n;
    io.npat = n;
    io.H = H;
    io.W = W;
    io.tmp = static_cast<float*>(tmp.p);
    const hipStream_t s = (hipStream_t)stream;
    const int e = map_err(launch_bandpass(io, make_band_taps(lo_px, hi_px), s));
    if (e) return e;
    // the temporary is released after the stream has used it
    if (hipStreamSynchronize(s) != hipSuccess) return EBSD_EDEVICE;
    return EBSD_OK;
}

// ---- the allocation-free pre-filter -------------------------------------------
// ebsd_stage_bandpass_static keeps its row pass (2 n H W floats) in this
// file-scope device array instead of a temporary; each device holds its own
// copy until the process ends.  Host code never passes the array's name to a
// kernel (on the host it is only a stand-in for the symbol): the first call on
// a device looks up that device's address of it, and every call uses that.
constexpr int64_t kStaticScratchFloats = int64_t(8) << 20;  // 32 MiB
static __device__ __align__(256) float scratch[kStaticScratchFloats];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch` (looked up once per device, with
// that device current).
int scratch_for_current_device(float** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return EBSD_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return EBSD_EDEVICE;
        }
        g_scratch_ptr[dev] = static_cast<float*>(p);
    }
    *out = g_scratch_ptr[dev];
    return EBSD_OK;
}
}  // namespace

int ebsd_stage_bandpass_static(const float* in, int32_t n, int32_t H, int32_t W, float lo_px, float hi_px,
                               float* out, void* stream)
{
    if (n < 0 || (n > 0 && (!in || !out))) return EBSD_EINVAL;
    if (!(lo_px >= 0.0f && lo_px <= 32.0f) || !(hi_px >= 0.0f && hi_px <= 32.0f)) return EBSD_EINVAL;
    if (H < 1 || W < 2 || W > 16384 || H > 65535 || n > 65535) return EBSD_ESHAPE;
    if (2 * (int64_t)n * H * W > kStaticScratchFloats) return EBSD_ETOOBIG;
    if (n == 0) return EBSD_OK;
    float* tmp = nullptr;
    const int e = scratch_for_current_device(&tmp);
    if (e) return e;
    BandIO io;
    std::memset(&io, 0, sizeof io);
    io.src = in;
    io.src_stride = (int64_t)H * W;
    io.dst_a = out;
    io.dst_b = nullptr;
    io.dst_stride = (int64_t)H * W;
    io.na = n;
    io.npat = n;
    io.H = H;
    io.W = W;
    io.tmp = tmp;  // fully written by the row pass before the column pass reads it
    return map_err(launch_bandpass(io, make_band_taps(lo_px, hi_px), (hipStream_t)stream));
}

int ebsd_stage_restrict(const float* in, int32_t n, int32_t H, int32_t W, float* out, void* stream)
{
    if (n < 0 || (n > 0 && (!in || !out))) return EBSD_EINVAL;
    if (H < 2 || W < 2 || H > 16384 || W > 16384 || n > 65535) return EBSD_ESHAPE;
    if (n == 0) return EBSD_OK;
    return map_err(launch_stage_restrict(in, n, H, W, out, (hipStream_t)stream));
}

int ebsd_stage_demons_iter(const float* R, const float* T, int32_t n, int32_t H, int32_t W,
                           const float* u_in, float sigma_px, float* u_out, double* rms,
                           void* stream)
{
    if (n < 0 || (n > 0 && (!R || !T || !u_in || !u_out)) || u_in == u_out) return EBSD_EINVAL;
    if (!(sigma_px >= 0.0f) || !(sigma_px <= 1.3f)) return EBSD_EINVAL;
    if (H < 1 || W < 1 || H > 16384 || W > 16384) return EBSD_ESHAPE;
    if (n == 0) return EBSD_OK;
    float taps[2 * kMaxRadius + 1] = {0};
    int radius = 0;
    if (sigma_px > 0.0f) {
        radius = (int)std::floor(3.0 * sigma_px + 0.5);
        double wsum = 0.0, wv[2 * kMaxRadius + 1];
        for (int j = -radius; j <= radius; j++) {
            wv[j + radius] = std::exp(-(double)(j * j) / (2.0 * (double)sigma_px * sigma_px));
            wsum += wv[j + radius];
        }
        for (int j = 0; j <= 2 * radius; j++) taps[j] = (float)(wv[j] / wsum);
    } else {
        taps[0] = 1.0f;
    }
    return map_err(launch_stage_demons_iter(R, T, n, H, W, u_in, taps, radius, u_out, rms,
                                            (hipStream_t)stream));
}

int ebsd_stage_prolong(const float* u, int32_t n, int32_t h, int32_t w, float* out, void* stream)
{
    if (n < 0 || (n > 0 && (!u || !out))) return EBSD_EINVAL;
    if (h < 1 || w < 1 || h > 8192 || w > 8192 || n > 65535) return EBSD_ESHAPE;
    if (n == 0) return EBSD_OK;
    return map_err(launch_stage_prolong(u, n, h, w, out, (hipStream_t)stream));
}

int ebsd_stage_xcf(const float* A, const float* B, int32_t n, int32_t N, int32_t window, float* q,
                   float* ph, void* stream)
{
    if (n < 0 || (n > 0 && (!A || !B || !q))) return EBSD_EINVAL;
    if (N != 32 && N != 64 && N != 128 && N != 256) return EBSD_EROI;
    if (window != 0 && window != 1) return EBSD_EINVAL;
    if (n == 0) return EBSD_OK;
    const hipStream_t s = (hipStream_t)stream;
    if (N < 256) return map_err(launch_stage_xcf(A, B, n, N, window, q, ph, nullptr, s));
    DeviceWideLock lk(capture_mutex());  // the temporary's free waits for the device
    DevBuf scr;
    if (hipMalloc(&scr.p, sizeof(float) * (size_t)xcf_scratch_floats(N, n)) != hipSuccess) {
        (void)hipGetLastError();
        return EBSD_ENOMEM;
    }
    const int e = map_err(launch_stage_xcf(A, B, n, N, window, q, ph, static_cast<float*>(scr.p), s));
    if (e) return e;
    // the scratch is released after the stream has used it
    if (hipStreamSynchronize(s) != hipSuccess) return EBSD_EDEVICE;
    return EBSD_OK;
}

int ebsd_stage_remap(const float* img, int32_t n, int32_t H, int32_t W, const double* R, double xs,
                     double ys, double zs, int32_t interp, float* coef, float* out, void* stream)
{
    if (n < 0 || (n > 0 && (!img || !R || !out))) return EBSD_EINVAL;
    if (interp != 1 && interp != 3) return EBSD_EINVAL;
    if (interp == 3 && n > 0 && !coef) return EBSD_EINVAL;
    if (!std::isfinite(xs) || !std::isfinite(ys) || !(zs > 0.0) || !std::isfinite(zs)) return EBSD_EINVAL;
    if (H < 3 || W < 3 || n > 65535) return EBSD_ESHAPE;
    if (n == 0) return EBSD_OK;
    return map_err(launch_stage_remap(img, n, H, W, R, xs, ys, zs, interp, coef, out, (hipStream_t)stream));
}

int ebsd_stage_solve(const float* q, int32_t n, int32_t n_roi, const double* cx, const double* cy,
                     double xs, double ys, double zs, double* F, double* R, uint32_t* status,
                     void* stream)
{
    if (n < 0 || (n > 0 && (!q || !cx || !cy || !F))) return EBSD_EINVAL;
    if (n_roi < 5 || n_roi > 256 || !(zs > 0.0)) return EBSD_EINVAL;
    if (n == 0) return EBSD_OK;
    return map_err(launch_stage_solve(q, n, n_roi, cx, cy, xs, ys, zs, F, R, status,
                                      (hipStream_t)stream));
}

int ebsd_traction_free(const float* q, int32_t n, int32_t n_roi, const double* cx, const double* cy,
                       double xs, double ys, double zs, const double* M, const double* g, const double* S,
                       double C11, double C12, double C44, double* F, double* eps_S, double* sigma_S,
                       uint32_t* status, void* stream)
{
    if (n < 0 || (n > 0 && (!q || !cx || !cy || !g || !F))) return EBSD_EINVAL;
    if (n_roi < 5 || n_roi > 256 || !(zs > 0.0) || !std::isfinite(xs) || !std::isfinite(ys) || !std::isfinite(zs))
        return EBSD_EINVAL;
    if (!S) return EBSD_EINVAL;
    // a rotation: S S^T = I, det S = +1
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            const double d = S[3 * i] * S[3 * j] + S[3 * i + 1] * S[3 * j + 1] + S[3 * i + 2] * S[3 * j + 2];
            if (!(std::fabs(d - (i == j ? 1.0 : 0.0)) <= 1e-9)) return EBSD_EINVAL;
        }
    const double det = S[0] * (S[4] * S[8] - S[5] * S[7]) - S[1] * (S[3] * S[8] - S[5] * S[6]) +
                       S[2] * (S[3] * S[7] - S[4] * S[6]);
    if (!(det > 0.0)) return EBSD_EINVAL;
    // a positive definite cubic stiffness
    if (!std::isfinite(C11) || !std::isfinite(C12) || !std::isfinite(C44) || !(C44 > 0.0) || !(C11 - C12 > 0.0) ||
        !(C11 + 2.0 * C12 > 0.0))
        return EBSD_EINVAL;
    if (n == 0) return EBSD_OK;
    TractionFrame tf;
    for (int i = 0; i < 9; i++) tf.S[i] = S[i];
    tf.c11 = C11;
    tf.c12 = C12;
    tf.c44 = C44;
    return map_err(launch_traction_free(q, n, n_roi, cx, cy, xs, ys, zs, M, g, tf, F, eps_S, sigma_S, status,
                                        (hipStream_t)stream));
}

}  // extern "C"

// ---- pipelined registration -------------------------------------------------------
//
// Batches submitted one after another run on `depth` registration handles, each
// with its own stream, workspace, captured graphs and network, from one host
// thread per handle (a call blocks its thread while a gated level waits for
// its counts), so `depth` batches are in flight at once.  Their phases drift
// apart within a few batches, and one batch's network forward, coarse levels
// and second pass then overlap another's finest level.  Each batch is a plain
// ebsd_register_batch call on its handle: results are the same bit for bit.
struct ebsd_pipeline {
    struct Job {
        std::vector<ebsd_pair> pairs;
        ebsd_outputs out;
        std::vector<int64_t> offs;  // copy of out.field_offset (host array)
        bool has_offs = false;
        hipEvent_t ready = nullptr;  // recorded on the caller's stream at submission
    };
    int depth = 0;
    int device = 0;
    std::vector<ebsd_handle*> h;
    std::vector<hipStream_t> st;
    std::vector<hipEvent_t> ev_done;     // per slot: its last batch is complete
    std::vector<std::deque<Job>> queue;  // per slot
    std::vector<std::thread> workers;
    std::mutex mu;
    std::condition_variable cv;
    uint64_t submitted = 0;  // batches submitted
    uint64_t finished = 0;   // batches whose calls have returned
    int error = 0;
    bool stop = false;
};

namespace {

void pipeline_worker(ebsd_pipeline* pl, int slot)
{
    for (;;) {
        ebsd_pipeline::Job job;
        {
            std::unique_lock<std::mutex> lk(pl->mu);
            pl->cv.wait(lk, [&] { return pl->stop || !pl->queue[slot].empty(); });
            if (pl->queue[slot].empty()) return;  // stop requested and nothing left
            job = std::move(pl->queue[slot].front());
            pl->queue[slot].pop_front();
        }
        DeviceGuard g(pl->device);
        int rc = g.ok ? EBSD_OK : EBSD_EDEVICE;
        hipStream_t s = pl->st[slot];
        if (rc == EBSD_OK && hipStreamWaitEvent(s, job.ready, 0) != hipSuccess) rc = EBSD_EDEVICE;
        (void)hipEventDestroy(job.ready);
        if (rc == EBSD_OK) {
            if (job.has_offs) job.out.field_offset = job.offs.data();
            rc = run(pl->h[slot], job.pairs.data(), (int)job.pairs.size(), Mode::Full, nullptr, nullptr, &job.out,
                     s);
        }
        if (hipEventRecord(pl->ev_done[slot], s) != hipSuccess && rc == EBSD_OK) rc = EBSD_EDEVICE;
        std::lock_guard<std::mutex> lk(pl->mu);
        if (rc != EBSD_OK && pl->error == EBSD_OK) pl->error = rc;
        pl->finished++;
        pl->cv.notify_all();
    }
}

void pipeline_free(ebsd_pipeline* pl)
{
    {
        std::lock_guard<std::mutex> lk(pl->mu);
        pl->stop = true;
        pl->cv.notify_all();
    }
    for (auto& t : pl->workers)
        if (t.joinable()) t.join();
    {
        DeviceGuard g(pl->device);
        for (hipStream_t s : pl->st)
            if (s) (void)hipStreamSynchronize(s);
        for (hipEvent_t e : pl->ev_done)
            if (e) (void)hipEventDestroy(e);
        for (hipStream_t s : pl->st)
            if (s) (void)hipStreamDestroy(s);
    }
    for (ebsd_handle* h : pl->h) (void)ebsd_destroy(h);
    delete pl;
}

}  // namespace

extern "C" {

int ebsd_pipeline_create(const ebsd_params* p, int device, int32_t depth, ebsd_pipeline** out)
{
    if (!out) return EBSD_EINVAL;
    *out = nullptr;
    if (depth < 1 || depth > kMaxPipelineDepth) return EBSD_EINVAL;
    int e = check_params(p);
    if (e) return e;
    ebsd_pipeline* pl = new (std::nothrow) ebsd_pipeline();
    if (!pl) return EBSD_ENOMEM;
    pl->depth = depth;
    pl->device = device;
    try {
        pl->h.assign(depth, nullptr);
        pl->st.assign(depth, nullptr);
        pl->ev_done.assign(depth, nullptr);
        pl->queue.resize(depth);
        pl->workers.reserve(depth);
    } catch (const std::bad_alloc&) {
        pipeline_free(pl);
        return EBSD_ENOMEM;
    }
    for (int k = 0; k < depth; k++) {
        e = ebsd_create(p, device, &pl->h[k]);
        if (e) {
            pipeline_free(pl);
            return e;
        }
    }
    {
        DeviceGuard g(device);
        bool ok = g.ok;
        for (int k = 0; ok && k < depth; k++)
            ok = hipStreamCreateWithFlags(&pl->st[k], hipStreamNonBlocking) == hipSuccess &&
                 hipEventCreateWithFlags(&pl->ev_done[k], hipEventDisableTiming) == hipSuccess;
        if (!ok) {
            pipeline_free(pl);
            return EBSD_EDEVICE;
        }
    }
    try {
        for (int k = 0; k < depth; k++) pl->workers.emplace_back(pipeline_worker, pl, k);
    } catch (...) {
        pipeline_free(pl);
        return EBSD_ENOMEM;
    }
    *out = pl;
    return EBSD_OK;
}

int ebsd_pipeline_handle(ebsd_pipeline* pl, int32_t slot, ebsd_handle** h)
{
    if (!pl || !h || slot < 0 || slot >= pl->depth) return EBSD_EINVAL;
    *h = pl->h[slot];
    return EBSD_OK;
}

int ebsd_pipeline_submit(ebsd_pipeline* pl, const ebsd_pair* pairs, int32_t n, const ebsd_outputs* out,
                         void* stream)
{
    if (!pl || !out || n < 0 || (n > 0 && !pairs)) return EBSD_EINVAL;
    const int e = check_pairs(pl->h[0]->p, pairs, n);
    if (e) return e;
    ebsd_pipeline::Job job;
    try {
        job.pairs.assign(pairs, pairs + n);
        if (out->field_offset && n > 0) job.offs.assign(out->field_offset, out->field_offset + n);
    } catch (...) {
        return EBSD_ENOMEM;
    }
    job.out = *out;
    job.has_offs = out->field_offset != nullptr;
    {
        DeviceGuard g(pl->device);
        if (!g.ok || hipEventCreateWithFlags(&job.ready, hipEventDisableTiming) != hipSuccess)
            return EBSD_EDEVICE;
        if (hipEventRecord(job.ready, reinterpret_cast<hipStream_t>(stream)) != hipSuccess) {
            (void)hipEventDestroy(job.ready);
            return EBSD_EDEVICE;
        }
    }
    std::lock_guard<std::mutex> lk(pl->mu);
    try {
        pl->queue[pl->submitted % pl->depth].push_back(std::move(job));
    } catch (const std::bad_alloc&) {  // the queue is unchanged and job still owns its event
        DeviceGuard g(pl->device);
        (void)hipEventDestroy(job.ready);
        return EBSD_ENOMEM;
    }
    pl->submitted++;
    pl->cv.notify_all();
    return EBSD_OK;
}

int ebsd_pipeline_wait(ebsd_pipeline* pl, void* stream)
{
    if (!pl) return EBSD_EINVAL;
    int err;
    {
        std::unique_lock<std::mutex> lk(pl->mu);
        pl->cv.wait(lk, [&] { return pl->finished == pl->submitted; });
        err = pl->error;
        pl->error = EBSD_OK;
    }
    DeviceGuard g(pl->device);
    if (!g.ok) return EBSD_EDEVICE;
    for (int k = 0; k < pl->depth; k++)
        if (hipStreamWaitEvent(reinterpret_cast<hipStream_t>(stream), pl->ev_done[k], 0) != hipSuccess)
            return EBSD_EDEVICE;
    return err;
}

int ebsd_pipeline_destroy(ebsd_pipeline* pl)
{
    if (!pl) return EBSD_OK;
    {
        std::unique_lock<std::mutex> lk(pl->mu);
        pl->cv.wait(lk, [&] { return pl->finished == pl->submitted; });
    }
    pipeline_free(pl);
    return EBSD_OK;
}

}  // extern "C"
