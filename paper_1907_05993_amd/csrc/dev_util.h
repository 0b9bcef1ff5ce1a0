// Small device helpers shared by the gfx950 demons kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ebsd_internal.h"

namespace ebsd {

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Global-address-space views of device pointers.  Pointers read from the
// bucket descriptor are otherwise generic (flat), and flat loads also count
// against the LDS wait counter, so every LDS wait before a barrier would drain
// all outstanding global loads.
#define EBSD_GLOBAL __attribute__((address_space(1)))
__device__ inline const EBSD_GLOBAL float* gptr(const float* p) { return (const EBSD_GLOBAL float*)p; }
__device__ inline EBSD_GLOBAL float* gptr(float* p) { return (EBSD_GLOBAL float*)p; }

// Bilinear sample at (x, y), coordinates clamped to the image before the floor
// (border replication).  fminf/fmaxf keep NaN coordinates inside the image.
template <class P>
__device__ inline float bilinear_clamped(P img, int h, int w, float x, float y)
{
    float xc = fminf(fmaxf(x, 0.0f), (float)(w - 1));
    float yc = fminf(fmaxf(y, 0.0f), (float)(h - 1));
    int x0 = (int)floorf(xc), y0 = (int)floorf(yc);
    x0 = clampi(x0, 0, w - 1);
    y0 = clampi(y0, 0, h - 1);
    float fx = xc - (float)x0, fy = yc - (float)y0;
    int x1 = min(x0 + 1, w - 1), y1 = min(y0 + 1, h - 1);
    auto r0 = img + (int64_t)y0 * w;
    auto r1 = img + (int64_t)y1 * w;
    float top = (1.0f - fx) * r0[x0] + fx * r0[x1];
    float bot = (1.0f - fx) * r1[x0] + fx * r1[x1];
    return (1.0f - fy) * top + fy * bot;
}

// A pointer value that is the same in every lane, made provably uniform
// (scalar registers) for the compiler.
template <class T>
__device__ inline T* uniform_ptr(T* p)
{
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return reinterpret_cast<T*>(((uint64_t)hi << 32) | lo);
}
__device__ inline int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Raw buffer access: a uniform resource descriptor (base, size in bytes) and
// 32-bit byte offsets; reads outside [0, bytes) return 0 instead of faulting.
// Descriptor word 3 = 0x00020000 (32-bit data, gfx9 family).
__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void* p, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(uniform_ptr(const_cast<void*>(p)), (short)0,
                                             (int)__builtin_amdgcn_readfirstlane(bytes), 0x00020000);
}
__device__ inline float bload(__amdgpu_buffer_rsrc_t r, unsigned byte_off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)byte_off, 0, 0));
}
__device__ inline void bstore(__amdgpu_buffer_rsrc_t r, unsigned byte_off, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)byte_off, 0, 0);
}

// The same with a uniform byte offset `soff` (a scalar register, no vector
// add).  Callers keep voff + soff inside the buffer.
__device__ inline float bload_s(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
__device__ inline void bstore_s(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)voff, (int)soff, 0);
}

// Bilinear sample through a buffer descriptor (image of h x w floats).
// xc, yc are clamped to the image by fminf/fmaxf (NaN -> the bound), so the
// floors need no further clamping.
__device__ inline float bilinear_buf(__amdgpu_buffer_rsrc_t img, int h, int w, float x, float y)
{
    const float xc = fminf(fmaxf(x, 0.0f), (float)(w - 1));
    const float yc = fminf(fmaxf(y, 0.0f), (float)(h - 1));
    const float xf = floorf(xc), yf = floorf(yc);
    const unsigned x0 = (unsigned)xf, y0 = (unsigned)yf;
    const float fx = xc - xf, fy = yc - yf;
    const unsigned dx = x0 + 1 < (unsigned)w ? 4u : 0u;
    const unsigned dy = y0 + 1 < (unsigned)h ? 4u * (unsigned)w : 0u;
    const unsigned o = 4u * (y0 * (unsigned)w + x0);
    const float v00 = bload(img, o), v01 = bload(img, o + dx);
    const float v10 = bload(img, o + dy), v11 = bload(img, o + dy + dx);
    const float top = (1.0f - fx) * v00 + fx * v01;
    const float bot = (1.0f - fx) * v10 + fx * v11;
    return (1.0f - fy) * top + fy * bot;
}

// Two halves of bilinear_buf, so that the loads of one row can be in flight
// while the previous row is processed.
struct Bilin {
    float v00, v01, v10, v11, fx, fy;
};
__device__ inline Bilin bilinear_issue(__amdgpu_buffer_rsrc_t img, int h, int w, float x, float y)
{
    Bilin b;
    const float xc = fminf(fmaxf(x, 0.0f), (float)(w - 1));
    const float yc = fminf(fmaxf(y, 0.0f), (float)(h - 1));
    const float xf = floorf(xc), yf = floorf(yc);
    const unsigned x0 = (unsigned)xf, y0 = (unsigned)yf;
    b.fx = xc - xf;
    b.fy = yc - yf;
    const unsigned dx = x0 + 1 < (unsigned)w ? 4u : 0u;
    const unsigned dy = y0 + 1 < (unsigned)h ? 4u * (unsigned)w : 0u;
    const unsigned o = 4u * (y0 * (unsigned)w + x0);
    b.v00 = bload(img, o);
    b.v01 = bload(img, o + dx);
    b.v10 = bload(img, o + dy);
    b.v11 = bload(img, o + dy + dx);
    return b;
}
// Per-level constants of the bilinear gather below.
struct BilGeom {
    float wm1, hm1;   // last column / row
    float wm2, hm2;   // largest left / top corner: max(w - 2, 0), max(h - 2, 0)
    float wf;         // row length
    unsigned dx, dy;  // byte steps to the right / lower neighbours (0 for a 1-px dimension)
};
__device__ inline BilGeom bil_geom(int h, int w)
{
    BilGeom g;
    g.wm1 = (float)(w - 1);
    g.hm1 = (float)(h - 1);
    g.wm2 = (float)max(w - 2, 0);
    g.hm2 = (float)max(h - 2, 0);
    g.wf = (float)w;
    g.dx = w > 1 ? 4u : 0u;
    g.dy = h > 1 ? 4u * (unsigned)w : 0u;
    return g;
}
// Gather half of a bilinear sample whose 2 x 2 cell always lies inside the
// image: the position is clamped to [0, w-1] x [0, h-1], the cell's corner to
// [0, w-2] x [0, h-2], so a sample on the last column or row takes weight 1
// on the far corner instead of weight 0 on a neighbour outside; blended with
// lerp_ends (exact at both weights 0 and 1), it returns that pixel exactly.
// One vector offset, the neighbours through the uniform byte steps
// (y0 w + x0 < 2^24 is exact in the fma).
__device__ inline Bilin bilinear_issue_g(__amdgpu_buffer_rsrc_t img, const BilGeom& g, float x, float y)
{
    Bilin b;
    const float xc = fminf(fmaxf(x, 0.0f), g.wm1);
    const float yc = fminf(fmaxf(y, 0.0f), g.hm1);
    const float xf = fminf(floorf(xc), g.wm2), yf = fminf(floorf(yc), g.hm2);
    b.fx = xc - xf;
    b.fy = yc - yf;
    const unsigned o = 4u * (unsigned)fmaf(yf, g.wf, xf);
    b.v00 = bload_s(img, o, 0u);
    b.v01 = bload_s(img, o, g.dx);
    b.v10 = bload_s(img, o, g.dy);
    b.v11 = bload_s(img, o, g.dx + g.dy);
    return b;
}

// Lerps as a + f (b - a) with one rounding for the product-sum (fmaf): exact
// for f = 0, and the same instruction sequence in every kernel variant (the
// library is built without automatic contraction).
__device__ inline float lerpf(float a, float b, float f) { return fmaf(f, b - a, a); }
__device__ inline float bilinear_blend(const Bilin& b)
{
    return lerpf(lerpf(b.v00, b.v01, b.fx), lerpf(b.v10, b.v11, b.fx), b.fy);
}
// Lerp as (a - f a) + f b with two fmas: returns a exactly for f = 0 and b
// exactly for f = 1.
__device__ inline float lerp_ends(float a, float b, float f) { return fmaf(f, b, fmaf(-f, a, a)); }
// Blend of a bilinear_issue_g gather.
__device__ inline float bilinear_blend_g(const Bilin& b)
{
    return lerp_ends(lerp_ends(b.v00, b.v01, b.fx), lerp_ends(b.v10, b.v11, b.fx), b.fy);
}

// Bilinear sample (lerp form, see lerpf) through a plain pointer.
template <class P>
__device__ inline float bilinear_lerp(P img, int h, int w, float x, float y)
{
    const float xc = fminf(fmaxf(x, 0.0f), (float)(w - 1));
    const float yc = fminf(fmaxf(y, 0.0f), (float)(h - 1));
    const float xf = floorf(xc), yf = floorf(yc);
    const int x0 = (int)xf, y0 = (int)yf;
    const int x1 = min(x0 + 1, w - 1), y1 = min(y0 + 1, h - 1);
    auto r0 = img + (int64_t)y0 * w;
    auto r1 = img + (int64_t)y1 * w;
    return lerpf(lerpf(r0[x0], r0[x1], xc - xf), lerpf(r1[x0], r1[x1], xc - xf), yc - yf);
}

// Same sample for a global image of fewer than 2^30 pixels, with 32-bit
// unsigned offsets from a uniform base (lets the compiler use the
// scalar-base + 32-bit vector-offset addressing form).  xc, yc are already
// clamped to [0, w-1] x [0, h-1] by fminf/fmaxf (NaN -> the bound), so the
// floors need no further clamping.
__device__ inline float bilinear_g32(const EBSD_GLOBAL float* __restrict__ img, int h, int w,
                                     float x, float y)
{
    const float xc = fminf(fmaxf(x, 0.0f), (float)(w - 1));
    const float yc = fminf(fmaxf(y, 0.0f), (float)(h - 1));
    const float xf = floorf(xc), yf = floorf(yc);
    const unsigned x0 = (unsigned)xf, y0 = (unsigned)yf;
    const float fx = xc - xf, fy = yc - yf;
    const unsigned dx = x0 + 1 < (unsigned)w ? 1u : 0u;
    const unsigned dy = y0 + 1 < (unsigned)h ? (unsigned)w : 0u;
    const unsigned o = y0 * (unsigned)w + x0;
    const float v00 = img[o], v01 = img[o + dx], v10 = img[o + dy], v11 = img[o + dy + dx];
    const float top = (1.0f - fx) * v00 + fx * v01;
    const float bot = (1.0f - fx) * v10 + fx * v11;
    return (1.0f - fy) * top + fy * bot;
}

// Map the hardware workgroup id so that each XCD (workgroups are dealt
// round-robin to the 8 XCDs) receives a contiguous range of logical units.
__device__ inline int xcd_logical_block(int hw_id, int G)
{
    const int G8 = (G / 8) * 8;
    if (hw_id >= G8) return hw_id;
    return (hw_id & 7) * (G8 >> 3) + (hw_id >> 3);
}

// Fixed-order sum of a pair's per-unit sums: 64 lanes take strided partial
// sums, then an xor butterfly.  Every workgroup that calls it for the same
// data obtains the same value.  Requires >= 64 threads; all must call it.
__device__ inline double pair_sum(const float* __restrict__ part, int nunits, double* sh)
{
    double acc = 0.0;
    if (threadIdx.x < 64) {
        for (int i = threadIdx.x; i < nunits; i += 64) acc += (double)part[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (threadIdx.x == 0) *sh = acc;
    }
    __syncthreads();
    acc = *sh;
    __syncthreads();
    return acc;
}

}  // namespace ebsd
