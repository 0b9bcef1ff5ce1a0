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
