// Small device helpers shared by the libpvl kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pvl_internal.h"

namespace pvl {

__device__ __forceinline__ uint32_t float_to_ordered(float f)
{
    uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ __forceinline__ float ordered_to_float(uint32_t b)
{
    return __uint_as_float((b & 0x80000000u) ? (b & 0x7fffffffu) : ~b);
}

// Box that owns global particle p (binary search over the box offsets).
__device__ __forceinline__ int box_of_particle(const BoxDesc *box, int nbox, int64_t p)
{
    int lo = 0, hi = nbox - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (box[mid].part_off <= p) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Wrap one coordinate into [0, L) in fp32 and return its cell index.
__device__ __forceinline__ float wrap_coord(float x, float L, float invL)
{
    float y = x - L * floorf(x * invL);
    return (y >= L) ? 0.0f : y;
}

__device__ __forceinline__ int cell_coord(float x, float inv_edge, int g)
{
    int c = (int)(x * inv_edge);
    return c < 0 ? 0 : (c >= g ? g - 1 : c);
}

// Projection of a cell-relative position on axis s (d_s / |d_s|).
__device__ __forceinline__ float proj_key(float x, float y, float z, int s)
{
    float e[3];
    dir_axis(s, e);
    return fmaf(x, e[0], fmaf(y, e[1], z * e[2]));
}

// Block-wide bitonic sort of `nseg` independent segments of `len` (power of
// two) uint64 keys in LDS, ascending.  All threads of the block must call it.
__device__ inline void bitonic_sort_segments(uint64_t *s, int len, int nseg)
{
    const int half = len >> 1;
    const int pairs = half * nseg;
    for (int k = 2; k <= len; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < pairs; t += blockDim.x) {
                int seg = t / half;
                int q = t - seg * half;
                int lo = (q / j) * 2 * j + (q % j);
                int hi = lo + j;
                uint64_t *b = s + (size_t)seg * len;
                uint64_t a = b[lo], c = b[hi];
                bool up = (lo & k) == 0;
                if ((a > c) == up) { b[lo] = c; b[hi] = a; }
            }
            __syncthreads();
        }
    }
}

__device__ __forceinline__ int next_pow2(int v)
{
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

}  // namespace pvl
