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

// Outputs of a sweep that does not run because an error was flagged
// before it (a crowded cell, a cut-off above the cell edge, a drift past the
// cells): NaN in every float output and -1 in the counts, written by the
// whole grid, so that no output is left as it was.
__device__ __forceinline__ void fill_error_outputs(int64_t n, float *a, int64_t na, float *b,
                                                   float *c, int32_t *cnt)
{
    const float q = __builtin_nanf("");
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        if (a)
            for (int64_t k = 0; k < na; ++k) a[na * i + k] = q;
        if (b) b[i] = q;
        if (c) c[i] = q;
        if (cnt) cnt[i] = -1;
    }
}

struct CellGeom {
    int cx, cy, cz;
    float ox, oy, oz;
};

__device__ __forceinline__ CellGeom cell_geom(const BoxDesc &B, int c)
{
    CellGeom g;
    int local = c - B.cell_off;
    g.cz = local % B.g[2];
    g.cy = (local / B.g[2]) % B.g[1];
    g.cx = local / (B.g[2] * B.g[1]);
    g.ox = (float)g.cx * B.edge[0];
    g.oy = (float)g.cy * B.edge[1];
    g.oz = (float)g.cz * B.edge[2];
    return g;
}

// Neighbour cell at offset (dx, dy, dz) with periodic wrap; returns its global
// index and the shift that maps its cell-relative positions into the frame of
// the receiver cell: shift = origin_b (+- L when wrapped) - origin_a, formed so
// that every operation is exact in fp32.
__device__ __forceinline__ int neighbour(const BoxDesc &B, const CellGeom &a, int dx, int dy,
                                         int dz, float &sx, float &sy, float &sz)
{
    int bx = a.cx + dx, by = a.cy + dy, bz = a.cz + dz;
    float wx = 0.0f, wy = 0.0f, wz = 0.0f;
    if (bx < 0) { bx += B.g[0]; wx = -B.L[0]; } else if (bx >= B.g[0]) { bx -= B.g[0]; wx = B.L[0]; }
    if (by < 0) { by += B.g[1]; wy = -B.L[1]; } else if (by >= B.g[1]) { by -= B.g[1]; wy = B.L[1]; }
    if (bz < 0) { bz += B.g[2]; wz = -B.L[2]; } else if (bz >= B.g[2]) { bz -= B.g[2]; wz = B.L[2]; }
    sx = ((float)bx * B.edge[0] - a.ox) + wx;
    sy = ((float)by * B.edge[1] - a.oy) + wy;
    sz = ((float)bz * B.edge[2] - a.oz) + wz;
    return B.cell_off + (bx * B.g[1] + by) * B.g[2] + bz;
}

}  // namespace pvl
