// Cell binning: a counting sort of the particles into the cells of each box
// (Section 2 of the paper: cells of edge >= the cut-off, each cell's particles
// stored together), finished by a per-cell sort on (x, original index): the
// cell-ordered layout then depends neither on atomic arrival order nor on the
// order of the input, and consecutive particles of a cell form x-slabs.
//
//   k_box_hmax    max cut-off per box (auto grid)
//   k_bin_count   cell of every particle, per-cell counts and max cut-off
//   k_scan        exclusive scan of the counts -> cell_start; occupancy check
//   k_scatter     particles -> scatter-ordered staging records
//   k_cell_finish per cell: order by (x, original index), shift positions to
//                 the cell origin, write the cell-ordered structure of arrays
#include "device_util.h"

namespace pvl {

__global__ void k_box_hmax(const BoxDesc *__restrict__ box, int nbox, int64_t n,
                           const float *__restrict__ h, uint32_t *__restrict__ box_hmax)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t v = 0;
    int b = -1;
    if (p < n) {
        b = box_of_particle(box, nbox, p);
        v = __float_as_uint(kGamma * h[p]);
    }
    // reduce within the wavefront when every lane has the same box
    int b0 = __shfl(b, 0);
    bool same = __all(b == b0);
    if (same) {
        for (int off = 32; off > 0; off >>= 1) {
            uint32_t o = __shfl_xor(v, off);
            v = v > o ? v : o;
        }
        if ((threadIdx.x & 63) == 0 && b0 >= 0) atomicMax(&box_hmax[b0], v);
    } else if (b >= 0) {
        atomicMax(&box_hmax[b], v);
    }
}

__global__ void k_bin_count(const BoxDesc *__restrict__ box, int nbox, int64_t n,
                            const float *__restrict__ pos, const float *__restrict__ h,
                            int32_t *__restrict__ cellid, int32_t *__restrict__ slot,
                            int32_t *__restrict__ count, int *__restrict__ dflags)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const BoxDesc &B = box[box_of_particle(box, nbox, p)];
    float x = wrap_coord(pos[3 * p + 0], B.L[0], 1.0f / B.L[0]);
    float y = wrap_coord(pos[3 * p + 1], B.L[1], 1.0f / B.L[1]);
    float z = wrap_coord(pos[3 * p + 2], B.L[2], 1.0f / B.L[2]);
    int cx = cell_coord(x, B.inv_edge[0], B.g[0]);
    int cy = cell_coord(y, B.inv_edge[1], B.g[1]);
    int cz = cell_coord(z, B.inv_edge[2], B.g[2]);
    int c = B.cell_off + (cx * B.g[1] + cy) * B.g[2] + cz;
    cellid[p] = c;
    // arrival order within the cell; made deterministic later by the
    // per-cell sort on the original index
    slot[p] = atomicAdd(&count[c], 1);
    float H = kGamma * h[p];
    float emin = fminf(B.edge[0], fminf(B.edge[1], B.edge[2]));
    if (!(H <= emin) || !(H > 0.0f)) atomicOr(dflags, kErrGrid);
}

// Single workgroup: exclusive scan of count[0..ncell) into start[0..ncell],
// largest count into dflags[1], overflow flagged.
__global__ void __launch_bounds__(1024) k_scan(int64_t ncell, int32_t *__restrict__ count,
                                                int32_t *__restrict__ start,
                                                int *__restrict__ dflags)
{
    __shared__ int32_t part[1024];
    const int T = blockDim.x;
    int64_t chunk = (ncell + T - 1) / T;
    int64_t b = threadIdx.x * chunk;
    int64_t e = b + chunk < ncell ? b + chunk : ncell;
    int32_t sum = 0, mx = 0;
    for (int64_t c = b; c < e; ++c) {
        int32_t v = count[c];
        sum += v;
        mx = v > mx ? v : mx;
    }
    part[threadIdx.x] = sum;
    __syncthreads();
    // Hillis-Steele inclusive scan over the thread sums
    for (int off = 1; off < T; off <<= 1) {
        int32_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int32_t run = part[threadIdx.x] - sum;
    for (int64_t c = b; c < e; ++c) {
        int32_t v = count[c];
        start[c] = run;
        run += v;
    }
    if (threadIdx.x == T - 1) start[ncell] = part[T - 1];
    for (int off = 32; off > 0; off >>= 1) {
        int32_t o = __shfl_xor(mx, off);
        mx = mx > o ? mx : o;
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&dflags[1], mx);
        if (mx > PV_MAX_CELL) atomicOr(&dflags[0], kErrOverflow);
    }
}

// Staging record of one particle: 32 bytes, written with one aligned store pair.
__global__ void k_scatter(const BoxDesc *__restrict__ box, int nbox, int64_t n,
                          const float *__restrict__ pos, const float *__restrict__ h,
                          const float *__restrict__ mass, const int32_t *__restrict__ cellid,
                          const int32_t *__restrict__ slot, const int32_t *__restrict__ start,
                          float4 *__restrict__ stage)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const BoxDesc &B = box[box_of_particle(box, nbox, p)];
    float x = wrap_coord(pos[3 * p + 0], B.L[0], 1.0f / B.L[0]);
    float y = wrap_coord(pos[3 * p + 1], B.L[1], 1.0f / B.L[1]);
    float z = wrap_coord(pos[3 * p + 2], B.L[2], 1.0f / B.L[2]);
    int64_t q = start[cellid[p]] + slot[p];
    stage[2 * q] = make_float4(x, y, z, kGamma * h[p]);
    stage[2 * q + 1] = make_float4(mass[p], __int_as_float((int)p), 0.f, 0.f);
}

// One workgroup per cell: order the cell's particles by (cell-relative x,
// original index) with a bucket sort in LDS (buckets are equal x ranges of
// the cell; the exact rank inside a bucket compares bucket mates), shift the
// positions to the cell origin, write the cell-ordered arrays and the cell's
// largest cut-off.
constexpr int kFinishMaxBuckets = 1024;

__global__ void __launch_bounds__(kBlock) k_cell_finish(
    const BoxDesc *__restrict__ box, const int32_t *__restrict__ cell_box,
    const int32_t *__restrict__ start, const float4 *__restrict__ stage,
    float4 *__restrict__ xyzm, float *__restrict__ Hout, int32_t *__restrict__ orig,
    uint32_t *__restrict__ cell_hmax)
{
    __shared__ float key[PV_MAX_CELL];
    __shared__ uint16_t slot[PV_MAX_CELL];
    __shared__ uint16_t border[PV_MAX_CELL];
    __shared__ uint32_t hist[kFinishMaxBuckets];
    __shared__ uint32_t hred[kBlock / 64];
    const int c = blockIdx.x;
    const int s0 = start[c];
    const int cnt = start[c + 1] - s0;
    if (cnt <= 0 || cnt > PV_MAX_CELL) {
        if (threadIdx.x == 0) cell_hmax[c] = 0u;
        return;
    }
    const BoxDesc &B = box[cell_box[c]];
    const int local = c - B.cell_off;
    const int cz = local % B.g[2];
    const int cy = (local / B.g[2]) % B.g[1];
    const int cx = local / (B.g[2] * B.g[1]);
    const float ox = (float)cx * B.edge[0], oy = (float)cy * B.edge[1], oz = (float)cz * B.edge[2];
    int NB = cnt <= 256 ? 128 : next_pow2(cnt) >> 2;
    NB = NB > kFinishMaxBuckets ? kFinishMaxBuckets : NB;
    const float scale = (float)NB / B.edge[0];
    auto bucket = [&](float xr) {
        int b = (int)(xr * scale);
        return b < 0 ? 0 : (b >= NB ? NB - 1 : b);
    };
    for (int b = threadIdx.x; b < NB; b += blockDim.x) hist[b] = 0u;
    __syncthreads();
    for (int r = threadIdx.x; r < cnt; r += blockDim.x) {
        const float xr = stage[2 * (int64_t)(s0 + r)].x - ox;
        key[r] = xr;
        slot[r] = (uint16_t)atomicAdd(&hist[bucket(xr)], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        const int per = (NB + 63) >> 6;
        uint32_t loc = 0;
        for (int k = 0; k < per; ++k) {
            const int q = lane * per + k;
            if (q < NB) loc += hist[q];
        }
        uint32_t inc = loc;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = (uint32_t)__shfl_up((int)inc, off);
            if (lane >= off) inc += o;
        }
        uint32_t run = inc - loc;
        for (int k = 0; k < per; ++k) {
            const int q = lane * per + k;
            if (q < NB) {
                const uint32_t v = hist[q];
                hist[q] = run;
                run += v;
            }
        }
    }
    __syncthreads();
    for (int r = threadIdx.x; r < cnt; r += blockDim.x)
        border[hist[bucket(key[r])] + slot[r]] = (uint16_t)r;
    __syncthreads();
    uint32_t hm = 0u;
    for (int r = threadIdx.x; r < cnt; r += blockDim.x) {
        const float k = key[r];
        const int b = bucket(k);
        const int q0 = (int)hist[b];
        const int q1 = b + 1 < NB ? (int)hist[b + 1] : cnt;
        const float4 a = stage[2 * (int64_t)(s0 + r)];
        const float4 m = stage[2 * (int64_t)(s0 + r) + 1];
        const int my_orig = __float_as_int(m.y);
        int rank = q0;
        for (int q = q0; q < q1; ++q) {
            const int r2 = border[q];
            const float k2 = key[r2];
            bool before = k2 < k;
            if (k2 == k && r2 != r)
                before = __float_as_int(stage[2 * (int64_t)(s0 + r2) + 1].y) < my_orig;
            rank += before;
        }
        xyzm[s0 + rank] = make_float4(k, a.y - oy, a.z - oz, m.x);
        Hout[s0 + rank] = a.w;
        orig[s0 + rank] = my_orig;
        hm = max(hm, __float_as_uint(a.w));
    }
    // largest cut-off of the cell (positive floats order as their bits)
    for (int off = 32; off > 0; off >>= 1) hm = max(hm, (uint32_t)__shfl_xor((int)hm, off));
    if ((threadIdx.x & 63) == 0) hred[threadIdx.x >> 6] = hm;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t mx = 0u;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) mx = max(mx, hred[w]);
        cell_hmax[c] = mx;
    }
}

__global__ void k_cell_box(const BoxDesc *__restrict__ box, int nbox, int64_t ncell,
                           int32_t *__restrict__ cell_box)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    int lo = 0, hi = nbox - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (box[mid].cell_off <= c) lo = mid; else hi = mid - 1;
    }
    cell_box[c] = lo;
}

__global__ void k_zero(uint32_t *__restrict__ p, int64_t words)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < words) p[i] = 0u;
}

static inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_zero(hipStream_t st, void *p, int64_t words)
{
    if (words <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3(blocks_for(words, 256)), dim3(256), 0, st, (uint32_t *)p, words);
    return hipGetLastError();
}

hipError_t launch_box_hmax(hipStream_t st, const DevCells &c, int nbox, int64_t n,
                           const float *h)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_box_hmax, dim3(blocks_for(n, 256)), dim3(256), 0, st, c.box, nbox, n,
                       h, c.box_hmax);
    return hipGetLastError();
}

hipError_t launch_bin(hipStream_t st, const DevCells &c, int nbox, int64_t n, int64_t ncell,
                      const float *pos, const float *h, const float *mass, int *dflags)
{
    hipLaunchKernelGGL(k_cell_box, dim3(blocks_for(ncell, 256)), dim3(256), 0, st, c.box, nbox,
                       ncell, c.cell_box);
    if (n > 0) {
        hipLaunchKernelGGL(k_bin_count, dim3(blocks_for(n, 256)), dim3(256), 0, st, c.box, nbox,
                           n, pos, h, c.cellid, c.slot, c.cursor, dflags);
    }
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, ncell, c.cursor, c.cell_start, dflags);
    if (n > 0) {
        hipLaunchKernelGGL(k_scatter, dim3(blocks_for(n, 256)), dim3(256), 0, st, c.box, nbox, n,
                           pos, h, mass, c.cellid, c.slot, c.cell_start, c.stage);
    }
    hipLaunchKernelGGL(k_cell_finish, dim3((unsigned)ncell), dim3(kBlock), 0, st, c.box,
                       c.cell_box, c.cell_start, c.stage, c.xyzm, c.H, c.orig, c.cell_hmax);
    return hipGetLastError();
}

}  // namespace pvl
