// Cell binning: a counting sort of the particles into the cells of each box
// (Section 2 of the paper: cells of edge >= the cut-off, each cell's particles
// stored together), finished by a per-cell sort on (x, original index): the
// cell-ordered layout then depends neither on arrival order nor on the order
// of the input, and consecutive particles of a cell form x-slabs.
//
// The counting sort needs no global atomics.  The particles of each box are
// cut into chunks (one workgroup each); a workgroup counts its chunk's
// particles per cell in LDS (the LDS atomic gives each particle its slot among
// the chunk's particles of that cell) and writes the counts as one row of the
// box's chunks x cells matrix (coalesced).  A pass down every cell's column
// turns the counts into the cell's offsets per chunk and its total; the scan
// of the totals gives the cell starts.
//
//   k_box_hmax    max cut-off per box (auto grid)
//   k_bin_local   cell of every particle, per-chunk cell counts, cut-off check
//   k_bin_columns per cell: owning box, offsets of the chunks' shares, particle
//                 count, the lists of the cells above 256 particles
//   k_scan        exclusive scan of the counts -> cell_start; occupancy check
//                 (k_tile_sums / k_scan / k_tile_scan when there are many cells)
//   k_scatter     particles -> scatter-ordered staging records
//   k_cell_finish per cell: order by (x, original index), shift positions to
//                 the cell origin, write the cell-ordered structure of arrays
//                 and the cell's largest cut-off (one kernel per size class)
#include "device_util.h"

namespace pvl {

// Largest cut-off per box.  A workgroup reduces a contiguous range of
// kBoxHmaxSpan particles; when the range lies in one box the workgroup issues a
// single atomic, otherwise (a box boundary inside the range) each lane flushes
// its running maximum whenever its box changes.
constexpr int kBoxHmaxSpan = 16 * kBlock;

__global__ void __launch_bounds__(kBlock) k_box_hmax(const BoxDesc *__restrict__ box, int nbox,
                                                     int64_t n, const float *__restrict__ h,
                                                     uint32_t *__restrict__ box_hmax)
{
    __shared__ uint32_t red[kBlock / 64];
    const int64_t p0 = (int64_t)blockIdx.x * kBoxHmaxSpan;
    const int64_t p1 = p0 + kBoxHmaxSpan < n ? p0 + kBoxHmaxSpan : n;
    const int b0 = box_of_particle(box, nbox, p0);
    const bool one_box = box_of_particle(box, nbox, p1 - 1) == b0;
    uint32_t v = 0;   // positive floats order as their bits
    int cur = b0;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
        if (!one_box) {
            const int b = box_of_particle(box, nbox, p);
            if (b != cur) {
                if (v) atomicMax(&box_hmax[cur], v);
                cur = b;
                v = 0;
            }
        }
        v = max(v, __float_as_uint(kGamma * h[p]));
    }
    if (!one_box) {
        if (v) atomicMax(&box_hmax[cur], v);
        return;
    }
    for (int off = 32; off > 0; off >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t m = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = max(m, red[w]);
        atomicMax(&box_hmax[b0], m);
    }
}

// Cells per LDS histogram pass of k_bin_local (64 KB); boxes with more cells
// are counted in several passes over the chunk.
constexpr int kBinSeg = 16384;
constexpr int kBinThreads = 1024;

// One workgroup per chunk: blocks[g] = (box, chunk index within the box, first
// particle, end).  Writes cellid and slot of every particle and the chunk's
// row of the box's count matrix: binm[moff + chunk * cells of the box + local cell].
__global__ void __launch_bounds__(kBinThreads) k_bin_local(
    const BoxDesc *__restrict__ box, const int4 *__restrict__ blocks,
    const float *__restrict__ pos, const float *__restrict__ h, int32_t *__restrict__ cellid,
    int32_t *__restrict__ slot, int32_t *__restrict__ binm, int *__restrict__ dflags,
    int64_t ncell, int32_t *__restrict__ lists, uint32_t *__restrict__ dx_all)
{
    __shared__ uint32_t hist[kBinSeg];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        // per-build state read later: the largest occupancy (raised by the
        // scan), the cell lists of the finish, the structure's displacement
        // bound
        dflags[1] = 0;
        for (int k = 0; k < kCellLists; ++k) cell_list(lists, ncell, k)[0] = 0;
        *dx_all = 0u;
    }
    const int4 blk = blocks[blockIdx.x];
    const BoxDesc &B = box[blk.x];
    const int ncb = B.g[0] * B.g[1] * B.g[2];
    const float inv0 = 1.0f / B.L[0], inv1 = 1.0f / B.L[1], inv2 = 1.0f / B.L[2];
    const float emin = fminf(B.edge[0], fminf(B.edge[1], B.edge[2]));
    bool bad = false;
    for (int seg = 0; seg < ncb; seg += kBinSeg) {
        const int segn = min(kBinSeg, ncb - seg);
        for (int t = threadIdx.x; t < segn; t += blockDim.x) hist[t] = 0u;
        __syncthreads();
        for (int p = blk.z + threadIdx.x; p < blk.w; p += blockDim.x) {
            int cl;
            if (seg == 0) {
                const float x = wrap_coord(pos[3 * (int64_t)p + 0], B.L[0], inv0);
                const float y = wrap_coord(pos[3 * (int64_t)p + 1], B.L[1], inv1);
                const float z = wrap_coord(pos[3 * (int64_t)p + 2], B.L[2], inv2);
                const int cx = cell_coord(x, B.inv_edge[0], B.g[0]);
                const int cy = cell_coord(y, B.inv_edge[1], B.g[1]);
                const int cz = cell_coord(z, B.inv_edge[2], B.g[2]);
                cl = (cx * B.g[1] + cy) * B.g[2] + cz;
                cellid[p] = B.cell_off + cl;
                const float H = kGamma * h[p];
                bad |= !(H <= emin) || !(H > 0.0f);
            } else {
                cl = cellid[p] - B.cell_off;
            }
            // arrival order within the chunk's share of the cell; made
            // deterministic later by the per-cell sort on the original index
            if (cl >= seg && cl < seg + segn) slot[p] = (int32_t)atomicAdd(&hist[cl - seg], 1u);
        }
        __syncthreads();
        for (int t = threadIdx.x; t < segn; t += blockDim.x)
            binm[(int64_t)B.moff + (int64_t)blk.y * ncb + seg + t] = (int32_t)hist[t];
        __syncthreads();
    }
    if (bad) atomicOr(dflags, kErrGrid);
}

// Per cell: the owning box (cell_box) and a cleared displacement bound; the
// chunks' counts become exclusive offsets (in place) and the cell's particle
// count goes to count[c]; a cell above 256 particles goes on the cell lists
// of its size class.  Reads and writes are coalesced across the cells of a
// box.
__global__ void __launch_bounds__(256) k_bin_columns(const BoxDesc *__restrict__ box, int nbox,
                                                     int64_t ncell, int32_t *__restrict__ binm,
                                                     int32_t *count, int32_t *__restrict__ cell_box,
                                                     float *__restrict__ cell_dx,
                                                     int32_t *__restrict__ lists)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < ncell) {
        int lo = 0, hi = nbox - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (box[mid].cell_off <= c) lo = mid; else hi = mid - 1;
        }
        cell_box[c] = lo;
        cell_dx[c] = 0.0f;
        const BoxDesc &B = box[lo];
        const int64_t ncb = (int64_t)B.g[0] * B.g[1] * B.g[2];
        int32_t *col = binm + B.moff + (c - B.cell_off);
        int32_t run = 0;
        // eight independent loads in flight per step
        for (int j0 = 0; j0 < B.nblk; j0 += 8) {
            int32_t v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = j0 + k < B.nblk ? col[(j0 + k) * ncb] : 0;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (j0 + k < B.nblk) col[(j0 + k) * ncb] = run;
                run += v[k];
            }
        }
        count[c] = run;
        // the rare size classes' cell lists: the finish above 256 particles,
        // the sorts of 257..kSortSmallMax, up to kSortLargeMax and larger
        if (run > 256) {
            int32_t *l = cell_list(lists, ncell, kListLarge);
            l[1 + atomicAdd(&l[0], 1)] = (int32_t)c;
            if (run <= PV_MAX_CELL) {
                l = cell_list(lists, ncell,
                              run > kSortLargeMax ? kListHuge
                                                  : (run > kSortSmallMax ? kListBig : kListMid));
                l[1 + atomicAdd(&l[0], 1)] = (int32_t)c;
            }
        }
    }
}

// Single workgroup: exclusive scan of count[0..ncell) into start[0..ncell]
// (the two may be the same array); with dflags, the largest count goes to
// dflags[1] and overflow is flagged.
__global__ void __launch_bounds__(1024) k_scan(int64_t ncell, const int32_t *count, int32_t *start,
                                                int *__restrict__ dflags)
{
    __shared__ int32_t wsum[1024 / 64];
    const int T = blockDim.x;   // a multiple of 64, at most 1024
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int64_t chunk = (ncell + T - 1) / T;
    int64_t b = threadIdx.x * chunk;
    int64_t e = b + chunk < ncell ? b + chunk : ncell;
    int32_t sum = 0, mx = 0;
    for (int64_t c = b; c < e; ++c) {
        int32_t v = count[c];
        sum += v;
        mx = v > mx ? v : mx;
    }
    // inclusive scan of the thread sums: within each wavefront by shuffles,
    // then the wavefront totals before each wavefront from LDS
    int32_t inc = sum;
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t o = __shfl_up(inc, off);
        if (lane >= off) inc += o;
    }
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    for (int w = 0; w < wid; ++w) inc += wsum[w];
    int32_t run = inc - sum;
    for (int64_t c = b; c < e; ++c) {
        int32_t v = count[c];
        start[c] = run;
        run += v;
    }
    if (threadIdx.x == T - 1) start[ncell] = inc;
    if (!dflags) return;
    for (int off = 32; off > 0; off >>= 1) {
        int32_t o = __shfl_xor(mx, off);
        mx = mx > o ? mx : o;
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&dflags[1], mx);
        if (mx > PV_MAX_CELL) atomicOr(&dflags[0], kErrOverflow);
    }
}

// Many cells: the counts are scanned in tiles of kScanTile.  k_tile_sums sums
// every tile (and checks occupancy), k_scan scans the tile sums into tile
// offsets, k_tile_scan scans each tile from its offset.
constexpr int kScanThreads = 1024;
constexpr int kScanPer = 8;
static_assert(kScanTile == kScanThreads * kScanPer, "scan tile");

__device__ __forceinline__ int32_t block_exclusive_scan(int32_t v, int32_t *red, int32_t &total)
{
    // inclusive scan in each wave, then over the wave totals
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int32_t inc = v;
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t o = __shfl_up(inc, off);
        if (lane >= off) inc += o;
    }
    if (lane == 63) red[wave] = inc;
    __syncthreads();
    if (wave == 0) {
        const int nw = (int)(blockDim.x >> 6);
        int32_t w = lane < nw ? red[lane] : 0;
        int32_t winc = w;
        for (int off = 1; off < 64; off <<= 1) {
            const int32_t o = __shfl_up(winc, off);
            if (lane >= off) winc += o;
        }
        if (lane < nw) red[lane] = winc - w;
        if (lane == nw - 1) red[63] = winc;
    }
    __syncthreads();
    total = red[63];
    return red[wave] + inc - v;
}

__global__ void __launch_bounds__(kScanThreads) k_tile_sums(int64_t ncell,
                                                            const int32_t *__restrict__ count,
                                                            int32_t *__restrict__ tsum,
                                                            int *__restrict__ dflags)
{
    __shared__ int32_t red[64];
    const int64_t c0 = (int64_t)blockIdx.x * kScanTile;
    int32_t sum = 0, mx = 0;
    for (int k = 0; k < kScanPer; ++k) {
        const int64_t c = c0 + (int64_t)k * kScanThreads + threadIdx.x;   // coalesced
        const int32_t v = c < ncell ? count[c] : 0;
        sum += v;
        mx = max(mx, v);
    }
    for (int off = 32; off > 0; off >>= 1) {
        sum += __shfl_xor(sum, off);
        mx = max(mx, __shfl_xor(mx, off));
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
        tsum[blockIdx.x] = t;
    }
    if (dflags && (threadIdx.x & 63) == 0) {
        atomicMax(&dflags[1], mx);
        if (mx > PV_MAX_CELL) atomicOr(&dflags[0], kErrOverflow);
    }
}

// count and start may be the same array (each thread reads its values first).
__global__ void __launch_bounds__(kScanThreads) k_tile_scan(int64_t ncell, const int32_t *count,
                                                            const int32_t *__restrict__ toff,
                                                            int32_t *start)
{
    __shared__ int32_t red[64];
    const int64_t c0 = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    int32_t v[kScanPer];
    int32_t sum = 0;
    for (int k = 0; k < kScanPer; ++k) {
        v[k] = c0 + k < ncell ? count[c0 + k] : 0;
        sum += v[k];
    }
    int32_t total;
    int32_t run = toff[blockIdx.x] + block_exclusive_scan(sum, red, total);
    for (int k = 0; k < kScanPer; ++k) {
        if (c0 + k < ncell) start[c0 + k] = run;
        run += v[k];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) start[ncell] = toff[gridDim.x];
}

// Staging record of one particle: 32 bytes, written with one aligned store pair.
__global__ void k_scatter(const BoxDesc *__restrict__ box, int nbox, int64_t n, int chunk,
                          const float *__restrict__ pos, const float *__restrict__ h,
                          const float *__restrict__ mass, const int32_t *__restrict__ cellid,
                          const int32_t *__restrict__ slot, const int32_t *__restrict__ binm,
                          const int32_t *__restrict__ start, float4 *__restrict__ stage)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const BoxDesc &B = box[box_of_particle(box, nbox, p)];
    const int j = (int)((p - B.part_off) / chunk);
    float x = wrap_coord(pos[3 * p + 0], B.L[0], 1.0f / B.L[0]);
    float y = wrap_coord(pos[3 * p + 1], B.L[1], 1.0f / B.L[1]);
    float z = wrap_coord(pos[3 * p + 2], B.L[2], 1.0f / B.L[2]);
    const int64_t ncb = (int64_t)B.g[0] * B.g[1] * B.g[2];
    const int c = cellid[p];
    const int64_t q = start[c] + binm[(int64_t)B.moff + j * ncb + (c - B.cell_off)] + slot[p];
    stage[2 * q] = make_float4(x, y, z, kGamma * h[p]);
    stage[2 * q + 1] = make_float4(mass[p], __int_as_float((int)p), 0.f, 0.f);
}

// Common mass of a cell from the workgroup's smallest and largest masses
// (red: one pair per wavefront): the mass itself when they agree, NaN when
// they differ (see DevCells::cell_m).
__device__ __forceinline__ void reduce_cell_mass(float mn, float mx, float2 *red, int nwave,
                                                 float *out)
{
    for (int off = 32; off > 0; off >>= 1) {
        mn = fminf(mn, __shfl_xor(mn, off));
        mx = fmaxf(mx, __shfl_xor(mx, off));
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = make_float2(mn, mx);
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < nwave; ++w) {
            mn = fminf(mn, red[w].x);
            mx = fmaxf(mx, red[w].y);
        }
        *out = mn == mx ? mn : __builtin_nanf("");
    }
}

// One workgroup per cell: order the cell's particles by (cell-relative x,
// original index) with a bucket sort in LDS (buckets are equal x ranges of
// the cell; the exact rank inside a bucket compares bucket mates), shift the
// positions to the cell origin, write the cell-ordered arrays and the cell's
// largest cut-off.  Cells of at most MAXC particles (64 or 256) take a
// workgroup of MAXC threads, one particle each, with small LDS arrays, so
// that many cells share a compute unit; larger cells take k_cell_finish_large.
template <int MAXC, int NB>
__global__ void __launch_bounds__(MAXC) k_cell_finish_small(
    const BoxDesc *__restrict__ box, const int32_t *__restrict__ cell_box,
    const int32_t *__restrict__ start, const float4 *__restrict__ stage,
    float4 *__restrict__ xyzm, float *__restrict__ Hout, int32_t *__restrict__ orig,
    uint32_t *__restrict__ cell_hmax, float *__restrict__ cell_m, int min_cnt)
{
    __shared__ float key[MAXC];
    __shared__ int32_t okey[MAXC];
    __shared__ uint16_t border[MAXC];
    __shared__ uint32_t hist[NB];
    __shared__ uint32_t hred[MAXC / 64];
    __shared__ float2 mred[MAXC / 64];
    const int c = blockIdx.x;
    const int s0 = start[c];
    const int cnt = start[c + 1] - s0;
    if (cnt > MAXC || cnt < min_cnt) return;   // another class (cells above 256: listed)
    if (cnt == 0) {
        if (threadIdx.x == 0) {
            cell_hmax[c] = 0u;
            cell_m[c] = INFINITY;   // empty
        }
        return;
    }
    const BoxDesc &B = box[cell_box[c]];
    const CellGeom G = cell_geom(B, c);
    const float scale = (float)NB / B.edge[0];
    for (int t = threadIdx.x; t < NB; t += blockDim.x) hist[t] = 0u;
    const int r = threadIdx.x;
    const bool on = r < cnt;
    float4 a = make_float4(0.f, 0.f, 0.f, 0.f), m = a;
    if (on) {
        a = stage[2 * (int64_t)(s0 + r)];
        m = stage[2 * (int64_t)(s0 + r) + 1];
    }
    const float k = a.x - G.ox;
    const int my_orig = __float_as_int(m.y);
    key[r] = k;
    okey[r] = my_orig;
    int b = (int)(k * scale);
    b = b < 0 ? 0 : (b >= NB ? NB - 1 : b);
    __syncthreads();
    const uint32_t sl = on ? atomicAdd(&hist[b], 1u) : 0u;
    __syncthreads();
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        constexpr int per = NB >= 64 ? NB / 64 : 1;
        uint32_t v[per];
        uint32_t loc = 0;
#pragma unroll
        for (int q = 0; q < per; ++q) {
            v[q] = lane * per + q < NB ? hist[lane * per + q] : 0u;
            loc += v[q];
        }
        uint32_t inc = loc;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = (uint32_t)__shfl_up((int)inc, off);
            if (lane >= off) inc += o;
        }
        uint32_t run = inc - loc;
#pragma unroll
        for (int q = 0; q < per; ++q) {
            if (lane * per + q < NB) hist[lane * per + q] = run;
            run += v[q];
        }
    }
    __syncthreads();
    const int q0 = (int)hist[b];
    if (on) border[q0 + (int)sl] = (uint16_t)r;
    __syncthreads();
    uint32_t hm = 0u;
    if (on) {
        const int q1 = b + 1 < NB ? (int)hist[b + 1] : cnt;
        int rank = q0;
        for (int q = q0; q < q1; ++q) {
            const int r2 = border[q];
            const float k2 = key[r2];
            rank += (k2 < k) || (k2 == k && okey[r2] < my_orig);
        }
        xyzm[s0 + rank] = make_float4(k, a.y - G.oy, a.z - G.oz, m.x);
        Hout[s0 + rank] = a.w;
        orig[s0 + rank] = my_orig;
        hm = __float_as_uint(a.w);
    }
    // largest cut-off of the cell (positive floats order as their bits)
    for (int off = 32; off > 0; off >>= 1) hm = max(hm, (uint32_t)__shfl_xor((int)hm, off));
    if ((threadIdx.x & 63) == 0) hred[threadIdx.x >> 6] = hm;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t mx = 0u;
        for (int w = 0; w < MAXC / 64; ++w) mx = max(mx, hred[w]);
        cell_hmax[c] = mx;
    }
    reduce_cell_mass(on ? m.x : INFINITY, on ? m.x : -INFINITY, mred, MAXC / 64, cell_m + c);
}

constexpr int kFinishMaxBuckets = 1024;



__global__ void __launch_bounds__(kBlock) k_cell_finish_large(
    const BoxDesc *__restrict__ box, const int32_t *__restrict__ cell_box,
    const int32_t *__restrict__ start, const float4 *__restrict__ stage,
    float4 *__restrict__ xyzm, float *__restrict__ Hout, int32_t *__restrict__ orig,
    uint32_t *__restrict__ cell_hmax, float *__restrict__ cell_m,
    const int32_t *__restrict__ large)
{
    __shared__ float key[PV_MAX_CELL];
    __shared__ uint16_t slot[PV_MAX_CELL];
    __shared__ uint16_t border[PV_MAX_CELL];
    __shared__ uint32_t hist[kFinishMaxBuckets];
    __shared__ uint32_t hred[kBlock / 64];
    __shared__ float2 mred[kBlock / 64];
    // the cells above 256 particles (listed by the column pass), a grid's
    // worth at a time
    const int nlarge = large[0];
    for (int item = blockIdx.x; item < nlarge; item += gridDim.x) {
        const int c = large[1 + item];
        const int s0 = start[c];
        const int cnt = start[c + 1] - s0;
        if (cnt > PV_MAX_CELL) {
            if (threadIdx.x == 0) {
                cell_hmax[c] = 0u;
                cell_m[c] = __builtin_nanf("");
            }
            continue;
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
        float mmin = INFINITY, mmax = -INFINITY;
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
            mmin = fminf(mmin, m.x);
            mmax = fmaxf(mmax, m.x);
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
        reduce_cell_mass(mmin, mmax, mred, (int)(blockDim.x >> 6), cell_m + c);
        __syncthreads();   // the next cell reuses the LDS
    }
}

// One workgroup per cell: add each particle's displacement (input order) to
// its cell-relative position, and the largest displacement of the cell to the
// cell's accumulated bound (single writer); the structure-wide largest bound
// goes to dx_all.
__global__ void __launch_bounds__(kBlock) k_drift(const int32_t *__restrict__ start,
                                                  const int32_t *__restrict__ orig,
                                                  const float *__restrict__ disp,
                                                  float4 *__restrict__ xyzm,
                                                  float *__restrict__ cell_dx,
                                                  uint32_t *__restrict__ dx_all)
{
    __shared__ float red[kBlock / 64];
    const int c = blockIdx.x;
    const int s0 = start[c], s1 = start[c + 1];
    float mx = 0.0f;
    for (int p = s0 + threadIdx.x; p < s1; p += blockDim.x) {
        const int64_t o = orig[p];
        const float dx = disp[3 * o + 0], dy = disp[3 * o + 1], dz = disp[3 * o + 2];
        float4 q = xyzm[p];
        q.x += dx;
        q.y += dy;
        q.z += dz;
        xyzm[p] = q;
        // |d| rounded up a little so that the bound stays an upper bound
        mx = fmaxf(mx, sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz))) * 1.0000005f);
    }
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        float m = 0.0f;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = fmaxf(m, red[w]);
        const float acc = (cell_dx[c] + m) * 1.0000005f;
        cell_dx[c] = acc;
        atomicMax(dx_all, __float_as_uint(acc));
    }
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

hipError_t launch_drift(hipStream_t st, const DevCells &c, int64_t ncell, const float *disp)
{
    if (ncell == 0) return hipSuccess;
    hipLaunchKernelGGL(k_drift, dim3((unsigned)ncell), dim3(kBlock), 0, st, c.cell_start, c.orig,
                       disp, c.xyzm, c.cell_dx, c.dx_all);
    return hipGetLastError();
}

hipError_t launch_box_hmax(hipStream_t st, const DevCells &c, int nbox, int64_t n,
                           const float *h)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_box_hmax, dim3(blocks_for(n, kBoxHmaxSpan)), dim3(kBlock), 0, st, c.box,
                       nbox, n, h, c.box_hmax);
    return hipGetLastError();
}

// Exclusive scan of count[0..len) into start[0..len] (in place allowed);
// with dflags, occupancy is checked on the way.
static void launch_scan(hipStream_t st, int64_t len, const int32_t *count, int32_t *start,
                        int32_t *scan_tmp, int *dflags)
{
    if (len <= kScanTile) {
        hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, len, count, start, dflags);
        return;
    }
    const unsigned nt = (unsigned)((len + kScanTile - 1) / kScanTile);
    hipLaunchKernelGGL(k_tile_sums, dim3(nt), dim3(kScanThreads), 0, st, len, count, scan_tmp,
                       dflags);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, (int64_t)nt, scan_tmp, scan_tmp,
                       (int *)nullptr);
    hipLaunchKernelGGL(k_tile_scan, dim3(nt), dim3(kScanThreads), 0, st, len, count, scan_tmp,
                       start);
}

hipError_t launch_bin(hipStream_t st, const DevCells &c, const BinPlan &plan, int nbox, int64_t n,
                      int64_t ncell, const float *pos, const float *h, const float *mass,
                      int *dflags)
{
    hipLaunchKernelGGL(k_bin_local, dim3((unsigned)plan.nblocks), dim3(kBinThreads), 0, st, c.box,
                       c.bin_blocks, pos, h, c.cellid, c.slot, c.binm, dflags, ncell, c.big,
                       c.dx_all);
    hipLaunchKernelGGL(k_bin_columns, dim3(blocks_for(ncell, 256)), dim3(256), 0, st, c.box, nbox,
                       ncell, c.binm, c.cell_start, c.cell_box, c.cell_dx, c.big);
    launch_scan(st, ncell, c.cell_start, c.cell_start, c.scan_tmp, dflags);
    if (n > 0) {
        hipLaunchKernelGGL(k_scatter, dim3(blocks_for(n, 256)), dim3(256), 0, st, c.box, nbox, n,
                           plan.chunk, pos, h, mass, c.cellid, c.slot, c.binm, c.cell_start,
                           c.stage);
    }
    // size classes: at most 64 particles (and empty cells), 65..256, more;
    // when cells hold 128 or more on average the first two are one launch
    // (small cells are then rare, and an empty class still costs a launch
    // over all cells)
    const bool dense = n >= kDenseCells * ncell;
    if (!dense)
        hipLaunchKernelGGL((k_cell_finish_small<64, 32>), dim3((unsigned)ncell), dim3(64), 0, st,
                           c.box, c.cell_box, c.cell_start, c.stage, c.xyzm, c.H, c.orig,
                           c.cell_hmax, c.cell_m, 0);
    hipLaunchKernelGGL((k_cell_finish_small<256, 128>), dim3((unsigned)ncell), dim3(256), 0,
                       st, c.box, c.cell_box, c.cell_start, c.stage, c.xyzm, c.H, c.orig,
                       c.cell_hmax, c.cell_m, dense ? 0 : 65);
    // the cells above 256 particles, listed by the column pass
    hipLaunchKernelGGL(k_cell_finish_large, dim3((unsigned)std::min<int64_t>(ncell, kListWgs)),
                       dim3(kBlock), 0, st, c.box, c.cell_box, c.cell_start, c.stage, c.xyzm,
                       c.H, c.orig, c.cell_hmax, c.cell_m,
                       (const int32_t *)cell_list(c.big, ncell, kListLarge));
    return hipGetLastError();
}

// Chunking of the count matrix: chunks of `chunk` particles (at least one per
// box), grown until the matrix has at most kBinMaxMatrix entries or the
// chunks reach 2^22 particles.
BinPlan plan_binning(std::vector<BoxDesc> &boxes, std::vector<int4> &blocks)
{
    constexpr int64_t kBinMaxMatrix = 32 << 20;
    BinPlan plan;
    auto nblk_of = [](const BoxDesc &B, int ch) { return B.n > 0 ? (B.n + ch - 1) / ch : 1; };
    auto mtot_of = [&](int ch) {
        int64_t t = 0;
        for (const BoxDesc &B : boxes) t += (int64_t)B.g[0] * B.g[1] * B.g[2] * nblk_of(B, ch);
        return t;
    };
    int chunk = 16384;
    while (mtot_of(chunk) > kBinMaxMatrix && chunk < (1 << 22)) chunk *= 2;
    blocks.clear();
    int64_t moff = 0;
    for (int b = 0; b < (int)boxes.size(); ++b) {
        BoxDesc &B = boxes[b];
        B.nblk = nblk_of(B, chunk);
        B.moff = (int)moff;
        for (int j = 0; j < B.nblk; ++j) {
            const int lo = B.part_off + std::min(B.n, j * chunk);
            const int hi = B.part_off + std::min(B.n, (j + 1) * chunk);
            blocks.push_back(make_int4(b, j, lo, hi));
        }
        moff += (int64_t)B.g[0] * B.g[1] * B.g[2] * B.nblk;
    }
    plan.chunk = chunk;
    plan.mtot = moff;
    plan.nblocks = (int64_t)blocks.size();
    return plan;
}

}  // namespace pvl
