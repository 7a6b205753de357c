// Per-cell, per-axis sort (Section 2 of the paper: the particles of each cell
// are projected on the axis joining the cell centres and sorted along it; 13
// axes cover all 26 neighbour directions once the +- symmetry is used).
//
// One workgroup per cell, sized to the cell: cells of at most 64, 256 or 512
// particles take a workgroup of that many threads, one particle per thread;
// larger cells a 256-thread workgroup that loops over its particles and
// handles as many axes per pass as fit the LDS.  For each axis s the key
// of particle r is its cell-relative position projected on d_s / |d_s|.  The
// keys are bucket sorted in LDS: the cell's key range along the axis is cut
// into equal buckets (the bucket index is a monotone function of the key), a
// histogram and its prefix sum place every bucket, and each particle's final
// rank is its bucket's start plus the number of bucket mates with a smaller
// (key, in-cell rank) pair.  Equal keys keep in-cell order, so the result is
// deterministic, and the work is linear in the occupancy unless a bucket is
// crowded.
// Output per axis: the in-cell ranks (uint16) in key order, and the first
// keys of every 16 positions from either end (the tile summaries the sweep's
// bounds read); a key itself is recomputed from the position where needed.
#include "device_util.h"

#include <algorithm>
#include <type_traits>

namespace pvl {

// the large-cell sort's LDS for cells of at most MAXCNT particles: histogram
// (at most MAXCNT / 4 buckets), keys and two lists of 16-bit ranks
constexpr int sort_lds_bytes(int maxcnt) { return 4 * (maxcnt / 4) + 8 * maxcnt; }
constexpr int64_t kSortLargeWgs = 256;   // cells in flight of the large-cell sort

__device__ __forceinline__ int sort_buckets(int cnt)
{
    if (cnt <= 256) return 128;
    int p = next_pow2(cnt);
    return cnt <= 1024 ? p >> 1 : p >> 2;
}

// Bucket of key k on an axis whose cell projection starts at kmin: the range
// split into NB equal parts (scale = NB / range).
__device__ __forceinline__ int key_bucket(float k, float kmin, float scale, int NB)
{
    const int b = (int)((k - kmin) * scale);
    return b < 0 ? 0 : (b >= NB ? NB - 1 : b);
}

// Cells of at most MAXC particles, one particle per thread (blockDim = MAXC),
// all 13 axes at once with the axis loops unrolled so that their LDS traffic
// overlaps.  Each key is quantised, monotonically, to QB bits of its axis'
// range within the cell and packed with the particle's in-cell rank into one
// 32-bit word, unique within the cell: ordering the words orders the keys
// (keys closer than 2^-QB of the range keep in-cell order, a swap far below
// the slack of every bound that reads the sorted lists).  NB equal buckets per
// axis.  The cell order is x order, so the x axis' list is the identity and
// is written without sorting.  The histograms and the bucket-order lists
// of words live in LDS (26 KB for MAXC = NB = 256); a particle's rank is its
// bucket's start plus the bucket mates with a smaller word, one LDS load and
// one compare per mate, the 13 axes' mates a round at a time.  Each particle
// writes its own entries of the sorted lists at its ranks, and the first keys
// of the tiles of 16 positions.  Five waves per SIMD at least (four for the
// 512 class): the register bound keeps the 13 axes' words, bucket places and
// ranks in registers without spilling.
template <int MAXC, int NB, bool LIST>
__global__ void __launch_bounds__(MAXC) __attribute__((amdgpu_waves_per_eu(MAXC > 256 ? 4 : 5)))
k_sort13_small(const BoxDesc *__restrict__ box, const int32_t *__restrict__ cell_box,
               const int32_t *__restrict__ start, const float4 *__restrict__ xyzm,
               const float *__restrict__ Hc, int64_t n, uint16_t *__restrict__ sidx,
               int64_t tslots, float *__restrict__ tiles, int min_cnt,
               const int32_t *__restrict__ list, int list_min)
{
    constexpr int RB = MAXC <= 64 ? 6 : (MAXC <= 256 ? 8 : 9);   // bits of the in-cell rank
    constexpr int QB = 32 - RB < 24 ? 32 - RB : 24;                // bits of the quantised key
    constexpr float QMAX = (float)((1u << QB) - 1u);               // exact in fp32
    __shared__ uint32_t hist[13][NB];
    __shared__ uint32_t bword[13][MAXC];
    __shared__ float2 axr[13];   // per axis: the cell's least key and 1 / key range
    // one cell (blockIdx.x), or LIST: the listed cells, a grid's worth at a time
    // LIST: the list's cells, unless it holds at most list_min of them
    // (then k_sort13_large sorts them, a workgroup per cell and axis)
    const int nitem = LIST ? (list[0] > list_min ? list[0] : 0) : 1;
    for (int item = LIST ? (int)blockIdx.x : 0; item < nitem; item += LIST ? (int)gridDim.x : 1) {
        const int c = LIST ? list[1 + item] : (int)blockIdx.x;
        const int s0 = start[c];
        const int cnt = start[c + 1] - s0;
        if (cnt < min_cnt || cnt > MAXC) continue;
        const BoxDesc &B = box[cell_box[c]];
        for (int t = threadIdx.x; t < 13 * NB; t += blockDim.x) (&hist[0][0])[t] = 0u;
        if (threadIdx.x < 13) {
            // the cell's key range on each axis (the same for every cell of a box)
            float e[3];
            dir_axis((int)threadIdx.x, e);
            const float kmin = fminf(e[0], 0.f) * B.edge[0] + fminf(e[1], 0.f) * B.edge[1] +
                               fminf(e[2], 0.f) * B.edge[2];
            const float kmax = fmaxf(e[0], 0.f) * B.edge[0] + fmaxf(e[1], 0.f) * B.edge[1] +
                               fmaxf(e[2], 0.f) * B.edge[2];
            axr[threadIdx.x] = make_float2(kmin, __builtin_amdgcn_rcpf(kmax - kmin));
        }
        const int r = threadIdx.x;
        const bool on = r < cnt;
        const float4 p = on ? xyzm[s0 + r] : make_float4(0.f, 0.f, 0.f, 0.f);
        const float Hi = on ? Hc[s0 + r] : 0.0f;
        __syncthreads();
        int b[13];
        uint32_t w[13], sl[13];
    #pragma unroll
        for (int g = 0; g < 13; ++g) {
            // the key's place t in [0, 1] across the cell's key range on axis g
            if (g == kTileAxisX) continue;
            const float2 ar = axr[g];
            const float kg = proj_key(p.x, p.y, p.z, g);
            const float t = __builtin_amdgcn_fmed3f((kg - ar.x) * ar.y, 0.0f, 1.0f);
            w[g] = ((uint32_t)(t * QMAX) << RB) | (uint32_t)r;
            const int bb = (int)(t * (float)NB);
            b[g] = bb < NB ? bb : NB - 1;
        }
        if (on) {
    #pragma unroll
            for (int g = 0; g < 13; ++g)
                if (g != kTileAxisX) sl[g] = atomicAdd(&hist[g][b[g]], 1u);
        }
        __syncthreads();
        {
            // exclusive scans of the 13 histograms, one wave per axis at a time,
            // NB / 64 buckets per lane (NB <= 64: one bucket on the first lanes)
            const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
            constexpr int per = NB >= 64 ? NB / 64 : 1;
            for (int g = wave; g < 13; g += (int)(blockDim.x >> 6)) {
                if (g == kTileAxisX) continue;
                uint32_t v[per];
                uint32_t loc = 0;
    #pragma unroll
                for (int q = 0; q < per; ++q) {
                    v[q] = lane * per + q < NB ? hist[g][lane * per + q] : 0u;
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
                    if (lane * per + q < NB) hist[g][lane * per + q] = run;
                    run += v[q];
                }
            }
        }
        __syncthreads();
        const int64_t slot0 = tile_slot(s0, c, 0);
        int q0[13];
        if (on) {
    #pragma unroll
            for (int g = 0; g < 13; ++g) {
                if (g == kTileAxisX) continue;
                q0[g] = (int)hist[g][b[g]];
                bword[g][q0[g] + (int)sl[g]] = w[g];
            }
        }
        __syncthreads();
        if (on) {
            // rank: bucket start + bucket mates with a smaller word.  The 13
            // axes' bucket scans advance together, one mate per axis per
            // round, so each round issues its LDS reads side by side; q0
            // packs the bucket start (low 16 bits) and its size (high 16)
            int rk[13];
            int maxlen = 0;
    #pragma unroll
            for (int g = 0; g < 13; ++g) {
                if (g == kTileAxisX) {
                    rk[g] = r;   // the cell order
                    continue;
                }
                const int q1 = b[g] + 1 < NB ? (int)hist[g][b[g] + 1] : cnt;
                rk[g] = q0[g];
                maxlen = max(maxlen, q1 - q0[g]);
                q0[g] |= (q1 - q0[g]) << 16;
            }
            for (int j = 0; j < maxlen; ++j) {
    #pragma unroll
                for (int g = 0; g < 13; ++g) {
                    if (g == kTileAxisX) continue;
                    // every bucket holds at least this particle, so the clamped
                    // index stays in it; past its end the round counts nothing
                    const int len = q0[g] >> 16;
                    const int q = (q0[g] & 0xffff) + min(j, len - 1);
                    rk[g] += (int)(j < len) & (int)(bword[g][q] < w[g]);
                }
            }
    #pragma unroll
            for (int g = 0; g < 13; ++g) {
                const int rank = rk[g];
                // the cell's list and tile rows on this axis (uniform bases,
                // so that each store adds only the lane's own offset)
                uint16_t *const lg = sidx + (size_t)g * (size_t)n + s0;
                float *const ts_g = tiles + kTileTS(g) * tslots + slot0;
                float *const te_g = tiles + kTileTE(g) * tslots + slot0;
                // (byte offsets as unsigned 32-bit values: a cell's rows are
                // far below 4 GB)
                *reinterpret_cast<uint16_t *>(reinterpret_cast<char *>(lg) + (uint32_t)(2 * rank)) =
                    (uint16_t)r;
                // tile summaries: the first keys of the tiles from either end
                // (the key recomputed as before: same operations, same value)
                const float kg = proj_key(p.x, p.y, p.z, g);
                const int re = cnt - 1 - rank;
                if ((rank & 15) == 0)
                    *reinterpret_cast<float *>(reinterpret_cast<char *>(ts_g) + (uint32_t)(rank >> 2 & ~3)) = kg;
                if ((re & 15) == 0)
                    *reinterpret_cast<float *>(reinterpret_cast<char *>(te_g) + (uint32_t)(re >> 2 & ~3)) = kg;
                if (g == kTileAxisX && ((rank & 15) == 15 || re == 0))
                    tiles[kTileTLX * tslots + slot0 + (rank >> 4)] = kg;
            }
        }
        // largest cut-off of each tile of the cell order (16 consecutive threads)
        float hx = Hi;
    #pragma unroll
        for (int off = 8; off > 0; off >>= 1) hx = fmaxf(hx, __shfl_xor(hx, off, 16));
        if (on && (r & 15) == 0) tiles[kTileBHX * tslots + slot0 + (r >> 4)] = hx;
        if constexpr (LIST) __syncthreads();   // the next cell reuses the LDS
    }
}

// Cells above kSortSmallMax particles (listed by the cell finish): one
// workgroup per (listed cell, axis), so that a large cell's 13 sorts run side
// by side; a grid of at most a few hundred cells by 13 axes loops over the
// list.  The keys, the arrival slots and the bucket-order list of the axis
// live in LDS: 36 KB for the list of cells of at most kSortLargeMax
// particles, 72 KB for the list of larger ones (up to PV_MAX_CELL).
template <int MAXCNT>
__global__ void __launch_bounds__(kBlock) k_sort13_large(const BoxDesc *__restrict__ box,
                                                    const int32_t *__restrict__ cell_box,
                                                    const int32_t *__restrict__ start,
                                                    const float4 *__restrict__ xyzm,
                                                    const float *__restrict__ Hc, int64_t n,
                                                    uint16_t *__restrict__ sidx,
                                                    int64_t tslots,
                                                    float *__restrict__ tiles,
                                                    const int32_t *__restrict__ big,
                                                    const int32_t *__restrict__ mid, int mid_max)
{
    __shared__ __align__(16) unsigned char lds[sort_lds_bytes(MAXCNT)];
    __shared__ float ax_kmin, ax_scale;
    const int s = blockIdx.y;   // the axis of this workgroup
    // the list's cells, then (mid, may be NULL) those of a second list when
    // it holds at most mid_max cells (else that list's whole-cell kernel
    // sorts them: few cells sort sooner a workgroup per cell and axis)
    const int nb1 = big[0];
    const int nb2 = mid && mid[0] <= mid_max ? mid[0] : 0;
    const int nbig = nb1 + nb2;
    for (int item = blockIdx.x; item < nbig; item += gridDim.x) {
        const int c = item < nb1 ? big[1 + item] : mid[1 + item - nb1];
        const int s0 = start[c];
        const int cnt = start[c + 1] - s0;
        const BoxDesc &B = box[cell_box[c]];
        const int NB = sort_buckets(cnt);
        // histogram (NB u32), keys (cnt f32), the arrival-slot list (later
        // reused for the final order) and the bucket-order list (cnt u16
        // each), rows rounded to 16 bytes
        const int keyw = ((cnt * 4 + 15) & ~15) / 4;
        const int u16w = ((cnt * 2 + 15) & ~15) / 2;
        uint32_t *hist = reinterpret_cast<uint32_t *>(lds);
        float *key = reinterpret_cast<float *>(lds + (size_t)NB * 4);
        uint16_t *slot = reinterpret_cast<uint16_t *>(key + keyw);
        uint16_t *border = slot + u16w;
        uint16_t *forder = slot;
        if (threadIdx.x == 0) {
            float e[3];
            dir_axis(s, e);
            const float kmin = fminf(e[0], 0.f) * B.edge[0] + fminf(e[1], 0.f) * B.edge[1] +
                               fminf(e[2], 0.f) * B.edge[2];
            const float kmax = fmaxf(e[0], 0.f) * B.edge[0] + fmaxf(e[1], 0.f) * B.edge[1] +
                               fmaxf(e[2], 0.f) * B.edge[2];
            ax_kmin = kmin;
            ax_scale = (float)NB / (kmax - kmin);
        }
        for (int t = threadIdx.x; t < NB; t += blockDim.x) hist[t] = 0u;
        __syncthreads();
        const float kmin = ax_kmin, scale = ax_scale;
        // the key of every particle; the histogram atomic gives each key its
        // arrival slot in its bucket
        for (int r = threadIdx.x; r < cnt; r += blockDim.x) {
            const float4 p = xyzm[s0 + r];
            const float k = proj_key(p.x, p.y, p.z, s);
            key[r] = k;
            slot[r] = (uint16_t)atomicAdd(&hist[key_bucket(k, kmin, scale, NB)], 1u);
        }
        __syncthreads();
        // exclusive scan of the histogram (first wavefront)
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
        // bucket start + arrival slot: the list of every bucket's members
        for (int r = threadIdx.x; r < cnt; r += blockDim.x)
            border[(int)hist[key_bucket(key[r], kmin, scale, NB)] + slot[r]] = (uint16_t)r;
        __syncthreads();
        // exact rank: bucket start + bucket mates with a smaller (key, rank);
        // the members of bucket b sit at [hist[b], hist[b+1])
        for (int r = threadIdx.x; r < cnt; r += blockDim.x) {
            const float k = key[r];
            const int b = key_bucket(k, kmin, scale, NB);
            const int q0 = (int)hist[b];
            const int q1 = b + 1 < NB ? (int)hist[b + 1] : cnt;
            // four mates at a time (clamped indices, bitwise predicates), so
            // each group's LDS reads are in flight together
            int rank = q0;
            for (int q = q0; q < q1; q += 4) {
                int r2[4];
                float k2[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) r2[u] = border[min(q + u, q1 - 1)];
#pragma unroll
                for (int u = 0; u < 4; ++u) k2[u] = key[r2[u]];
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    rank += (int)(q + u < q1) &
                            ((int)(k2[u] < k) | ((int)(k2[u] == k) & (int)(r2[u] < r)));
            }
            forder[rank] = (uint16_t)r;
        }
        __syncthreads();
        // coalesced output of the sorted list and of the tiles' first keys
        const int64_t slot0 = tile_slot(s0, c, 0);
        const size_t o = (size_t)s * (size_t)n + (size_t)s0;
        for (int q = threadIdx.x; q < cnt; q += blockDim.x) {
            const int r = forder[q];
            const float kq = key[r];
            sidx[o + q] = (uint16_t)r;
            const int re = cnt - 1 - q;
            if ((q & 15) == 0) tiles[kTileTS(s) * tslots + slot0 + (q >> 4)] = kq;
            if ((re & 15) == 0) tiles[kTileTE(s) * tslots + slot0 + (re >> 4)] = kq;
            if (s == kTileAxisX && ((q & 15) == 15 || re == 0))
                tiles[kTileTLX * tslots + slot0 + (q >> 4)] = kq;
        }
        // largest cut-off of each tile of the cell order (once per cell)
        if (s == kTileAxisX) {
            for (int j = threadIdx.x; j * 16 < cnt; j += blockDim.x) {
                float hx = 0.0f;
                for (int q = 16 * j; q < min(16 * j + 16, cnt); ++q) hx = fmaxf(hx, Hc[s0 + q]);
                tiles[kTileBHX * tslots + slot0 + j] = hx;
            }
        }
        __syncthreads();
    }
}

// One launch per size class: the classes of at most 64 and 65..256
// particles over all cells, each skipping the others; the cells of 257..512
// and above 512 from the lists the cell finish made, so that a grid without
// such cells launches only a few workgroups for them.  (Larger
// one-particle-per-thread classes measured slower than the looping kernel:
// their LDS leaves two workgroups per compute unit.)
// Lists of 257..512-particle cells up to this long are sorted a workgroup per
// (cell, axis) with the large cells; longer ones a workgroup per cell.
constexpr int kMidSplit = 64;

hipError_t launch_sort13(hipStream_t st, const DevCells &c, int64_t n, int64_t ncell)
{
    if (ncell == 0 || n == 0) return hipSuccess;
    // with 128 or more particles per cell on average, cells of at most 64 are
    // rare: the 256 class takes them, one launch over all cells fewer (the
    // 257..512 class stays: the looping kernel is slower on such cells)
    const bool dense = n >= kDenseCells * ncell;
    int32_t *lists = c.big;
    if (!dense)
        hipLaunchKernelGGL((k_sort13_small<64, 32, false>), dim3((unsigned)ncell), dim3(64), 0, st,
                           c.box, c.cell_box, c.cell_start, c.xyzm, c.H, n, c.sidx,
                           c.tslots, c.tiles, 1, (const int32_t *)nullptr, 0);
    hipLaunchKernelGGL((k_sort13_small<256, 256, false>), dim3((unsigned)ncell), dim3(256), 0, st,
                       c.box, c.cell_box, c.cell_start, c.xyzm, c.H, n, c.sidx,
                       c.tslots, c.tiles, dense ? 1 : 65, (const int32_t *)nullptr, 0);
    // the cells of 257..512 particles, listed by the cell finish (a long
    // list; a short one goes with the large cells below)
    const int32_t *mid = cell_list(lists, ncell, kListMid);
    const unsigned list_wgs = (unsigned)std::min<int64_t>(ncell, kListWgs);
    hipLaunchKernelGGL((k_sort13_small<512, 256, true>), dim3(list_wgs), dim3(512), 0, st, c.box,
                       c.cell_box, c.cell_start, c.xyzm, c.H, n, c.sidx, c.tslots,
                       c.tiles, 257, mid, kMidSplit);
    // the listed large cells (and a short list of 257..512-particle cells),
    // one workgroup per (cell, axis)
    const unsigned big_wgs = (unsigned)std::min<int64_t>(ncell, kSortLargeWgs);
    hipLaunchKernelGGL(k_sort13_large<kSortLargeMax>, dim3(big_wgs, 13), dim3(kBlock), 0, st,
                       c.box, c.cell_box, c.cell_start, c.xyzm, c.H, n, c.sidx,
                       c.tslots, c.tiles, (const int32_t *)cell_list(lists, ncell, kListBig), mid,
                       kMidSplit);
    hipLaunchKernelGGL(k_sort13_large<PV_MAX_CELL>, dim3(big_wgs, 13), dim3(kBlock), 0, st,
                       c.box, c.cell_box, c.cell_start, c.xyzm, c.H, n, c.sidx,
                       c.tslots, c.tiles, (const int32_t *)cell_list(lists, ncell, kListHuge),
                       (const int32_t *)nullptr, 0);
    return hipGetLastError();
}

}  // namespace pvl
