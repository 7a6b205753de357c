// Tiled pseudo-Verlet density sweep for wave64.
//
// The paper's SIMD strategy (Section 3.1) holds one receiver and streams a
// vector of sources past it; its loop bounds (Section 3.3: first_a and the
// per-receiver last candidate) keep only sources whose projected separation on
// the cell-pair axis is below the receiver's cut-off, and its cache
// (Section 3.2) holds the sources in sorted order.  On a 64-lane wavefront the
// same bounds are applied to 16 x 16 tiles:
//
//   * a row of 16 lanes holds 16 receivers that are consecutive in the
//     interface-first sorted order of the receiver cell, and 16 consecutive
//     sources of the neighbour's sorted list (one per lane, loaded once);
//   * the 16 pairings of the tile are the 16 rotations of the sources across
//     the row (DPP row_ror, folded into the subtractions), so each source is
//     fetched once per 16 pair tests;
//   * a row's task is (neighbour direction, block of 16 receivers); its number
//     of source tiles is the paper's bound taken for the block: the sources up
//     to the largest key + cut-off of its receivers.  Receivers are ordered by
//     that reach (key + H toward a neighbour ahead on the axis, key - H toward
//     one behind) rather than by key, so the 16 bounds of a block are close;
//   * tasks run longest first, four to a wave, so the rows of a wave finish
//     together;
//   * receivers past first_a (none of their candidates can be in range, judged
//     with the cell's largest cut-off) get no task.
//
// The receiver's own cell (which the paper does not treat) uses the same
// tiles on the cell's sorted list along x: a block of 16 receivers only meets
// the source tiles whose keys lie within the block's key range widened by its
// largest cut-off on both sides.  Each wave accumulates its
// rows in registers and adds them, once per task, into its own LDS array;
// the four arrays are summed in a fixed order at the end, so the result does
// not depend on timing.  One workgroup (4 waves) per cell of at most
// kTiledMaxCell receivers; larger cells go through the scalar sweep.
#include "device_util.h"

namespace pvl {

// Per size class MAXC (largest cell handled by one workgroup): task slots and
// receivers (over all 26 directions) that can be ordered by reach in LDS.
template <int MAXC> struct TiledLimits {
    static constexpr int tasks = 27 * (MAXC / 16);
    static constexpr int recv = 6 * MAXC;
    static_assert(recv * 10 <= 4 * MAXC * 16, "set-up arrays alias the accumulators");
};

template <int K>
__device__ __forceinline__ float ror16(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x120 + K, 0xf, 0xf, true));
}

struct TileAcc {
    float rho, wc, dh, cnt;
};

__device__ __forceinline__ void tile_interact(float r2, float mj, float invH, TileAcc &a)
{
    float u = __builtin_amdgcn_sqrtf(r2) * invH;   // v_sqrt_f32, 1 ulp
    float u2 = u * u;
    float v = 1.0f - u;
    float v2 = v * v;
    float wi = fmaf(u2, fmaf(6.0f, u, -6.0f), 1.0f);
    float di = fmaf(u2, fmaf(36.0f, u, -30.0f), 3.0f);
    float wo = 2.0f * v2 * v;
    float dout = v2 * fmaf(-12.0f, u, 6.0f);
    bool in = u < 0.5f;
    float w = in ? wi : wo;
    float d3 = in ? di : dout;
    a.rho = fmaf(mj, w, a.rho);
    a.wc += w;
    a.dh = fmaf(mj, d3, a.dh);
    a.cnt += 1.0f;
}

#define PVL_TILE_STEP(K)                                                  \
    {                                                                     \
        float dx = ror16<K>(sx) - tx;                                     \
        float dy = ror16<K>(sy) - ty;                                     \
        float dz = ror16<K>(sz) - tz;                                     \
        float mj = ror16<K>(sm);                                          \
        float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));                   \
        if (r2 < H2) tile_interact(r2, mj, invH, acc);                    \
    }

// Task word: bits 0-8 source tiles, 9-14 receiver block, 15-19 direction
// (0..25 neighbour, 26 = own cell), 20-28 first source tile.
__device__ __forceinline__ uint32_t pack_task(int dir, int blk, int nt, int t0)
{
    return (uint32_t)nt | ((uint32_t)blk << 9) | ((uint32_t)dir << 15) | ((uint32_t)t0 << 20);
}

// Axis of the own-cell sort: d = (1, 0, 0).
constexpr int kSelfAxis = 4;

__device__ __forceinline__ int nb_offset(int dir, int &dx, int &dy, int &dz)
{
    int o = dir < 13 ? dir : dir + 1;   // skip the centre of the 3x3x3 block
    dx = o / 9 - 1;
    dy = (o / 3) % 3 - 1;
    dz = o % 3 - 1;
    return o;
}

// PLAIN = true gives the plain cell-list comparator on the same tiles: every
// receiver of the cell meets every particle of the 27 cells, in cell order,
// with no sorted lists and no pruning (Listing 1).
template <int MAXC, bool PLAIN>
__global__ void __launch_bounds__(kBlock) k_sweep_tiled(
    const BoxDesc *__restrict__ box, const int32_t *__restrict__ cell_box,
    const int32_t *__restrict__ start, const float4 *__restrict__ xyzm,
    const float *__restrict__ Hc, const uint32_t *__restrict__ cell_hmax,
    const int32_t *__restrict__ orig, const uint16_t *__restrict__ sidx,
    const float *__restrict__ skey, int64_t n, float *rho, float *wcount, float *drho_dh,
    int32_t *ncount, const int *__restrict__ dflags, int min_na, int max_na, int reach_order,
    int task_sort)
{
    constexpr int kTiledMaxRecv = TiledLimits<MAXC>::recv;
    constexpr int kTiledMaxTasks = TiledLimits<MAXC>::tasks;
    // per-wave accumulators; during set-up the same bytes hold the receiver
    // reach values and indices being sorted
    __shared__ float4 acc_lds[4][MAXC];
    __shared__ uint16_t rlist[kTiledMaxRecv];
    __shared__ uint32_t tasks[kTiledMaxTasks];
    __shared__ uint16_t torder[kTiledMaxTasks];
    __shared__ int n_act[27];
    __shared__ int task_off[28];
    __shared__ int recv_off[27];
    float *rv = reinterpret_cast<float *>(&acc_lds[0][0]);               // reach, key order
    float *rvs = rv + kTiledMaxRecv;                                     // reach, sorted
    uint16_t *ria = reinterpret_cast<uint16_t *>(rvs + kTiledMaxRecv);   // receiver, key order

    if (dflags[0]) return;
    const int a = blockIdx.x;
    const int sa = start[a];
    const int na = start[a + 1] - sa;
    if (na <= min_na || na > max_na) return;
    const BoxDesc &B = box[cell_box[a]];
    const CellGeom ga = cell_geom(B, a);
    const float slack = 1.52587890625e-5f * (B.edge[0] + B.edge[1] + B.edge[2]);
    const float hmax_a = __uint_as_float(cell_hmax[a]);
    const int tid = threadIdx.x;

    // receivers of each direction that can have a candidate (first_a)
    if (tid < 26) {
        int dx, dy, dz;
        nb_offset(tid, dx, dy, dz);
        float sx, sy, sz;
        int b = neighbour(B, ga, dx, dy, dz, sx, sy, sz);
        int sb = start[b], nb = start[b + 1] - sb;
        int act = 0;
        if (PLAIN) {
            act = nb > 0 ? na : 0;
        } else if (nb > 0) {
            int sign;
            int s = dir_canon(dx, dy, dz, &sign);
            float e[3];
            dir_axis(s, e);
            float se = fmaf(sx, e[0], fmaf(sy, e[1], sz * e[2]));
            const float *ka = skey + (size_t)s * n + sa;
            const float *kb = skey + (size_t)s * n + sb;
            if (sign > 0) {
                // receivers with key_i + Hmax_a > key_b[0] + se
                float thr = (kb[0] + se) - hmax_a - slack;
                int lo = 0, hi = na;
                while (lo < hi) { int m = (lo + hi) >> 1; if (ka[m] <= thr) lo = m + 1; else hi = m; }
                act = na - lo;
            } else {
                // receivers with key_i - Hmax_a < key_b[nb-1] + se
                float thr = (kb[nb - 1] + se) + hmax_a + slack;
                int lo = 0, hi = na;
                while (lo < hi) { int m = (lo + hi) >> 1; if (ka[m] < thr) lo = m + 1; else hi = m; }
                act = lo;
            }
        }
        n_act[tid] = act;
    }
    if (tid == 26) n_act[26] = na;
    __syncthreads();
    if (tid == 0) {
        int off = 0, roff = 0;
        for (int d = 0; d < 27; ++d) {
            task_off[d] = off;
            off += (n_act[d] + 15) >> 4;
            if (d < 26) {
                recv_off[d] = roff;
                roff += n_act[d];
            }
        }
        task_off[27] = off;
        // reach ordering needs room for every active receiver
        recv_off[26] = (!PLAIN && reach_order && roff <= kTiledMaxRecv) ? roff : -1;
    }
    __syncthreads();
    const int ntask = task_off[27];
    const bool by_reach = recv_off[26] >= 0;
    const int nrecv = by_reach ? recv_off[26] : 0;

    // Order each direction's active receivers by how far past the shared face
    // their cut-off reaches (key + H toward a neighbour ahead, key - H toward
    // one behind), so a block of 16 has nearly equal loop bounds.
    if (by_reach) {
        for (int q = tid; q < nrecv; q += blockDim.x) {
            int dir = 0;
            while (dir < 25 && recv_off[dir + 1] <= q) ++dir;
            int r = q - recv_off[dir];
            int dx, dy, dz, sign;
            nb_offset(dir, dx, dy, dz);
            int s = dir_canon(dx, dy, dz, &sign);
            int qs = sign > 0 ? na - 1 - r : r;
            int ia = sidx[(size_t)s * n + sa + qs];
            float k = skey[(size_t)s * n + sa + qs];
            float H = Hc[sa + ia];
            rv[q] = sign > 0 ? -(k + H) : (k - H);
            ria[q] = (uint16_t)ia;
        }
        __syncthreads();
        for (int q = tid; q < nrecv; q += blockDim.x) {
            int dir = 0;
            while (dir < 25 && recv_off[dir + 1] <= q) ++dir;
            int o = recv_off[dir], r = q - o, m = n_act[dir];
            float v = rv[q];
            int rank = 0;
            for (int k = 0; k < m; ++k) {
                float w = rv[o + k];
                rank += (w < v) || (w == v && k < r);
            }
            rlist[o + rank] = ria[q];
            rvs[o + rank] = v;
        }
        __syncthreads();
    }

    // source tiles of every task: the paper's bound for the block of receivers
    for (int t = tid; t < ntask; t += blockDim.x) {
        int dir = 0;
        while (task_off[dir + 1] <= t) ++dir;
        int blk = t - task_off[dir];
        int nt, t0 = 0;
        if (PLAIN) {
            int nb = na;
            if (dir < 26) {
                int dx, dy, dz;
                nb_offset(dir, dx, dy, dz);
                float sx, sy, sz;
                int b = neighbour(B, ga, dx, dy, dz, sx, sy, sz);
                nb = start[b + 1] - start[b];
            }
            nt = (nb + 15) >> 4;
        } else if (dir == 26) {
            // two-sided window on the x-sorted list: |key_j - key_i| < H_i
            const float *ka = skey + (size_t)kSelfAxis * n + sa;
            const uint16_t *ia = sidx + (size_t)kSelfAxis * n + sa;
            int r0 = blk * 16, r1 = min(r0 + 16, na);
            float hb = 0.0f;
            for (int r = r0; r < r1; ++r) hb = fmaxf(hb, Hc[sa + ia[r]]);
            float lo_k = ka[r0] - hb - slack, hi_k = ka[r1 - 1] + hb + slack;
            int lo = 0, hi = na;
            while (lo < hi) { int m = (lo + hi) >> 1; if (ka[m] <= lo_k) lo = m + 1; else hi = m; }
            int j0 = lo;
            lo = 0; hi = na;
            while (lo < hi) { int m = (lo + hi) >> 1; if (ka[m] < hi_k) lo = m + 1; else hi = m; }
            int j1 = lo;
            t0 = j0 >> 4;
            nt = ((j1 + 15) >> 4) - t0;
        } else {
            int dx, dy, dz;
            nb_offset(dir, dx, dy, dz);
            float sx, sy, sz;
            int b = neighbour(B, ga, dx, dy, dz, sx, sy, sz);
            int sb = start[b], nb = start[b + 1] - sb;
            int sign;
            int s = dir_canon(dx, dy, dz, &sign);
            float e[3];
            dir_axis(s, e);
            float se = fmaf(sx, e[0], fmaf(sy, e[1], sz * e[2]));
            const float *ka = skey + (size_t)s * n + sa;
            const uint16_t *ia = sidx + (size_t)s * n + sa;
            const float *kb = skey + (size_t)s * n + sb;
            int r0 = blk * 16, r1 = min(r0 + 16, n_act[dir]);
            // block reach: the largest key + H (ahead) or smallest key - H (behind)
            float T;
            if (by_reach) {
                float v = rvs[recv_off[dir] + r0];
                T = sign > 0 ? -v : v;
            } else if (sign > 0) {
                T = -INFINITY;
                for (int r = r0; r < r1; ++r) {
                    int q = na - 1 - r;
                    T = fmaxf(T, ka[q] + Hc[sa + ia[q]]);
                }
            } else {
                T = INFINITY;
                for (int r = r0; r < r1; ++r) T = fminf(T, ka[r] - Hc[sa + ia[r]]);
            }
            int nsrc;
            if (sign > 0) {
                T = (T - se) + slack;
                int lo = 0, hi = nb;
                while (lo < hi) { int m = (lo + hi) >> 1; if (kb[m] < T) lo = m + 1; else hi = m; }
                nsrc = lo;
            } else {
                T = (T - se) - slack;
                int lo = 0, hi = nb;
                while (lo < hi) { int m = (lo + hi) >> 1; if (kb[m] <= T) lo = m + 1; else hi = m; }
                nsrc = nb - lo;
            }
            nt = (nsrc + 15) >> 4;
        }
        tasks[t] = pack_task(dir, blk, nt, t0);
    }
    __syncthreads();
    // longest tasks first, so the four rows of a wave carry similar loads
    for (int t = tid; t < ntask; t += blockDim.x) {
        int rank = t;
        if (task_sort) {
            int nt = (int)(tasks[t] & 511u);
            rank = 0;
            for (int q = 0; q < ntask; ++q) {
                int nq = (int)(tasks[q] & 511u);
                rank += (nq > nt) || (nq == nt && q < t);
            }
        }
        torder[rank] = (uint16_t)t;
    }
    for (int t = tid; t < 4 * MAXC; t += blockDim.x)
        (&acc_lds[0][0])[t] = make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();

    // tasks in groups of 4 (one per row); group g runs on wave g % 4
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int row = lane >> 4;
    const int l16 = lane & 15;
    for (int g = wave; g * 4 < ntask; g += 4) {
        const int t = g * 4 + row;
        const bool row_valid = t < ntask;
        uint32_t tw = row_valid ? tasks[torder[t]] : 0u;
        int nt = row_valid ? (int)(tw & 511u) : 0;
        int blk = (int)((tw >> 9) & 63u);
        int dir = (int)((tw >> 15) & 31u);
        const int t0 = (int)(tw >> 20);
        // receiver of this lane and the source list of its row
        int dx = 0, dy = 0, dz = 0, sb = sa, nb = na, sign = 1, s = kSelfAxis;
        float shx = 0.f, shy = 0.f, shz = 0.f;
        if (dir < 26) {
            nb_offset(dir, dx, dy, dz);
            int b = neighbour(B, ga, dx, dy, dz, shx, shy, shz);
            sb = start[b];
            nb = start[b + 1] - sb;
            s = dir_canon(dx, dy, dz, &sign);
        }
        const int r = blk * 16 + l16;
        const bool recv_ok = row_valid && r < n_act[dir];
        int ia = 0;
        if (recv_ok) {
            if (PLAIN) ia = r;
            else if (dir == 26) ia = sidx[(size_t)s * n + sa + r];
            else if (by_reach) ia = rlist[recv_off[dir] + r];
            else if (sign > 0) ia = sidx[(size_t)s * n + sa + (na - 1 - r)];
            else ia = sidx[(size_t)s * n + sa + r];
        }
        float4 pi = recv_ok ? xyzm[sa + ia] : make_float4(0.f, 0.f, 0.f, 0.f);
        float Hi = recv_ok ? Hc[sa + ia] : 0.0f;
        const float H2 = Hi * Hi;
        const float invH = recv_ok ? 1.0f / Hi : 0.0f;
        // pair frame: receiver moved for +1 offsets, source for -1 offsets
        const float tx = dx > 0 ? pi.x - shx : pi.x;
        const float ty = dy > 0 ? pi.y - shy : pi.y;
        const float tz = dz > 0 ? pi.z - shz : pi.z;
        const float ux = dx < 0 ? shx : 0.0f;
        const float uy = dy < 0 ? shy : 0.0f;
        const float uz = dz < 0 ? shz : 0.0f;
        const uint16_t *lb = PLAIN ? nullptr : sidx + (size_t)s * n + sb;

        int ntmax = nt;
        ntmax = max(ntmax, __shfl_xor(ntmax, 16));
        ntmax = max(ntmax, __shfl_xor(ntmax, 32));
        TileAcc acc = {0.f, 0.f, 0.f, 0.f};
        for (int it = 0; it < ntmax; ++it) {
            const int tile = t0 + it;
            const int j = tile * 16 + l16;
            float4 q = make_float4(1e30f, 1e30f, 1e30f, 0.f);
            if (it < nt && j < nb) {
                int p = PLAIN ? j : (int)lb[sign > 0 ? j : nb - 1 - j];
                q = xyzm[sb + p];
                q.x += ux;
                q.y += uy;
                q.z += uz;
            }
            const float sx = q.x, sy = q.y, sz = q.z, sm = q.w;
            if (it < nt) {
                if (!(dir == 26 && tile == blk)) {
                    float dx0 = sx - tx, dy0 = sy - ty, dz0 = sz - tz;
                    float r2 = fmaf(dx0, dx0, fmaf(dy0, dy0, dz0 * dz0));
                    if (r2 < H2) tile_interact(r2, sm, invH, acc);
                }
                PVL_TILE_STEP(1) PVL_TILE_STEP(2) PVL_TILE_STEP(3) PVL_TILE_STEP(4)
                PVL_TILE_STEP(5) PVL_TILE_STEP(6) PVL_TILE_STEP(7) PVL_TILE_STEP(8)
                PVL_TILE_STEP(9) PVL_TILE_STEP(10) PVL_TILE_STEP(11) PVL_TILE_STEP(12)
                PVL_TILE_STEP(13) PVL_TILE_STEP(14) PVL_TILE_STEP(15)
            }
        }
        if (recv_ok) {
            float *dst = reinterpret_cast<float *>(&acc_lds[wave][ia]);
            atomicAdd(dst + 0, acc.rho);
            atomicAdd(dst + 1, acc.wc);
            atomicAdd(dst + 2, acc.dh);
            atomicAdd(dst + 3, acc.cnt);
        }
    }
    __syncthreads();

    for (int i = tid; i < na; i += blockDim.x) {
        float4 s0 = acc_lds[0][i], s1 = acc_lds[1][i], s2 = acc_lds[2][i], s3 = acc_lds[3][i];
        float sr = ((s0.x + s1.x) + s2.x) + s3.x;
        float sw = ((s0.y + s1.y) + s2.y) + s3.y;
        float sd = ((s0.z + s1.z) + s2.z) + s3.z;
        float sc = ((s0.w + s1.w) + s2.w) + s3.w;
        float H = Hc[sa + i];
        float mi = xyzm[sa + i].w;
        float invH = 1.0f / H;
        float norm = (8.0f / kPi) * invH * invH * invH;
        int o = orig[sa + i];
        if (rho) rho[o] = norm * (sr + mi);
        if (wcount) wcount[o] = norm * (sw + 1.0f);
        if (drho_dh) drho_dh[o] = -norm * (kGamma * invH) * (sd + 3.0f * mi);
        if (ncount) ncount[o] = (int32_t)sc;
    }
}

hipError_t launch_sweep_tiled(hipStream_t st, const DevCells &c, int64_t n, int64_t ncell,
                              float *rho, float *wcount, float *drho_dh, int32_t *ncount,
                              const int *dflags, const SweepTuning &tune, bool plain)
{
    if (plain) {
        int tmax = tune.tiled_max < 0 ? 0 : (tune.tiled_max > kTiledMaxCell ? kTiledMaxCell : tune.tiled_max);
        hipLaunchKernelGGL((k_sweep_tiled<256, true>), dim3((unsigned)ncell), dim3(kBlock), 0, st,
                           c.box, c.cell_box, c.cell_start, c.xyzm, c.H, c.cell_hmax, c.orig,
                           c.sidx, c.skey, n, rho, wcount, drho_dh, ncount, dflags, 0,
                           tmax < 256 ? tmax : 256, 0, tune.task_sort);
        if (tmax > 256)
            hipLaunchKernelGGL((k_sweep_tiled<kTiledMaxCell, true>), dim3((unsigned)ncell),
                               dim3(kBlock), 0, st, c.box, c.cell_box, c.cell_start, c.xyzm, c.H,
                               c.cell_hmax, c.orig, c.sidx, c.skey, n, rho, wcount, drho_dh,
                               ncount, dflags, 256, tmax, 0, tune.task_sort);
        return hipGetLastError();
    }
    if (ncell == 0 || n == 0) return hipSuccess;
    int tmax = tune.tiled_max < 0 ? 0 : (tune.tiled_max > kTiledMaxCell ? kTiledMaxCell : tune.tiled_max);
    // two size classes: the common small cells run with half the LDS, hence
    // more workgroups per compute unit
    hipLaunchKernelGGL((k_sweep_tiled<256, false>), dim3((unsigned)ncell), dim3(kBlock), 0, st, c.box,
                       c.cell_box, c.cell_start, c.xyzm, c.H, c.cell_hmax, c.orig, c.sidx, c.skey,
                       n, rho, wcount, drho_dh, ncount, dflags, 0, tmax < 256 ? tmax : 256,
                       tune.reach_order, tune.task_sort);
    if (tmax > 256)
        hipLaunchKernelGGL((k_sweep_tiled<kTiledMaxCell, false>), dim3((unsigned)ncell), dim3(kBlock), 0, st,
                           c.box, c.cell_box, c.cell_start, c.xyzm, c.H, c.cell_hmax, c.orig,
                           c.sidx, c.skey, n, rho, wcount, drho_dh, ncount, dflags, 256, tmax,
                           tune.reach_order, tune.task_sort);
    return hipGetLastError();
}

}  // namespace pvl
