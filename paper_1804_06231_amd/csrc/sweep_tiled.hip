// Tiled pseudo-Verlet density sweep for wave64, fed by a device work queue.
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
//     to the largest key + cut-off of its receivers (optionally the receivers
//     are first ordered by that reach);
//   * receivers past first_a (none of their candidates can be in range, judged
//     with the cell's largest cut-off) get no task;
//   * tasks run longest first, four to a wave, so the rows of a wave finish
//     together.
//
// The receiver's own cell (which the paper does not treat) uses the same tiles
// in cell order, which is x order: a block of 16 receivers meets only the
// source tiles whose x lies within the block's range widened by its largest
// cut-off on both sides.
//
// Work items are (cell, chunk of at most `chunk` receivers, a tuning parameter
// of at most kChunk); a cell's chunks are
// consecutive x-slabs.  For a chunk of a large cell the active receivers of
// every direction are compacted out of the cell's sorted lists in order.
// Persistent workgroups take items from a device queue that lists the chunks
// of large cells first, so uneven occupancy and many boxes of different sizes
// share one launch; the last cells of the queue may run as 2 or 4 items that
// share out the cell's row tasks, whose sums a second kernel adds in part
// order (so the workgroups finish together).  Each wave adds its rows' sums,
// once per task, into its own LDS array; the four arrays are summed in a fixed
// order at the end, so the result does not depend on timing or on which
// workgroup took the item.
//
// The set-up's searches (first_a, the own cell's window, the source tiles of
// a block) count tiles from the first keys of every 16 sorted positions that
// the per-cell sort leaves beside the lists.  Where a cell and its non-empty
// neighbours share one mass the density steps run with unit masses.
//
// Four sweeps share this code (the MODE template argument):
//   * kModeSorted: the density with the pruned bounds above;
//   * kModePlain: the plain cell-list comparator on the same tiles: every
//     receiver meets every particle of the 27 cells, in cell order, with no
//     sorted lists and no pruning (Listing 1);
//   * kModeAdjoint: the gradient of a loss through rho.  A receiver k gathers
//       dL/dx_k = sum_j [G_k m_j W_r(r, H_k) + G_j m_k W_r(r, H_j)] (x_k - x_j) / r
//       dL/dh_k = G_k drho_dh_k
//     (G = dL/drho, W_r = dW/dr), so every output has one writer.  A pair
//     counts when r < max(H_k, H_j): the bounds use max(H_k, largest cut-off
//     of the source cell) in place of H_k, which keeps every pair that the
//     source's own cut-off decides;
//   * kModeLJ: Lennard-Jones forces and energies over the same pairs (the
//     method serves molecular dynamics as well as SPH):
//       F_i = sum_j (24 eps / r^2) [2 (sigma/r)^12 - (sigma/r)^6] (x_i - x_j),
//       E_i = 1/2 sum_j 4 eps [(sigma/r)^12 - (sigma/r)^6]   over r < H_i.
#include "device_util.h"

#include <algorithm>
#include <type_traits>

namespace pvl {

constexpr int kModeSorted = 0;
constexpr int kModePlain = 1;
constexpr int kModeAdjoint = 2;
constexpr int kModeLJ = 3;

constexpr int kChunk = 256;                    // largest receivers per work item
static_assert(kChunk == kTailRecv, "tail slots hold one chunk");
static_assert(kChunk <= 256, "an item's receiver ranks fit a byte");
// Cells per work item that a mode's LDS holds: the plain sweep takes one cell
// per item (its smaller LDS then leaves room for five workgroups per compute
// unit), the others up to kGroupMax.
constexpr int group_cap(int mode) { return mode == kModePlain ? 1 : kGroupMax; }
// task slots per item: 27 directions of at most chunk / 16 blocks per cell,
// plus one partial block per (cell, direction) when several cells share it
constexpr int max_tasks(int G) { return 27 * (kChunk / 16 + (G > 1 ? G : 0)); }
static_assert(kRecvListBytes == 26 * kChunk, "receiver lists hold a chunk per direction");
constexpr int kSelfAxis = 4;                   // d = (1, 0, 0): cell order is x order
constexpr int kReachBuckets = 16;              // reach levels of the receiver ordering
constexpr int kTaskLevels = 16;                // tile-count levels of the task ordering

// Value of lane (l + K) mod 16 of the same 16-lane row (DPP row_ror:K).
template <int K>
__device__ __forceinline__ float ror16(float v)
{
    if constexpr (K == 0)
        return v;
    else
        return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x120 + K, 0xf, 0xf, true));
}

// x clamped to [0, 1] (one instruction: the clamp bit of the producing
// operation)
__device__ __forceinline__ float clamp01(float x) { return __builtin_amdgcn_fmed3f(x, 0.0f, 1.0f); }

struct TileAcc {
    float rho, wc, dh, cnt;
};

struct GradAcc {
    float gx, gy, gz;   // dL/dx_k
    float dh;           // sum over r < H_k of m_j (3 w + u w')
};

__device__ __forceinline__ void tile_interact(float r2, float mj, float invH2, TileAcc &a)
{
    float u2 = r2 * invH2;
    float u = __builtin_amdgcn_sqrtf(u2);   // v_sqrt_f32, 1 ulp
    // inner piece (u < 1/2): w = 1 - 6u^2 + 6u^3, u w' = 18u^3 - 12u^2.
    // The outer piece differs from it by t^3 in w and by -6 u t^2 in u w'
    // with t = 1 - 2u, so with t = min(0, 1 - 2u) (formed as -clamp(2u - 1)
    // to [0, 1], the same for 0 <= u <= 1) one expression covers both:
    // w = 2 (1-u)^3 and u w' = -6 u (1-u)^2 for u >= 1/2.  The sum of
    // m_j (3w + u w') behind drho_dh is 3 (the density sum) + the sum of
    // m_j u w', so only the latter is accumulated.
    float t = -clamp01(fmaf(2.0f, u, -1.0f));
    float t2 = t * t;
    float w = fmaf(t2, t, fmaf(u2, fmaf(6.0f, u, -6.0f), 1.0f));
    float uw = fmaf(-6.0f * u, t2, u2 * fmaf(18.0f, u, -12.0f));
    a.rho = fmaf(mj, w, a.rho);
    a.wc += w;
    a.dh = fmaf(mj, uw, a.dh);
    a.cnt += 1.0f;
}

// Unit-mass sums (the caller scales them by the common mass).  With
// v = 1 - u and s = max(0, 1 - 2u) the spline is w = 2 v^3 - s^3 on both
// pieces (s vanishes for u >= 1/2) and u w' = 6 u (s^2 - v^2), so a pair
// adds to four cubic sums, each term in [0, 1], and the receiver combines
// them once: sum w = 2 sum v^3 - sum s^3, sum u w' = 6 (sum u s^2 -
// sum u v^2).  The s terms are small against the v terms on average (the
// inner piece is an eighth of the volume), so the combination loses little.
struct UnitAcc {
    float v3, s3, uv2, us2, cnt;
};

__device__ __forceinline__ void tile_interact_unit(float r2, float invH2, UnitAcc &a)
{
    float u2 = r2 * invH2;
    float u = __builtin_amdgcn_sqrtf(u2);   // v_sqrt_f32, 1 ulp
    float v = 1.0f - u;
    float s = clamp01(fmaf(-2.0f, u, 1.0f));
    float v2 = v * v;
    float s2 = s * s;
    a.v3 = fmaf(v2, v, a.v3);
    a.s3 = fmaf(s2, s, a.s3);
    a.uv2 = fmaf(u, v2, a.uv2);
    a.us2 = fmaf(u, s2, a.us2);
    a.cnt += 1.0f;
}

// Both terms of the adjoint for a source j within max(H_k, H_j) of receiver
// k (d = x_j - x_k, r2 = |d|^2; in_k: r < H_k, in_j: r < H_j).  A source at
// the receiver's position (r2 = 0, a distinct coincident particle) adds
// 3 w(0) m_j to the drho_dh sum and nothing to the gradient.  Receiver
// constants: 1/H_k, ck = G_k 8 / (pi H_k^4), m_k; source: m_j, 1/H_j,
// cj = G_j 8 / (pi H_j^4).  Accumulates dL/dx_k and sum m_j (3 w + u w')
// over r < H_k.
__device__ __forceinline__ void grad_interact(float dx, float dy, float dz, float r2, float mj,
                                              float invHj, float cj, bool in_j, bool in_k,
                                              float invHk, float ck, float mk, GradAcc &a)
{
    float invr = r2 > 0.0f ? __builtin_amdgcn_rsqf(r2) : 0.0f;   // v_rsq_f32, 1 ulp
    float r = r2 * invr;
    float uk = r * invHk;
    float uj = r * invHj;
    // w' = -12u + 18u^2 (u < 1/2), -6 (1-u)^2 (u >= 1/2): the outer piece is
    // the inner one minus 6 t^2 with t = min(0, 1 - 2u) (for u <= 1; a
    // receiver or source beyond its cut-off gets t = -1 and a zero mass
    // factor); w as in the forward
    float tk = -clamp01(fmaf(2.0f, uk, -1.0f));
    float tj = -clamp01(fmaf(2.0f, uj, -1.0f));
    float tk2 = tk * tk, tj2 = tj * tj;
    float dwk = fmaf(-6.0f, tk2, uk * fmaf(18.0f, uk, -12.0f));
    float wk = fmaf(tk2, tk, fmaf(uk * uk, fmaf(6.0f, uk, -6.0f), 1.0f));
    float dwj = fmaf(-6.0f, tj2, uj * fmaf(18.0f, uj, -12.0f));
    // the receiver's own cut-off decides its term and its drho_dh sum, the
    // source's cut-off the source's term
    const float mjk = in_k ? mj : 0.0f;
    const float cmj = in_j ? cj * mk : 0.0f;
    float coef = fmaf(ck * mjk, dwk, cmj * dwj);
    a.dh = fmaf(mjk, fmaf(uk, dwk, 3.0f * wk), a.dh);
    // (x_k - x_j) / r = -d / r
    float c = -coef * invr;
    a.gx = fmaf(c, dx, a.gx);
    a.gy = fmaf(c, dy, a.gy);
    a.gz = fmaf(c, dz, a.gz);
}

#define PVL_GRAD_STEP(K)                                                  \
    {                                                                     \
        float dx = ror16<K>(sx) - tx;                                     \
        float dy = ror16<K>(sy) - ty;                                     \
        float dz = ror16<K>(sz) - tz;                                     \
        float mj = ror16<K>(sm);                                          \
        float hj2 = ror16<K>(sh2);                                        \
        float ij = ror16<K>(sinv);                                        \
        float cj = ror16<K>(sc);                                          \
        float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));                   \
        /* bitwise, not short-circuit: one lane mask per step */      \
        const bool in_k = r2 < H2, in_j = r2 < hj2;                       \
        if (in_k | in_j)                                                  \
            grad_interact(dx, dy, dz, r2, mj, ij, cj, in_j, in_k, invH, ck, mi, acc); \
    }

// Symmetric pair update in the receiver's own cell (Section 3.3's update of
// both particles of a pair from one distance test).  A tile of sources j
// against the row's receivers k is swept once for the unordered pairs: the
// receiver's sums as in the gathered step, the source's in registers that
// move one lane per step with the source they belong to (lane l holds the
// sums of the source it meets at step K), so that after 16 steps each lane
// holds its own source's sums again.
//
// Density, equal masses: both sides add to the four cubic sums of their own
// cut-off (v = clamp(1 - u), s = clamp(1 - 2u) vanish for u >= 1, so a pair
// beyond one particle's cut-off adds nothing to it) and to its count.
__device__ __forceinline__ void unit_pair_sym(float r2, float invHk, float invHj, bool in_k,
                                              bool in_j, bool src_on, UnitAcc &a, UnitAcc &b)
{
    const float r = __builtin_amdgcn_sqrtf(r2);   // v_sqrt_f32, 1 ulp
    const float uk = r * invHk, uj = r * invHj;
    const float vk = clamp01(1.0f - uk), sk = clamp01(fmaf(-2.0f, uk, 1.0f));
    const float vk2 = vk * vk, sk2 = sk * sk;
    a.v3 = fmaf(vk2, vk, a.v3);
    a.s3 = fmaf(sk2, sk, a.s3);
    a.uv2 = fmaf(uk, vk2, a.uv2);
    a.us2 = fmaf(uk, sk2, a.us2);
    a.cnt += in_k ? 1.0f : 0.0f;
    const float on = src_on ? 1.0f : 0.0f;
    const float vj = on * clamp01(1.0f - uj), sj = on * clamp01(fmaf(-2.0f, uj, 1.0f));
    const float vj2 = vj * vj, sj2 = sj * sj;
    b.v3 = fmaf(vj2, vj, b.v3);
    b.s3 = fmaf(sj2, sj, b.s3);
    b.uv2 = fmaf(uj, vj2, b.uv2);
    b.us2 = fmaf(uj, sj2, b.us2);
    b.cnt += (in_j & src_on) ? 1.0f : 0.0f;
}

// Adjoint: the force term of a pair is antisymmetric (the bracket
// G_k m_j W_r(r, H_k) + G_j m_k W_r(r, H_j) times the unit vector between
// them), so the source gets the receiver's term with the opposite sign; its
// drho_dh sum takes m_k (3 w + u w') of its own cut-off.
__device__ __forceinline__ void grad_pair_sym(float dx, float dy, float dz, float r2, float mj,
                                              float invHj, float cj, bool in_j, bool in_k,
                                              float invHk, float ck, float mk, bool src_on,
                                              GradAcc &a, GradAcc &b)
{
    float invr = r2 > 0.0f ? __builtin_amdgcn_rsqf(r2) : 0.0f;   // v_rsq_f32, 1 ulp
    float r = r2 * invr;
    float uk = r * invHk;
    float uj = r * invHj;
    float tk = -clamp01(fmaf(2.0f, uk, -1.0f));
    float tj = -clamp01(fmaf(2.0f, uj, -1.0f));
    float tk2 = tk * tk, tj2 = tj * tj;
    float dwk = fmaf(-6.0f, tk2, uk * fmaf(18.0f, uk, -12.0f));
    float wk = fmaf(tk2, tk, fmaf(uk * uk, fmaf(6.0f, uk, -6.0f), 1.0f));
    float dwj = fmaf(-6.0f, tj2, uj * fmaf(18.0f, uj, -12.0f));
    float wj = fmaf(tj2, tj, fmaf(uj * uj, fmaf(6.0f, uj, -6.0f), 1.0f));
    const float mjk = in_k ? mj : 0.0f;
    const float cmj = in_j ? cj * mk : 0.0f;
    float coef = fmaf(ck * mjk, dwk, cmj * dwj);
    a.dh = fmaf(mjk, fmaf(uk, dwk, 3.0f * wk), a.dh);
    float c = -coef * invr;
    a.gx = fmaf(c, dx, a.gx);
    a.gy = fmaf(c, dy, a.gy);
    a.gz = fmaf(c, dz, a.gz);
    const float cs = src_on ? -c : 0.0f;
    const float mkj = (in_j & src_on) ? mk : 0.0f;
    b.dh = fmaf(mkj, fmaf(uj, dwj, 3.0f * wj), b.dh);
    b.gx = fmaf(cs, dx, b.gx);
    b.gy = fmaf(cs, dy, b.gy);
    b.gz = fmaf(cs, dz, b.gz);
}

// The source sums one lane on (row_ror:1), so that they stay with the source
// the next step meets.
__device__ __forceinline__ void rotate_sums(UnitAcc &b)
{
    b.v3 = ror16<1>(b.v3);
    b.s3 = ror16<1>(b.s3);
    b.uv2 = ror16<1>(b.uv2);
    b.us2 = ror16<1>(b.us2);
    b.cnt = ror16<1>(b.cnt);
}
__device__ __forceinline__ void rotate_sums(GradAcc &b)
{
    b.gx = ror16<1>(b.gx);
    b.gy = ror16<1>(b.gy);
    b.gz = ror16<1>(b.gz);
    b.dh = ror16<1>(b.dh);
}

// One symmetric step K of a tile (every lane-crossing read before the branch:
// a DPP read from a lane outside the branch gives zero).  On the diagonal tile (the receivers' own
// block) each unordered pair meets twice: steps 1..7 take both sides, step 8
// (lane l with l + 8, and l + 8 with l) the receiver's side only, steps 0
// (the particle itself) and 9..15 nothing.
#define PVL_SYM_STEP_U(K)                                                   \
    {                                                                       \
        const bool rk = (K == 0 || K > 8) ? !on_diag : true;                \
        const bool sk = (K == 0 || K > 7) ? !on_diag : true;                \
        float dx = ror16<K>(sx) - tx;                                       \
        float dy = ror16<K>(sy) - ty;                                       \
        float dz = ror16<K>(sz) - tz;                                       \
        const float hj2 = ror16<K>(sh2), ij = ror16<K>(sinv);               \
        float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));                     \
        const bool in_k = r2 < H2, in_j = r2 < hj2;                         \
        if ((in_k | in_j) & rk)                                             \
            unit_pair_sym(r2, invH, ij, in_k, in_j, sk, uacc, usrc);        \
        rotate_sums(usrc);                                                  \
    }

#define PVL_SYM_STEP_G(K)                                                   \
    {                                                                       \
        const bool rk = (K == 0 || K > 8) ? !on_diag : true;                \
        const bool sk = (K == 0 || K > 7) ? !on_diag : true;                \
        float dx = ror16<K>(sx) - tx;                                       \
        float dy = ror16<K>(sy) - ty;                                       \
        float dz = ror16<K>(sz) - tz;                                       \
        const float mj = ror16<K>(sm), hj2 = ror16<K>(sh2);                 \
        const float ij = ror16<K>(sinv), cj = ror16<K>(sc);                 \
        float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));                     \
        const bool in_k = r2 < H2, in_j = r2 < hj2;                         \
        if ((in_k | in_j) & rk)                                             \
            grad_pair_sym(dx, dy, dz, r2, mj, ij, cj, in_j, in_k, invH, ck, mi, sk, gacc, \
                          gsrc);                                            \
        rotate_sums(gsrc);                                                  \
    }

// Lennard-Jones pair term (d = x_j - x_i, 0 < r2 < H_i^2).
__device__ __forceinline__ void lj_interact(float dx, float dy, float dz, float r2, float sig2,
                                            float eps, TileAcc &a)
{
    float inv = __builtin_amdgcn_rcpf(r2);   // v_rcp_f32, 1 ulp
    float s2 = sig2 * inv;
    float s6 = s2 * s2 * s2;
    float s12 = s6 * s6;
    float c = (24.0f * eps) * inv * fmaf(2.0f, s12, -s6);
    // F_i += c (x_i - x_j) = -c d
    a.rho = fmaf(-c, dx, a.rho);
    a.wc = fmaf(-c, dy, a.wc);
    a.dh = fmaf(-c, dz, a.dh);
    a.cnt = fmaf(2.0f * eps, s12 - s6, a.cnt);
}

#define PVL_LJ_STEP(K)                                                    \
    {                                                                     \
        float dx = ror16<K>(sx) - tx;                                     \
        float dy = ror16<K>(sy) - ty;                                     \
        float dz = ror16<K>(sz) - tz;                                     \
        float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));                   \
        if (r2 < H2 && r2 > 0.0f) lj_interact(dx, dy, dz, r2, sig2, eps, acc); \
    }

#define PVL_TILE_STEP(K)                                                  \
    {                                                                     \
        float dx = ror16<K>(sx) - tx;                                     \
        float dy = ror16<K>(sy) - ty;                                     \
        float dz = ror16<K>(sz) - tz;                                     \
        float mj = ror16<K>(sm);                                          \
        float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));                   \
        if (r2 < H2) tile_interact(r2, mj, invH2, acc);                   \
    }

// The same step when all masses are equal (no source mass, no density sum).
#define PVL_TILE_STEP_U(K)                                                \
    {                                                                     \
        float dx = ror16<K>(sx) - tx;                                     \
        float dy = ror16<K>(sy) - ty;                                     \
        float dz = ror16<K>(sz) - tz;                                     \
        float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));                   \
        if (r2 < H2) tile_interact_unit(r2, invH2, uacc);                 \
    }

// Neighbour count (bits 0-15), sorted list's axis (16-19), direction sign
// (bit 20: -1) and own cell (bit 21) of a (cell, direction) entry.
__device__ __forceinline__ int pack_geo(int nb, int s, int sign, bool own)
{
    return nb | (s << 16) | ((sign < 0) << 20) | ((int)own << 21);
}
static_assert(PV_MAX_CELL < 65536, "neighbour counts fit 16 bits");

// Task word: bits 0-9 source tiles, 10-14 receiver block, 15-22 the item's
// cell and direction (27 g + d: d 0..25 neighbour, 26 = own cell), 23-31
// first source tile.  A cell has at most PV_MAX_CELL / 16 tiles.
static_assert(PV_MAX_CELL / 16 <= 512, "tile counts and first tiles fit the task word");
__device__ __forceinline__ uint32_t pack_task(int gd, int blk, int nt, int t0)
{
    return (uint32_t)nt | ((uint32_t)blk << 10) | ((uint32_t)gd << 15) | ((uint32_t)t0 << 23);
}
__device__ __forceinline__ int task_tiles(uint32_t tw) { return (int)(tw & 1023u); }

__device__ __forceinline__ void nb_offset(int dir, int &dx, int &dy, int &dz)
{
    int o = dir < 13 ? dir : dir + 1;   // skip the centre of the 3x3x3 block
    dx = o / 9 - 1;
    dy = (o / 3) % 3 - 1;
    dz = o % 3 - 1;
}

// Length of the prefix of the sorted array a[0, len) (len >= 1) on which
// v OP x holds (OP 0: <, 1: <=, 2: >; the predicate is true on a prefix).
// Up to 16 entries are loaded at once and counted; longer arrays are
// bisected.
template <int OP>
__device__ __forceinline__ int prefix_count(const float *__restrict__ a, int len, float x)
{
    auto pred = [x](float v) { return OP == 0 ? v < x : (OP == 1 ? v <= x : v > x); };
    if (len <= 16) {
        float v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = a[min(u, len - 1)];
        int c = 0;
#pragma unroll
        for (int u = 0; u < 16; ++u) c += (u < len && pred(v[u])) ? 1 : 0;
        return c;
    }
    int lo = 0, hi = len;
    while (lo < hi) {
        const int m = (lo + hi) >> 1;
        if (pred(a[m])) lo = m + 1; else hi = m;
    }
    return lo;
}

struct SweepArgs {
    const BoxDesc *box;
    const int32_t *cell_box;
    const int32_t *start;
    const float4 *xyzm;
    const float *Hc;
    const uint32_t *cell_hmax;
    const int32_t *orig;
    const uint16_t *sidx;
    // this launch's receiver lists, kRecvListBytes per workgroup: per
    // direction (compacted or reach-ordered), in-cell ranks less the item's
    // first rank r_lo, below the chunk size, so one byte each
    uint8_t *rlist;
    int64_t n;
    float *rho, *wcount, *drho_dh;
    int32_t *ncount;
    const float *gcell;          // adjoint: upstream gradient in cell order
    float *grad_pos, *grad_h;    // adjoint outputs (input order)
    float lj_eps, lj_sigma2;     // Lennard-Jones parameters
    float *force, *energy;       // Lennard-Jones outputs (input order)
    int *dflags;
    const float *cell_m;         // common mass per cell (NaN: mixed, +inf: empty)
    const float *tiles;          // tile summaries of the sorted lists (see DevCells)
    int64_t tslots;
    const float *cell_dx;        // accumulated displacement bound per cell (pv_drift)
    const uint32_t *dx_all;      // its largest value (fp32 bits)
    const int2 *items;   // queue: [0, nbig) large-cell chunks, [cap - nsmall, cap) cells
    const int *qcount;   // [0] nbig, [1] nsmall
    int *head;           // items taken after the first static round
    // XCD ranges: heads of the large-cell chunks [0], of the tail items [1]
    // and of the kXcds ranges of the single-chunk items [2 + r]
    int *xq;
    int xcd_ranges;
    int cap;
    int tail_cells;      // single-chunk cells among the last tail_cells cells ...
    int tail_parts;      // ... run last, as this many items each (1: no split)
    int tail_split;      // 0: the parts share the task groups; 1: the receivers
    float4 *partial;     // sums of the split items: [tail cell][part][receiver]
    int reach_order;
    int task_sort;
    int chunk;           // receivers per work item: a multiple of 16 in [kChunkMin, kChunk]
    unsigned long long *slots;   // census: pair slots executed (NULL: not counted)
};

template <int G>
struct SweepLds {
    float4 acc[4][kChunk];       // per-wave receiver sums; aliased during set-up
    uint32_t tasks[max_tasks(G)];
    // the task order (0xffff: a gap that keeps the symmetric own-cell tasks
    // in groups of their own); also each task's (cell, direction) (bytes)
    // until ordered
    uint16_t torder[max_tasks(G) + 4];
    // per (cell g of the item, direction d): entry 27 g + d (26 g + d for the
    // neighbour directions alone)
    int n_act[27 * G];
    int act_cell[26 * G];
    int task_off[27 * G + 1];
    int recv_off[26 * G];
    // per (cell g, direction d), entry 27 g + d (d = 26: the own cell), as
    // the set-up finds them: the pair frame's shifts (geo_r: the receiver's,
    // for +1 offsets; geo_u: the source's, for -1 offsets; one of the two is
    // zero on each axis and their sum is the neighbour's origin less the
    // cell's), the neighbour's first slot (geo_r.w) and cell (geo_u.w, both
    // as integer bits), and its particle count with the sorted list's axis
    // and direction sign (nb_pk, see pack_geo)
    float4 geo_r[27 * G], geo_u[27 * G];
    int nb_pk[27 * G];
    // per cell of the item: first particle, count, largest cut-off,
    // displacement bound
    int gsa[G], gna[G];
    float ghmax[G], gdx[G];
    int mbad[4];         // per wave: a mass differs from the first cell's
    int item;
    int qphase, qstep;   // thread 0's place in the order of the XCD ranges
    int ntask_eff;       // entries of the task order, gaps included
};

// Outputs of receiver p (cell order) from its sums over all sources: the
// density with its self term and normalisation, the adjoint's gradients or
// the Lennard-Jones force and energy, written at the particle's input index.
template <int MODE>
__device__ __forceinline__ void finalize_receiver(const SweepArgs &A, int p, float sr, float sw,
                                                  float sd, float sc)
{
    const float H = A.Hc[p];
    const float mi = A.xyzm[p].w;
    const float invH = 1.0f / H;
    const float norm = (8.0f / kPi) * invH * invH * invH;
    const int o = A.orig[p];
    if constexpr (MODE == kModeAdjoint) {
        // (sr, sw, sd) is dL/dx; sc is the sum behind drho_dh
        if (A.grad_pos) {
            A.grad_pos[3 * (int64_t)o + 0] = sr;
            A.grad_pos[3 * (int64_t)o + 1] = sw;
            A.grad_pos[3 * (int64_t)o + 2] = sd;
        }
        if (A.grad_h) A.grad_h[o] = A.gcell[p] * (-norm * (kGamma * invH) * (sc + 3.0f * mi));
    } else if constexpr (MODE == kModeLJ) {
        // (sr, sw, sd) is the force, sc the energy
        if (A.force) {
            A.force[3 * (int64_t)o + 0] = sr;
            A.force[3 * (int64_t)o + 1] = sw;
            A.force[3 * (int64_t)o + 2] = sd;
        }
        if (A.energy) A.energy[o] = sc;
    } else {
        if (A.rho) A.rho[o] = norm * (sr + mi);                          // self: w(0) = 1
        if (A.wcount) A.wcount[o] = norm * (sw + 1.0f);
        // sum of m_j (3w + u w') over the neighbours and the self term (3 m_i)
        if (A.drho_dh) A.drho_dh[o] = -norm * (kGamma * invH) * fmaf(3.0f, sr + mi, sd);
        if (A.ncount) A.ncount[o] = (int32_t)sc;
    }
}

// Exclusive prefix sums over entries k < m (m <= 256) on one wavefront, entry
// k in lane k % 64 of column k / 64: emit(k, offset, value(k)) for every
// entry; returns the total (wavefront-uniform).
template <class V, class E>
__device__ __forceinline__ int wave_scan(int m, int lane, V value, E emit)
{
    int run = 0;   // sum of the earlier columns
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        if (u * 64 >= m) break;
        const int k = u * 64 + lane;
        const int c = k < m ? value(k) : 0;
        int inc = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(inc, o);
            if (lane >= o) inc += v;
        }
        if (k < m) emit(k, run + inc - c, c);
        run += __shfl(inc, 63);
    }
    return run;
}

// One work item.  chunk >= 0: receivers [chunk * csize, ...) of cell a (csize
// a multiple of 16: A.chunk, or a tail cell's share of its receivers); an
// item split into nparts > 1 parts (tail slot `slot`) runs every nparts-th
// group of tasks and leaves its sums in A.partial for k_tail_combine.
// chunk < 0: the -chunk consecutive cells a, a + 1, ... of one row of cells
// along z, each swept whole (small cells whose particles fit one chunk
// together).  The item's receivers are numbered in cell order from the
// first receiver's position.
template <int MODE, bool SYM>
__device__ void sweep_item(const SweepArgs &A, SweepLds<group_cap(MODE)> &L, int a, int chunk,
                           int part, int nparts, int slot, int csize)
{
    constexpr bool PLAIN = MODE == kModePlain;
    constexpr bool ADJ = MODE == kModeAdjoint;
    constexpr bool LJ = MODE == kModeLJ;
    static_assert(kBlock == 256, "four wavefronts");
    const int64_t n = A.n;
    const int ncg = chunk < 0 ? -chunk : 1;   // cells of the item (the queue keeps
                                              // it within group_cap(MODE))
    if (chunk < 0) chunk = 0;
    const int sa0 = A.start[a];
    const int na0 = A.start[a + 1] - sa0;
    const int r_lo = chunk * csize;
    // the item's receivers: positions [base, base + nrt) of the cell order
    const int base = sa0 + r_lo;
    const int nrt = ncg > 1 ? A.start[a + ncg] - sa0 : min(r_lo + csize, na0) - r_lo;
    const bool whole = na0 <= csize;   // grouped cells are single-chunk
    const BoxDesc &B = A.box[A.cell_box[a]];
    const CellGeom ga = cell_geom(B, a);
    const float slack = 1.52587890625e-5f * (B.edge[0] + B.edge[1] + B.edge[2]);
    // the thread index, opaque to the compiler: values derived from it are
    // then formed per item, not kept in registers across the item loop
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int wave = tid >> 6, lane = tid & 63;
    const uint16_t *sidx = A.sidx;
    const int64_t ts = A.tslots;
    const float *tiles = A.tiles;
    // cell g of the item: g steps along z in the first cell's row
    auto geom_of = [&](int g) {
        CellGeom c = ga;
        c.cz += g;
        c.oz = (float)c.cz * B.edge[2];
        return c;
    };

    // per cell of the item: first particle, count, largest cut-off and
    // displacement bound
    if (tid < ncg) {
        const int c = a + tid;
        const int s0 = A.start[c];
        const float hm = __uint_as_float(A.cell_hmax[c]);
        const float dxc = A.cell_dx[c];
        L.gsa[tid] = s0;
        L.gna[tid] = A.start[c + 1] - s0;
        L.geo_r[27 * tid + 26] = make_float4(0.0f, 0.0f, 0.0f, __int_as_float(s0));
        L.geo_u[27 * tid + 26] = make_float4(0.0f, 0.0f, 0.0f, __int_as_float(c));
        L.nb_pk[27 * tid + 26] = pack_geo(A.start[c + 1] - s0, kSelfAxis, 1, true);
        L.ghmax[tid] = hm;
        L.gdx[tid] = dxc;
        // Section 2: sorted lists stay usable after the particles move, with
        // every projected bound widened by the displacements; the cells stay
        // usable while H + dx_i + dx_j fits the edge
        const float dx_all = __uint_as_float(*A.dx_all);
        const float emin = fminf(B.edge[0], fminf(B.edge[1], B.edge[2]));
        if (dx_all > 0.0f && hm + dxc + dx_all > emin) atomicOr(A.dflags, kErrDrift);
    }

    // receivers of each (cell, direction) that can have a candidate (first_a),
    // whole cell, rounded up to whole tiles of the interface-first order (the
    // extra receivers have no candidate either; they only fill their row)
    float mb = INFINITY;   // the neighbour's common mass (see DevCells::cell_m)
    if (tid < 26 * ncg) {
        const int g = tid / 26, d = tid - 26 * g;
        const int c = a + g;
        const int sa = A.start[c], na = A.start[c + 1] - sa;
        const float hmax_a = __uint_as_float(A.cell_hmax[c]);
        const float dx_a = A.cell_dx[c];
        int dx, dy, dz;
        nb_offset(d, dx, dy, dz);
        float sx, sy, sz;
        int b = neighbour(B, geom_of(g), dx, dy, dz, sx, sy, sz);
        int sb = A.start[b], nb = A.start[b + 1] - sb;
        int sign;
        const int s = dir_canon(dx, dy, dz, &sign);
        L.geo_r[tid + g] = make_float4(dx > 0 ? sx : 0.0f, dy > 0 ? sy : 0.0f, dz > 0 ? sz : 0.0f,
                                       __int_as_float(sb));
        L.geo_u[tid + g] = make_float4(dx < 0 ? sx : 0.0f, dy < 0 ? sy : 0.0f, dz < 0 ? sz : 0.0f,
                                       __int_as_float(b));
        L.nb_pk[tid + g] = pack_geo(nb, s, sign, false);
        if (!ADJ && !LJ) mb = A.cell_m[b];
        int act = 0;
        if (PLAIN) {
            act = nb > 0 ? na : 0;
        } else if (nb > 0 && na > 0) {
            float e[3];
            dir_axis(s, e);
            float se = fmaf(sx, e[0], fmaf(sy, e[1], sz * e[2]));
            const int64_t slot_a = tile_slot(sa, c, 0);
            const int64_t slot_b = tile_slot(sb, b, 0);
            const int ntile_a = (na + 15) >> 4;
            // the adjoint also keeps pairs decided by the source's cut-off
            const float reach = (ADJ ? fmaxf(hmax_a, __uint_as_float(A.cell_hmax[b])) : hmax_a) +
                                (dx_a + A.cell_dx[b]);
            int ntl;
            if (sign > 0) {
                // receivers with key_i + reach > key_b[0] + se: a suffix, whose
                // tiles counted from the end have their first key above thr
                const float thr = (tiles[kTileTS(s) * ts + slot_b] + se) - reach - slack;
                ntl = prefix_count<2>(tiles + kTileTE(s) * ts + slot_a, ntile_a, thr);
            } else {
                // receivers with key_i - reach < key_b[nb-1] + se: a prefix
                const float thr = (tiles[kTileTE(s) * ts + slot_b] + se) + reach + slack;
                ntl = prefix_count<0>(tiles + kTileTS(s) * ts + slot_a, ntile_a, thr);
            }
            act = min(16 * ntl, na);
        }
        L.act_cell[tid] = act;
    }
    // equal masses: when the item's cells and every non-empty neighbour share
    // one mass m, the density sums are m times the unit-mass sums, and the
    // steps need neither the sources' masses nor a separate density sum
    const float ma = (!ADJ && !LJ) ? A.cell_m[a] : 0.0f;
    if constexpr (!ADJ && !LJ) {
        bool ok = mb == ma || mb == INFINITY;
        if (tid >= 26 * ncg && tid < 27 * ncg) {
            const float mc = A.cell_m[a + (tid - 26 * ncg)];
            ok = mc == ma || mc == INFINITY;
        }
        const uint64_t bad = __ballot(!ok);
        if (lane == 0) L.mbad[wave] = bad != 0;
    }
    __syncthreads();
    float mass = __builtin_nanf("");
    if constexpr (!ADJ && !LJ) {
        if ((L.mbad[0] | L.mbad[1] | L.mbad[2] | L.mbad[3]) == 0 && ma == ma && ma != INFINITY)
            mass = ma;
    }
    // own cells by the symmetric update: items of whole cells, in the
    // adjoint and in the equal-mass density
    const bool symitem = SYM && whole && (ADJ || (!LJ && !PLAIN && mass == mass));

    // active receivers of this item, per (cell, direction): n_act[27 g + d]
    uint8_t *const rlist = A.rlist + (size_t)blockIdx.x * kRecvListBytes;
    bool listed = false;   // receivers taken from the lists
    if (PLAIN) {
        if (tid < 26 * ncg) {
            const int g = tid / 26;
            L.n_act[tid + g] = L.act_cell[tid] > 0 ? (ncg > 1 ? L.gna[g] : nrt) : 0;
        }
    } else if (whole) {
        if (tid < 26 * ncg) L.n_act[tid + tid / 26] = L.act_cell[tid];
        listed = !ADJ && A.reach_order;
        if (listed) {
            // each (cell, direction) list at the sum of the ones before it
            if (wave == 0)
                wave_scan(26 * ncg, lane, [&](int k) { return L.act_cell[k]; },
                          [&](int k, int off, int) { L.recv_off[k] = off; });
            __syncthreads();
            // Receivers of a face direction are ordered by how far past the
            // shared face their cut-off reaches (key + H toward a neighbour ahead
            // on the axis, H - key toward one behind), quantised to
            // kReachBuckets levels and interface-first within a level, so that
            // the receivers of a block of 16 have similar loop bounds.  A
            // stable counting sort made of wavefront ballots (one wavefront per
            // direction, no atomics: the order is deterministic).  Edge and
            // corner directions keep the interface-first key order.
            for (int gd = wave; gd < 26 * ncg; gd += (int)(blockDim.x >> 6)) {
                const int g = gd / 26, d = gd - 26 * g;
                const int sa = L.gsa[g], na = L.gna[g];
                const float hmax_a = L.ghmax[g];
                const int act = L.act_cell[gd];
                int dx, dy, dz, sign;
                nb_offset(d, dx, dy, dz);
                const int s = dir_canon(dx, dy, dz, &sign);
                const uint16_t *il = sidx + (size_t)s * n + sa;
                uint8_t *out = rlist + L.recv_off[gd];
                const bool face = (dx != 0) + (dy != 0) + (dz != 0) == 1;
                if (!face) {
                    for (int q = lane; q < act; q += 64)
                        out[q] = (uint8_t)il[sign > 0 ? na - 1 - q : q];
                    continue;
                }
                if (act == 0) continue;
                // the cell's smallest and largest keys on the axis (its tiles'
                // first keys from either end)
                const int64_t slot_a = tile_slot(sa, a + g, 0);
                const float kmin = tiles[kTileTS(s) * ts + slot_a];
                const float kmax = tiles[kTileTE(s) * ts + slot_a];
                const float lo = sign > 0 ? kmin : -kmax;
                const float hi = (sign > 0 ? kmax : -kmin) + hmax_a;
                const float scale = (float)kReachBuckets / fmaxf(hi - lo, 1e-30f);
                constexpr int R = kChunk / 64;
                int bk[R], pos[R];
                uint16_t iav[R];
                const int nc = (act + 63) >> 6;
#pragma unroll
                for (int c = 0; c < R; ++c) {
                    const int q = c * 64 + lane;
                    bk[c] = kReachBuckets;   // no entry
                    iav[c] = 0;
                    pos[c] = 0;
                    if (c < nc && q < act) {
                        const int qs = sign > 0 ? na - 1 - q : q;
                        const int ia = il[qs];
                        const float4 pq = A.xyzm[sa + ia];
                        const float k = proj_key(pq.x, pq.y, pq.z, s);
                        const float H = A.Hc[sa + ia];
                        const float T = sign > 0 ? k + H : H - k;
                        const int b = (int)((hi - T) * scale);
                        bk[c] = b < 0 ? 0 : (b >= kReachBuckets ? kReachBuckets - 1 : b);
                        iav[c] = (uint16_t)ia;
                    }
                }
                int run = 0;   // entries placed so far (wavefront-uniform)
                for (int b = 0; b < kReachBuckets; ++b) {
#pragma unroll
                    for (int c = 0; c < R; ++c) {
                        if (c >= nc) break;
                        const bool mine = bk[c] == b;
                        const uint64_t m = __ballot(mine);
                        if (mine)
                            pos[c] = run + (int)__builtin_amdgcn_mbcnt_hi(
                                               (uint32_t)(m >> 32),
                                               __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                        run += __popcll(m);
                    }
                }
#pragma unroll
                for (int c = 0; c < R; ++c)
                    if (c < nc && bk[c] < kReachBuckets) out[pos[c]] = (uint8_t)iav[c];
            }
        }
    } else {
        // one cell larger than a chunk: compact, in interface-first order, the
        // active receivers that belong to this chunk (in-cell rank in [r_lo,
        // r_lo + nrt)): one wavefront per direction, ballots over the
        // direction's list (four loads in flight per lane), into the
        // direction's own slot of chunk entries (a direction keeps at most the
        // chunk's receivers), so the directions need no barrier or prefix
        // between them
        listed = true;
        const int r_hi = r_lo + nrt;
        for (int d = wave; d < 26; d += (int)(blockDim.x >> 6)) {
            const int act = L.act_cell[d];
            int dx, dy, dz, sign;
            nb_offset(d, dx, dy, dz);
            const int s = dir_canon(dx, dy, dz, &sign);
            const uint16_t *il = sidx + (size_t)s * n + sa0;
            uint8_t *out = rlist + d * csize;
            int cnt = 0;   // wavefront-uniform
            for (int q0 = 0; q0 < act; q0 += 4 * 64) {
                int iv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int q = q0 + u * 64 + lane;
                    iv[u] = q < act ? (int)il[sign > 0 ? na0 - 1 - q : q] : -1;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const bool keep = iv[u] >= r_lo && iv[u] < r_hi;
                    const uint64_t m = __ballot(keep);
                    if (keep)
                        out[cnt + (int)__builtin_amdgcn_mbcnt_hi(
                                      (uint32_t)(m >> 32),
                                      __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))] =
                            (uint8_t)(iv[u] - r_lo);
                    cnt += __popcll(m);
                }
            }
            if (lane == 0) {
                L.n_act[d] = cnt;
                L.recv_off[d] = d * csize;
            }
        }
    }
    if (tid < ncg) L.n_act[27 * tid + 26] = ncg > 1 ? L.gna[tid] : nrt;
    uint8_t *tdir = reinterpret_cast<uint8_t *>(L.torder);
    __syncthreads();
    // tasks (blocks of 16 receivers) per (cell, direction), their offsets by a
    // scan on the first wavefront, and the (cell, direction) of every task
    const int ne = 27 * ncg;
    if (wave == 0) {
        const int tot = wave_scan(
            ne, lane, [&](int k) { return (L.n_act[k] + 15) >> 4; },
            [&](int k, int off, int c) {
                L.task_off[k] = off;
                for (int t = off; t < off + c; ++t) tdir[t] = (uint8_t)k;
            });
        if (lane == 0) L.task_off[ne] = tot;
    }
    __syncthreads();
    const int ntask = L.task_off[ne];

    // source tiles of every task: the paper's bound for the block of receivers
    for (int t = tid; t < ntask; t += blockDim.x) {
        const int gd = tdir[t];
        const int g = gd / 27, dir = gd - 27 * g;
        const int blk = t - L.task_off[gd];
        const int c = a + g;
        const int sa = L.gsa[g], na = L.gna[g];
        const int64_t slot_a = tile_slot(sa, c, 0);
        const int ntile_a = (na + 15) >> 4;
        const float hmax_a = L.ghmax[g], dx_a = L.gdx[g];
        int nt, t0 = 0;
        if (PLAIN) {
            const int nb = L.nb_pk[gd] & 0xffff;
            nt = (nb + 15) >> 4;
        } else if (dir == 26) {
            // two-sided window in x over the whole cell: |x_j - x_i| < H_i.
            // The block is tile jb of the cell order (chunks are whole tiles);
            // the source tiles are those whose last x is above the block's
            // first x - reach and whose first x is below its last x + reach.
            const int jb = (r_lo >> 4) + blk;
            const float *first_x = tiles + kTileTS(kSelfAxis) * ts + slot_a;
            const float *last_x = tiles + kTileTLX * ts + slot_a;
            if (symitem) {
                // symmetric update: each unordered pair once, from the block
                // of the one with the smaller x; a pair counts for either
                // particle's cut-off, at most the cell's largest
                const float hi_k = last_x[jb] + hmax_a + slack + 2.0f * dx_a;
                t0 = jb;
                nt = prefix_count<0>(first_x, ntile_a, hi_k) - jb;
            } else {
                // the adjoint's pairs reach max(H_i, H_j) <= the cell's largest cut-off
                const float hb = ADJ ? hmax_a : tiles[kTileBHX * ts + slot_a + jb];
                const float lo_k = first_x[jb] - hb - slack - 2.0f * dx_a;
                const float hi_k = last_x[jb] + hb + slack + 2.0f * dx_a;
                t0 = prefix_count<1>(last_x, ntile_a, lo_k);
                nt = prefix_count<0>(first_x, ntile_a, hi_k) - t0;
            }
        } else {
            const float4 gr = L.geo_r[gd], gu = L.geo_u[gd];
            const int pk = L.nb_pk[gd];
            const int sb = __float_as_int(gr.w), b = __float_as_int(gu.w), nb = pk & 0xffff;
            const int s = (pk >> 16) & 15, sign = (pk >> 20) & 1 ? -1 : 1;
            // the neighbour's origin less the cell's (one term is zero)
            const float sx = gr.x + gu.x, sy = gr.y + gu.y, sz = gr.z + gu.z;
            float e[3];
            dir_axis(s, e);
            float se = fmaf(sx, e[0], fmaf(sy, e[1], sz * e[2]));
            const uint16_t *il = sidx + (size_t)s * n + sa;
            const int r0 = blk * 16, r1 = min(r0 + 16, L.n_act[gd]);
            const float hmax_b = __uint_as_float(A.cell_hmax[b]);
            const float mg = dx_a + A.cell_dx[b];
            // block reach: the largest key + H (ahead) or smallest key - H
            // (behind), keys projected from the receivers' positions.  The
            // block's 16 ranks are loaded at once (clamped indices), then
            // their positions and cut-offs: two round trips to memory.
            int iv[16];
            if (listed) {
                const uint8_t *rl = rlist + L.recv_off[26 * g + dir];
#pragma unroll
                for (int u = 0; u < 16; ++u) iv[u] = r_lo + rl[min(r0 + u, r1 - 1)];
            } else {
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int r = min(r0 + u, r1 - 1);
                    iv[u] = il[sign > 0 ? na - 1 - r : r];
                }
            }
            float T = sign > 0 ? -INFINITY : INFINITY;
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const float4 p = A.xyzm[sa + iv[u]];
                const float hv = A.Hc[sa + iv[u]];
                const float kv = proj_key(p.x, p.y, p.z, s);
                const float H = ADJ ? fmaxf(hv, hmax_b) : hv;
                T = sign > 0 ? fmaxf(T, kv + H) : fminf(T, kv - H);
            }
            // source tiles with a key below the reach (ahead), or above it
            // (behind, counted from the end): from the tiles' first keys
            const int64_t slot_b = tile_slot(sb, b, 0);
            const int ntile_b = (nb + 15) >> 4;
            if (sign > 0) {
                T = (T - se) + slack + mg;
                nt = prefix_count<0>(tiles + kTileTS(s) * ts + slot_b, ntile_b, T);
            } else {
                T = (T - se) - slack - mg;
                nt = prefix_count<2>(tiles + kTileTE(s) * ts + slot_b, ntile_b, T);
            }
        }
        L.tasks[t] = pack_task(gd, blk, nt, t0);
    }
    __syncthreads();
    // longest tasks first, so the four rows of a wave carry similar loads: a
    // stable counting sort on the tile count (kTaskLevels levels, longer
    // counts share the top one) made of ballots on one wavefront; ties keep
    // task order, so the order is deterministic
    // With symmetric own cells their tasks take the top half of the levels
    // (by half their tile count) and the others the bottom half, and the
    // order leaves a gap of up to 3 entries after the last symmetric task, so
    // that no group of four mixes the two kinds.
    auto level_of = [&](int t) {
        const uint32_t tw = L.tasks[t];
        const int nt = task_tiles(tw);
        if (!symitem) return min(nt, kTaskLevels - 1);
        const bool own = (int)((tw >> 15) & 255u) % 27 == 26;
        return own ? kTaskLevels / 2 + min(nt >> 1, kTaskLevels / 2 - 1)
                   : min(nt, kTaskLevels / 2 - 1);
    };
    if (!A.task_sort && !symitem) {
        for (int t = tid; t < ntask; t += blockDim.x) L.torder[t] = (uint16_t)t;
        if (tid == 0) L.ntask_eff = ntask;
    } else if (wave == 0) {
        int below[kTaskLevels];   // tasks of each level in the chunks so far
        int start[kTaskLevels];
#pragma unroll
        for (int v = 0; v < kTaskLevels; ++v) below[v] = 0;
        for (int c = 0; c < ntask; c += 64) {
            const int t = c + lane;
            const int lv = t < ntask ? level_of(t) : -1;
#pragma unroll
            for (int v = 0; v < kTaskLevels; ++v) below[v] += __popcll(__ballot(lv == v));
        }
        int run = 0, gap = 0;
#pragma unroll
        for (int v = kTaskLevels - 1; v >= 0; --v) {
            if (symitem && v == kTaskLevels / 2 - 1) {
                gap = ((run + 3) & ~3) - run;
                if (lane < gap) L.torder[run + lane] = 0xffffu;
                run += gap;
            }
            start[v] = run;
            run += below[v];
            below[v] = 0;
        }
        if (lane == 0) L.ntask_eff = ntask + gap;
        for (int c = 0; c < ntask; c += 64) {
            const int t = c + lane;
            const int lv = t < ntask ? level_of(t) : -1;
            int pos = 0;
#pragma unroll
            for (int v = 0; v < kTaskLevels; ++v) {
                const uint64_t m = __ballot(lv == v);
                if (lv == v)
                    pos = start[v] + below[v] +
                          (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                below[v] += __popcll(m);
            }
            if (t < ntask) L.torder[pos] = (uint16_t)t;
        }
    }
    for (int t = tid; t < 4 * kChunk; t += blockDim.x)
        (&L.acc[0][0])[t] = make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();

    // Row phase.  Tasks run in groups of 4, one per 16-lane row; the part's
    // groups (every nparts-th) are dealt to the waves in turn, and a wave
    // runs each group for its longest row's tile count.  The loads are
    // software-pipelined over the wave's whole sequence of groups: while a
    // tile is computed, the next tile's source data (with, at the start of
    // a group, the row's receiver) and the source index of the tile after
    // it are in flight, so a new group starts without waiting for memory.
    const int row = lane >> 4;
    const int l16 = lane & 15;
    auto group_of = [&](int q) { return part + nparts * (wave + 4 * q); };
    // task word of this row in the wave's group q (0: none)
    const int ntask_eff = L.ntask_eff;
    const bool by_tiles = A.task_sort && !symitem;   // tasks in falling tile count
    auto task_word = [&](int q, bool &ok) -> uint32_t {
        const int t = group_of(q) * 4 + row;
        const int k = t < ntask_eff ? (int)L.torder[t] : 0xffff;
        ok = k != 0xffff;
        return ok ? L.tasks[k] : 0u;
    };
    // the sources of entry gd = 27 g + dir: first slot, count, sorted list's
    // axis and sign
    auto task_src = [&](int gd, int &sb, int &nb, int &s, int &sign) {
        sb = __float_as_int(L.geo_r[gd].w);
        const int pk = L.nb_pk[gd];
        nb = pk & 0xffff;
        s = (pk >> 16) & 15;
        sign = (pk >> 20) & 1 ? -1 : 1;
    };

    // the cursor: the (group, tile) position two tiles ahead of the
    // computation, with what its source indices need
    int cq = 0, ci = 0, cmax = 0;
    uint32_t c_tw = 0;   // the row's task word at the cursor's group (0: none)
    bool cvalid = false;
    // this lane's source in the row's task: tiles that hold one (c_lim), its
    // in-cell index at the cursor (c_j, own cell) or its place in the sorted
    // list (c_ptr, stepping c_step per tile), and the neighbour's first slot
    int c_lim = 0, c_j = 0, c_step = 16, c_sb = 0;
    const uint16_t *c_ptr = sidx;
    bool c_direct = true;
    // index stage (two tiles ahead, at the cursor): source index; at a group
    // start the receiver's rank, loaded by cursor_enter
    bool e2_valid = false, e2_start = false, e2_rok = false;
    int e2_src = -1, e2_sb = 0, e2_ria = 0, e2_sa = 0, e2_m = 0;
    uint32_t e2_tw = 0;
    // first group at or after q with a source tile on any row (groups
    // without one add nothing); issues the load of the row's receiver rank
    // straight into the index stage
    auto cursor_enter = [&](int q) {
        cvalid = false;
        while (group_of(q) * 4 < ntask_eff) {
            bool ok;
            const uint32_t tw = task_word(q, ok);
            const int nt = ok ? task_tiles(tw) : 0;
            // the longest row's tiles (a row's lanes share its task)
            const int m = max(max(__builtin_amdgcn_readlane(nt, 0), __builtin_amdgcn_readlane(nt, 16)),
                              max(__builtin_amdgcn_readlane(nt, 32), __builtin_amdgcn_readlane(nt, 48)));
            if (m == 0) {
                // in an order by tile count every later group is empty too
                if (by_tiles) return;
                ++q;
                continue;
            }
            if (A.slots && ok && l16 == 0) atomicAdd(A.slots, 256ull * (unsigned)nt);
            const int blk = (int)((tw >> 10) & 31u);
            const int gd = (int)((tw >> 15) & 255u);
            const int g = gd / 27, dir = gd - 27 * g;
            int nbs, axs, sgn;
            task_src(gd, c_sb, nbs, axs, sgn);
            const int j0 = (int)(tw >> 23) * 16 + l16;   // first tile's source
            c_lim = min(nt, max(0, (nbs - j0 + 15) >> 4));
            c_direct = PLAIN || dir == 26;
            c_j = j0;
            c_step = sgn > 0 ? 16 : -16;
            c_ptr = sidx + (size_t)axs * n + c_sb + (sgn > 0 ? j0 : nbs - 1 - j0);
            e2_sa = L.gsa[g];
            const int r = blk * 16 + l16;
            e2_rok = ok && r < L.n_act[gd];
            e2_ria = 0;
            if (e2_rok) {
                if (c_direct) e2_ria = r_lo + r;
                else if (listed) e2_ria = r_lo + rlist[L.recv_off[26 * g + dir] + r];
                else e2_ria = sidx[(size_t)axs * n + e2_sa + (sgn > 0 ? L.gna[g] - 1 - r : r)];
            }
            cq = q;
            ci = 0;
            cmax = m;
            c_tw = ok ? tw : 0u;
            cvalid = true;
            return;
        }
    };
    auto cursor_next = [&]() {
        if (++ci >= cmax) {
            cursor_enter(cq + 1);
        } else {
            c_j += 16;
            c_ptr += c_step;
        }
    };

    auto stage_index = [&]() {
        e2_valid = cvalid;
        e2_start = cvalid && ci == 0;
        e2_tw = c_tw;
        e2_m = cmax;
        e2_src = -1;
        if (cvalid && ci < c_lim) e2_src = c_direct ? c_j : (int)*c_ptr;
        e2_sb = c_sb;
    };
    // data stage (one tile ahead): source data; at a group start the receiver
    // (a lane without a source loads slot 0, and its x is replaced when used)
    bool e1_valid = false, e1_start = false, e1_rok = false, e1_sv = false;
    int e1_pr = 0, e1_m = 0;
    uint32_t e1_tw = 0;
    float4 e1_s = make_float4(0.f, 0.f, 0.f, 0.f), e1_r = e1_s;
    float e1_sh = 0.0f, e1_sg = 0.0f, e1_rh = 0.0f, e1_rg = 0.0f;
    auto stage_data = [&]() {
        e1_valid = e2_valid;
        e1_start = e2_start;
        e1_tw = e2_tw;
        e1_m = e2_m;
        e1_sv = e2_src >= 0;
        const int p = e1_sv ? e2_sb + e2_src : 0;
        e1_s = A.xyzm[p];
        if constexpr (ADJ) {
            e1_sh = A.Hc[p];
            e1_sg = A.gcell[p];
        } else if (symitem) {
            e1_sh = A.Hc[p];
        }
        if (e2_start) {
            e1_rok = e2_rok;
            e1_pr = e2_sa + e2_ria;
            if (e1_rok) {
                e1_r = A.xyzm[e1_pr];
                e1_rh = A.Hc[e1_pr];
                if constexpr (ADJ) e1_rg = A.gcell[e1_pr];
            }
        }
    };

    cursor_enter(0);
    stage_index();
    stage_data();
    cursor_next();
    stage_index();

    // the row loop, built apart for equal masses (the unit sums) and for
    // the rest, so that neither carries the other's accumulators (one build
    // with the choice made at run time in the symmetric form and the plain
    // comparator, whose two builds would not fit the registers)
    auto rows = [&](auto unit_c) {
        const bool unit = static_cast<bool>(unit_c);
        // the computation's group: task, receiver, pair frame and sums
        int nt = 0, t0 = 0, it = 0, ntmax = 0, diag = -1, ai = 0;
        bool recv_ok = false;
        float tx = 0.f, ty = 0.f, tz = 0.f, ux = 0.f, uy = 0.f, uz = 0.f, H2 = 0.f, invH = 0.f,
              invH2 = 0.f, ck = 0.f, mi = 0.f;
        TileAcc acc = {0.f, 0.f, 0.f, 0.f};
        UnitAcc uacc = {0.f, 0.f, 0.f, 0.f, 0.f};
        GradAcc gacc = {0.f, 0.f, 0.f, 0.f};
        // symmetric own-cell groups: the sources' sums of the current tile, and
        // the row's cell (for the sources' places in the item)
        UnitAcc usrc = {0.f, 0.f, 0.f, 0.f, 0.f};
        GradAcc gsrc = {0.f, 0.f, 0.f, 0.f};
        bool symg = false;
        int cell_off = 0, cell_n = 0;
        const float sig2 = A.lj_sigma2, eps = A.lj_eps;
        while (e1_valid) {   // wave-uniform
            const float4 q = e1_s;
            const float qh = e1_sh, qg = e1_sg;
            // a lane without a source sits far away: no receiver reaches it and
            // its own cut-off reaches none (x alone is enough: any distance to it
            // overflows to infinity)
            const float qx = e1_sv ? q.x : 1e30f;
            if (e1_start) {
                // a new group: this row's task (carried from the cursor: a row
                // without one has word 0, no tiles, direction 0), receiver and
                // pair frame
                const uint32_t tw = e1_tw;
                nt = task_tiles(tw);
                ntmax = e1_m;
                t0 = (int)(tw >> 23);
                const int blk = (int)((tw >> 10) & 31u);
                const int gd = (int)((tw >> 15) & 255u);
                const int g = gd / 27, dir = gd - 27 * g;
                const float4 gr = L.geo_r[gd], gu = L.geo_u[gd];
                recv_ok = e1_rok;
                ai = e1_pr - base;
                // a lane without a receiver sits far away, so that no source
                // is within its own or the source's cut-off (the symmetric
                // update and the adjoint also add to the source)
                const float4 pi = recv_ok ? e1_r : make_float4(1e30f, 1e30f, 1e30f, 0.f);
                const float Hi = recv_ok ? e1_rh : 0.0f;
                H2 = Hi * Hi;
                invH = recv_ok ? __builtin_amdgcn_rcpf(Hi) : 0.0f;   // v_rcp_f32, 1 ulp
                invH2 = invH * invH;
                // pair frame: receiver moved for +1 offsets, source for -1 offsets
                // (x - 0 is x: the unshifted side keeps its bits)
                tx = pi.x - gr.x;
                ty = pi.y - gr.y;
                tz = pi.z - gr.z;
                ux = gu.x;
                uy = gu.y;
                uz = gu.z;
                // the own cell's diagonal tile pairs each receiver with itself
                // at K = 0: the group's tile index it of that tile (-1: none)
                diag = dir == 26 ? (r_lo >> 4) + blk - t0 : -1;
                it = 0;
                // groups of symmetric own-cell tasks hold nothing else
                symg = symitem && __ballot(dir == 26) != 0;
                cell_off = L.gsa[g] - base;
                cell_n = L.gna[g];
                if constexpr (ADJ) {
                    ck = (recv_ok ? e1_rg : 0.0f) * ((8.0f / kPi) * (invH * invH) * (invH * invH));
                    mi = pi.w;
                }
            }
            stage_data();
            cursor_next();
            stage_index();

            const int tile = t0 + it;
            const float sx = qx + ux, sy = q.y + uy, sz = q.z + uz, sm = q.w;
            if (SYM && symg) {
                // the own cell, each unordered pair once
                if (it < nt && (ADJ || !LJ)) {
                    const bool on_diag = it == diag;
                    const float hj = qh;
                    const float sinv = hj > 0.0f ? __builtin_amdgcn_rcpf(hj) : 0.0f;   // v_rcp_f32, 1 ulp
                    const float sh2 = hj * hj;
                    if constexpr (ADJ) {
                        const float sc = qg * ((8.0f / kPi) * (sinv * sinv) * (sinv * sinv));
                        PVL_SYM_STEP_G(0) PVL_SYM_STEP_G(1) PVL_SYM_STEP_G(2) PVL_SYM_STEP_G(3)
                        PVL_SYM_STEP_G(4) PVL_SYM_STEP_G(5) PVL_SYM_STEP_G(6) PVL_SYM_STEP_G(7)
                        PVL_SYM_STEP_G(8) PVL_SYM_STEP_G(9) PVL_SYM_STEP_G(10) PVL_SYM_STEP_G(11)
                        PVL_SYM_STEP_G(12) PVL_SYM_STEP_G(13) PVL_SYM_STEP_G(14) PVL_SYM_STEP_G(15)
                    } else {
                        PVL_SYM_STEP_U(0) PVL_SYM_STEP_U(1) PVL_SYM_STEP_U(2) PVL_SYM_STEP_U(3)
                        PVL_SYM_STEP_U(4) PVL_SYM_STEP_U(5) PVL_SYM_STEP_U(6) PVL_SYM_STEP_U(7)
                        PVL_SYM_STEP_U(8) PVL_SYM_STEP_U(9) PVL_SYM_STEP_U(10) PVL_SYM_STEP_U(11)
                        PVL_SYM_STEP_U(12) PVL_SYM_STEP_U(13) PVL_SYM_STEP_U(14) PVL_SYM_STEP_U(15)
                    }
                    // the tile's sources (back on their own lanes after 16 steps)
                    // add their sums to the wave's array
                    const int j = tile * 16 + l16;
                    float4 res;
                    if constexpr (ADJ) {
                        res = make_float4(gsrc.gx, gsrc.gy, gsrc.gz, gsrc.dh);
                        gsrc = GradAcc{0.f, 0.f, 0.f, 0.f};
                    } else {
                        res = make_float4(0.0f, fmaf(2.0f, usrc.v3, -usrc.s3),
                                          6.0f * (usrc.us2 - usrc.uv2), usrc.cnt);
                        usrc = UnitAcc{0.f, 0.f, 0.f, 0.f, 0.f};
                    }
                    if (j < cell_n) {
                        float *dst = reinterpret_cast<float *>(&L.acc[wave][cell_off + j]);
                        atomicAdd(dst + 0, res.x);
                        atomicAdd(dst + 1, res.y);
                        atomicAdd(dst + 2, res.z);
                        atomicAdd(dst + 3, res.w);
                    }
                }
            } else if (it < nt) {
                if constexpr (ADJ) {
                    const float hj = qh, gj = qg;
                    const float sinv = hj > 0.0f ? __builtin_amdgcn_rcpf(hj) : 0.0f;   // v_rcp_f32, 1 ulp
                    const float sh2 = hj * hj;
                    const float sc = gj * ((8.0f / kPi) * (sinv * sinv) * (sinv * sinv));
                    GradAcc &acc = gacc;
                    if (it != diag) PVL_GRAD_STEP(0)
                    PVL_GRAD_STEP(1) PVL_GRAD_STEP(2) PVL_GRAD_STEP(3) PVL_GRAD_STEP(4)
                    PVL_GRAD_STEP(5) PVL_GRAD_STEP(6) PVL_GRAD_STEP(7) PVL_GRAD_STEP(8)
                    PVL_GRAD_STEP(9) PVL_GRAD_STEP(10) PVL_GRAD_STEP(11) PVL_GRAD_STEP(12)
                    PVL_GRAD_STEP(13) PVL_GRAD_STEP(14) PVL_GRAD_STEP(15)
                } else if constexpr (LJ) {
                    if (it != diag) PVL_LJ_STEP(0)
                    PVL_LJ_STEP(1) PVL_LJ_STEP(2) PVL_LJ_STEP(3) PVL_LJ_STEP(4)
                    PVL_LJ_STEP(5) PVL_LJ_STEP(6) PVL_LJ_STEP(7) PVL_LJ_STEP(8)
                    PVL_LJ_STEP(9) PVL_LJ_STEP(10) PVL_LJ_STEP(11) PVL_LJ_STEP(12)
                    PVL_LJ_STEP(13) PVL_LJ_STEP(14) PVL_LJ_STEP(15)
                } else if (unit) {
                    if (it != diag) PVL_TILE_STEP_U(0)
                    PVL_TILE_STEP_U(1) PVL_TILE_STEP_U(2) PVL_TILE_STEP_U(3) PVL_TILE_STEP_U(4)
                    PVL_TILE_STEP_U(5) PVL_TILE_STEP_U(6) PVL_TILE_STEP_U(7) PVL_TILE_STEP_U(8)
                    PVL_TILE_STEP_U(9) PVL_TILE_STEP_U(10) PVL_TILE_STEP_U(11) PVL_TILE_STEP_U(12)
                    PVL_TILE_STEP_U(13) PVL_TILE_STEP_U(14) PVL_TILE_STEP_U(15)
                } else {
                    if (it != diag) PVL_TILE_STEP(0)
                    PVL_TILE_STEP(1) PVL_TILE_STEP(2) PVL_TILE_STEP(3) PVL_TILE_STEP(4)
                    PVL_TILE_STEP(5) PVL_TILE_STEP(6) PVL_TILE_STEP(7) PVL_TILE_STEP(8)
                    PVL_TILE_STEP(9) PVL_TILE_STEP(10) PVL_TILE_STEP(11) PVL_TILE_STEP(12)
                    PVL_TILE_STEP(13) PVL_TILE_STEP(14) PVL_TILE_STEP(15)
                }
            }
            if (++it == ntmax) {
                // the group's last tile: the row's sums go to its wave's array
                float4 res;
                if constexpr (ADJ) {
                    res = make_float4(gacc.gx, gacc.gy, gacc.gz, gacc.dh);
                    gacc = GradAcc{0.f, 0.f, 0.f, 0.f};
                } else if (!LJ && unit) {
                    res = make_float4(0.0f, fmaf(2.0f, uacc.v3, -uacc.s3),
                                      6.0f * (uacc.us2 - uacc.uv2), uacc.cnt);
                    uacc = UnitAcc{0.f, 0.f, 0.f, 0.f, 0.f};
                } else {
                    res = make_float4(acc.rho, acc.wc, acc.dh, acc.cnt);
                    acc = TileAcc{0.f, 0.f, 0.f, 0.f};
                }
                if (recv_ok) {
                    float *dst = reinterpret_cast<float *>(&L.acc[wave][ai]);
                    atomicAdd(dst + 0, res.x);
                    atomicAdd(dst + 1, res.y);
                    atomicAdd(dst + 2, res.z);
                    atomicAdd(dst + 3, res.w);
                }
            }
        }
    };
    if constexpr (!LJ && !ADJ && !SYM && !PLAIN) {
        if (mass == mass)
            rows(std::true_type{});
        else
            rows(std::false_type{});
    } else if constexpr (!LJ && !ADJ) {
        rows(mass == mass);
    } else {
        rows(std::false_type{});
    }
    __syncthreads();

    for (int i = tid; i < nrt; i += blockDim.x) {
        const float4 s0 = L.acc[0][i], s1 = L.acc[1][i], s2 = L.acc[2][i], s3 = L.acc[3][i];
        float sr = ((s0.x + s1.x) + s2.x) + s3.x;
        const float sw = ((s0.y + s1.y) + s2.y) + s3.y;
        float sd = ((s0.z + s1.z) + s2.z) + s3.z;
        const float sc = ((s0.w + s1.w) + s2.w) + s3.w;
        if (!ADJ && !LJ && mass == mass) {
            // equal masses: the sums were taken with unit masses
            sr = mass * sw;
            sd = mass * sd;
        }
        if (nparts > 1)
            A.partial[((size_t)slot * nparts + part) * kChunk + i] = make_float4(sr, sw, sd, sc);
        else
            finalize_receiver<MODE>(A, base + i, sr, sw, sd, sc);
    }
}

// Waves per SIMD: five (at most 96 registers), four for the symmetric
// own-cell forms, whose steps keep both sides' sums live.  At five the
// adjoint keeps three loop-invariant lane values in scratch memory, reloaded
// only in the set-up phases, and still runs faster than at four.
constexpr int queue_waves(int mode, bool sym)
{
    return (mode == kModePlain || !sym) ? 5 : 4;
}

// CENSUS only names the launch that counts pair slots (A.slots set), so that
// a kernel trace keeps it apart from the timed launches.
template <int MODE, bool SYM = false, bool CENSUS = false>
__global__ void __launch_bounds__(kBlock)
    __attribute__((amdgpu_waves_per_eu(queue_waves(MODE, SYM), 8))) k_sweep_queue(SweepArgs A)
{
    __shared__ SweepLds<group_cap(MODE)> L;
    if (A.dflags[0]) {
        // an error flagged before the sweep (pv_check reports it)
        if constexpr (MODE == kModeAdjoint)
            fill_error_outputs(A.n, A.grad_pos, 3, A.grad_h, nullptr, nullptr);
        else if constexpr (MODE == kModeLJ)
            fill_error_outputs(A.n, A.force, 3, A.energy, nullptr, nullptr);
        else
            fill_error_outputs(A.n, A.rho, 1, A.wcount, A.drho_dh, A.ncount);
        return;
    }
    const int nbig = A.qcount[0], nsmall = A.qcount[1];
    // the tail cells (a fixed set: single-chunk cells among the last
    // tail_cells cells) run after all others, as tail_parts items each, so
    // that the final items are short and the workgroups finish together
    const int ntail = A.qcount[3];
    const int nwhole = nbig + nsmall;
    const int nitems = nwhole + ntail * A.tail_parts;
    // XCD ranges: the large-cell chunks first (one queue), then the
    // single-chunk items, cut into kXcds ranges of consecutive cells; a
    // workgroup starts on its die's range (workgroups are dealt to the dies
    // in turn by index) and moves on to the next ranges as they run dry, so
    // that each die's L2 holds one region's neighbourhood; then the tail
    // items (one queue).  Thread 0 keeps its place in this order in LDS.
    // (The symmetric density form takes the one queue: with the ranges its
    // registers overflow.)
    constexpr bool XCD = !(SYM && MODE == kModeSorted);
    auto next_xcd = [&A]() -> int {
        const int xcd = (int)(blockIdx.x % kXcds);
        const int nb = A.qcount[0], ns = A.qcount[1];
        while (true) {
            if (L.qphase == 0) {
                const int i = atomicAdd(&A.xq[0], 1);
                if (i < nb) return i;
                L.qphase = 1;
            } else if (L.qphase == 1) {
                const int r = (xcd + L.qstep) % kXcds;
                const int lo = (int)((int64_t)ns * r / kXcds);
                const int hi = (int)((int64_t)ns * (r + 1) / kXcds);
                const int i = atomicAdd(&A.xq[2 + r], 1);
                if (lo + i < hi) return nb + lo + i;
                if (++L.qstep == kXcds) L.qphase = 2;
            } else {
                const int i = atomicAdd(&A.xq[1], 1);
                return nb + ns + i;   // past the end when the tail is done
            }
        }
    };
    int item = blockIdx.x;
    if (XCD && A.xcd_ranges) {
        if (threadIdx.x == 0) {
            L.qphase = 0;
            L.qstep = 0;
            L.item = next_xcd();
        }
        __syncthreads();
        item = L.item;
    }
    while (item < nitems) {
        // the item's cell (or first cell), chunk, part of a split tail cell
        // and receivers per chunk
        int ca, ch, part = 0, nparts = 1, slot = 0, cs = A.chunk;
        bool run = true;
        if (item < nwhole) {
            const int2 w = item < nbig ? A.items[item] : A.items[A.cap - nsmall + (item - nbig)];
            ca = w.x;
            ch = w.y;
        } else {
            const int j = item - nwhole;
            slot = j / A.tail_parts;
            ca = A.items[A.cap + slot].x;
            const int p = j - slot * A.tail_parts;
            if (A.tail_split) {
                // part p of the cell's receivers, in whole tiles; it writes
                // its receivers' outputs itself
                const int na = A.start[ca + 1] - A.start[ca];
                cs = ((na + A.tail_parts - 1) / A.tail_parts + 15) & ~15;
                ch = p;
                run = p * cs < na;
            } else {
                ch = 0;
                part = p;
                nparts = A.tail_parts;
            }
        }
        if (run) sweep_item<MODE, SYM>(A, L, ca, ch, part, nparts, slot, cs);
        __syncthreads();
        if (threadIdx.x == 0)
            L.item = (XCD && A.xcd_ranges) ? next_xcd() : (int)gridDim.x + atomicAdd(A.head, 1);
        __syncthreads();
        item = L.item;
    }
}

// Receivers of the split tail cells: the parts' sums added in part order (so
// the result does not depend on which part finished first), then finalised.
// One workgroup per tail cell.
template <int MODE>
__global__ void __launch_bounds__(kBlock) k_tail_combine(SweepArgs A)
{
    // the sweep did not run (its workgroups wrote the error outputs)
    if (A.dflags[0]) return;
    const int ntail = A.qcount[3];
    const int slot = blockIdx.x;
    if (slot >= ntail) return;
    const int a = A.items[A.cap + slot].x;
    const int sa = A.start[a];
    const int na = A.start[a + 1] - sa;
    for (int i = threadIdx.x; i < na; i += blockDim.x) {
        const float4 *pp = A.partial + (size_t)slot * A.tail_parts * kChunk + i;
        float4 t = pp[0];
        for (int q = 1; q < A.tail_parts; ++q) {
            const float4 u = pp[(size_t)q * kChunk];
            t.x += u.x;
            t.y += u.y;
            t.z += u.z;
            t.w += u.w;
        }
        finalize_receiver<MODE>(A, sa + i, t.x, t.y, t.z, t.w);
    }
}

// Work items: the chunks of cells larger than one chunk at the front, in any
// order; the other items at the back, counted from the end; the tail cells
// (single-chunk cells with index >= tail_from) after cap.  The other items
// are single cells or, with group > 1, runs of consecutive single-chunk cells
// whose particles fit one chunk together: each row of cells along z is cut
// into blocks of `group` cells, and one thread per block fills runs greedily
// in cell order (empty cells join the run they fall in; a run starts and ends
// at a non-empty cell), then reserves its items' places with one atomic per
// kind.  Items depend only on the cell counts and the box's
// own cell numbering, not on the other boxes of a batch.
// Places for n items of one kind, reserved for the whole wavefront with one
// atomic: this lane's first place.  All 64 lanes must call it together.
__device__ __forceinline__ int wave_reserve(int *counter, int n)
{
    const int lane = threadIdx.x & 63;
    int inc = n;
    for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(inc, off);
        if (lane >= off) inc += o;
    }
    const int total = __shfl(inc, 63);
    int base = 0;
    if (lane == 0 && total) base = atomicAdd(counter, total);
    return __shfl(base, 0) + inc - n;
}

__global__ void k_queue_items(const BoxDesc *__restrict__ box, const int32_t *__restrict__ cell_box,
                              const int32_t *__restrict__ start, int64_t ncell, int cap, int chunk,
                              int group, int64_t tail_from, int2 *__restrict__ items,
                              int *__restrict__ qcount)
{
    // every lane stays to the reservations (a wavefront-wide scan); a lane
    // past the cells, or not at the first cell of a block, has an empty block
    const int64_t c0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = c0 < ncell;
    int end = live ? (int)c0 + 1 : (int)c0;
    if (live && group > 1) {
        const BoxDesc &B = box[cell_box[c0]];
        const int zr = ((int)c0 - B.cell_off) % B.g[2];   // place in its z-row
        end = zr % group != 0 ? (int)c0                    // not the first of a block
                              : (int)c0 + min(group, B.g[2] - zr);
    }
    // the block's cell counts, loaded side by side
    int na[kGroupMax];
#pragma unroll
    for (int u = 0; u < kGroupMax; ++u) {
        const int c = (int)c0 + u;
        na[u] = c < end ? start[c + 1] - start[c] : 0;
    }
    // the block's items: the first pass counts them, the second writes them
    // where one atomic per kind reserved their places
    int base_small = 0, base_chunk = 0, base_tail = 0;
    for (int pass = 0; pass < 2; ++pass) {
        int nsmall = 0, nchunk = 0, ntail = 0;
        int first = -1, last = -1, sum = 0;   // the open run
        auto close_run = [&]() {
            if (first < 0) return;
            if (pass)
                items[cap - 1 - (base_small + nsmall)] =
                    make_int2(first, last > first ? -(last - first + 1) : 0);
            ++nsmall;
            first = -1;
        };
#pragma unroll
        for (int u = 0; u < kGroupMax; ++u) {
            const int c = (int)c0 + u;
            if (na[u] <= 0) continue;   // empty, or past the block
            if (na[u] > chunk) {
                close_run();
                const int nch = (na[u] + chunk - 1) / chunk;
                if (pass)
                    for (int k = 0; k < nch; ++k) items[base_chunk + nchunk + k] = make_int2(c, k);
                nchunk += nch;
            } else if (c >= tail_from) {
                close_run();
                if (pass) items[cap + base_tail + ntail] = make_int2(c, 0);
                ++ntail;
            } else if (first >= 0 && sum + na[u] <= chunk) {
                sum += na[u];
                last = c;
            } else {
                close_run();
                first = last = c;
                sum = na[u];
            }
        }
        close_run();
        if (pass == 0) {
            base_small = wave_reserve(&qcount[1], nsmall);
            base_chunk = wave_reserve(&qcount[0], nchunk);
            base_tail = wave_reserve(&qcount[3], ntail);
        }
    }
}

// Persistent workgroups of a queue sweep: a few per compute unit, never more
// than the cells.
int64_t queue_grid(const SweepTuning &tune, int64_t ncell)
{
    const int64_t wgs = (int64_t)tune.queue_wgs_per_cu * tune.num_cu;
    return std::max<int64_t>(1, std::min<int64_t>(wgs, ncell));
}

// Cells of the split tail.  Auto: a quarter of the workgroups' worth of
// cells, when the queue holds at least two cells per workgroup (with fewer
// there is no tail to trim).
int tail_cells_of(const SweepTuning &tune, int64_t ncell)
{
    const int64_t grid = queue_grid(tune, ncell);
    return tune.tail_parts == 1 ? 0
           : tune.tail_cells > 0 ? tune.tail_cells
           : ncell >= 2 * grid  ? (int)std::min<int64_t>(grid / 4, kTailMaxCells)
                                : 0;
}

// Queue set-up and the persistent sweep in the given mode.
static hipError_t launch_queue_sweep(hipStream_t st, const DevCells &c, int64_t n, int64_t ncell,
                                     SweepArgs A, const SweepTuning &tune, int mode)
{
    if (ncell == 0 || n == 0) {
        // nothing to sweep: a timed launch takes no time
        if (tune.kt_start) (void)hipEventRecord(tune.kt_start, st);
        if (tune.kt_stop) (void)hipEventRecord(tune.kt_stop, st);
        return hipSuccess;
    }
    const int cap = (int)queue_main(n, ncell);
    const int64_t wgs = (int64_t)tune.queue_wgs_per_cu * tune.num_cu;
    // (every workgroup has its own receiver lists)
    const int64_t grid = std::min<int64_t>(queue_grid(tune, ncell), c.rlist_wgs);
    if (grid < 1) return hipErrorInvalidValue;
    // small cells per item, at most.  Auto: eight with at least 16 cells per
    // workgroup (long runs then still leave every workgroup several items),
    // four with at least two, two with at least one, else one cell per item
    // (fewer items than workgroups would leave compute units idle)
    int group = tune.group > 0  ? tune.group
                : ncell >= 16 * wgs ? 8
                : ncell >= 2 * wgs  ? 4
                : ncell >= wgs      ? 2
                                    : 1;
    group = std::min(group, group_cap(mode));
    if (group < 1 || group > kGroupMax) return hipErrorInvalidValue;
    A.tail_parts = tune.tail_parts;
    A.tail_split = tune.tail_split;
    A.tail_cells = tail_cells_of(tune, ncell);
    // the counters (chunks, cells, head, tail cells) start at zero
    hipError_t e = launch_zero(st, c.qcount, kQueueCounters);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_queue_items, dim3((unsigned)((ncell + 255) / 256)), dim3(256), 0, st,
                       c.box, c.cell_box, c.cell_start, ncell, cap, tune.chunk, group,
                       ncell - A.tail_cells, c.items, c.qcount);
    A.box = c.box;
    A.cell_box = c.cell_box;
    A.start = c.cell_start;
    A.xyzm = c.xyzm;
    A.Hc = c.H;
    A.cell_hmax = c.cell_hmax;
    A.orig = c.orig;
    A.sidx = c.sidx;
    A.n = n;
    A.cell_m = c.cell_m;
    A.tiles = c.tiles;
    A.rlist = c.rlist;
    A.tslots = c.tslots;
    A.cell_dx = c.cell_dx;
    A.dx_all = c.dx_all;
    A.items = c.items;
    A.qcount = c.qcount;
    A.head = c.qcount + 2;
    A.xq = c.qcount + 4;
    A.xcd_ranges = tune.xcd_ranges;
    A.cap = cap;
    A.partial = c.partial;
    A.reach_order = tune.reach_order;
    A.task_sort = tune.task_sort;
    A.chunk = tune.chunk;
    if (tune.kt_start) (void)hipEventRecord(tune.kt_start, st);
    if (mode == kModePlain && A.slots)
        hipLaunchKernelGGL((k_sweep_queue<kModePlain, false, true>), dim3((unsigned)grid),
                           dim3(kBlock), 0, st, A);
    else if (mode == kModePlain)
        hipLaunchKernelGGL(k_sweep_queue<kModePlain>, dim3((unsigned)grid), dim3(kBlock), 0, st, A);
    else if (mode == kModeSorted && A.slots && !tune.sym_self)
        hipLaunchKernelGGL((k_sweep_queue<kModeSorted, false, true>), dim3((unsigned)grid),
                           dim3(kBlock), 0, st, A);
    else if (mode == kModeAdjoint && tune.sym_self)
        hipLaunchKernelGGL((k_sweep_queue<kModeAdjoint, true>), dim3((unsigned)grid), dim3(kBlock), 0,
                           st, A);
    else if (mode == kModeAdjoint)
        hipLaunchKernelGGL(k_sweep_queue<kModeAdjoint>, dim3((unsigned)grid), dim3(kBlock), 0, st, A);
    else if (mode == kModeLJ)
        hipLaunchKernelGGL(k_sweep_queue<kModeLJ>, dim3((unsigned)grid), dim3(kBlock), 0, st, A);
    else if (tune.sym_self)
        hipLaunchKernelGGL((k_sweep_queue<kModeSorted, true>), dim3((unsigned)grid), dim3(kBlock), 0,
                           st, A);
    else
        hipLaunchKernelGGL(k_sweep_queue<kModeSorted>, dim3((unsigned)grid), dim3(kBlock), 0, st, A);
    if (tune.kt_stop) (void)hipEventRecord(tune.kt_stop, st);
    if (A.tail_cells > 0 && !A.tail_split) {
        const dim3 tg((unsigned)A.tail_cells);
        if (mode == kModePlain)
            hipLaunchKernelGGL(k_tail_combine<kModePlain>, tg, dim3(kBlock), 0, st, A);
        else if (mode == kModeAdjoint)
            hipLaunchKernelGGL(k_tail_combine<kModeAdjoint>, tg, dim3(kBlock), 0, st, A);
        else if (mode == kModeLJ)
            hipLaunchKernelGGL(k_tail_combine<kModeLJ>, tg, dim3(kBlock), 0, st, A);
        else
            hipLaunchKernelGGL(k_tail_combine<kModeSorted>, tg, dim3(kBlock), 0, st, A);
    }
    return hipGetLastError();
}

hipError_t launch_sweep_tiled(hipStream_t st, const DevCells &c, int64_t n, int64_t ncell,
                              float *rho, float *wcount, float *drho_dh, int32_t *ncount,
                              int *dflags, const SweepTuning &tune, bool plain,
                              unsigned long long *slots)
{
    SweepArgs A = {};
    A.slots = slots;
    A.rho = rho;
    A.wcount = wcount;
    A.drho_dh = drho_dh;
    A.ncount = ncount;
    A.dflags = dflags;
    return launch_queue_sweep(st, c, n, ncell, A, tune, plain ? kModePlain : kModeSorted);
}

hipError_t launch_lj_tiled(hipStream_t st, const DevCells &c, int64_t n, int64_t ncell,
                           float eps, float sigma, float *force, float *energy, int *dflags,
                           const SweepTuning &tune)
{
    SweepArgs A = {};
    A.lj_eps = eps;
    A.lj_sigma2 = sigma * sigma;
    A.force = force;
    A.energy = energy;
    A.dflags = dflags;
    return launch_queue_sweep(st, c, n, ncell, A, tune, kModeLJ);
}

hipError_t launch_backward_tiled(hipStream_t st, const DevCells &c, int64_t n, int64_t ncell,
                                 float *grad_pos, float *grad_h, int *dflags,
                                 const SweepTuning &tune)
{
    SweepArgs A = {};
    A.gcell = c.gcell;
    A.grad_pos = grad_pos;
    A.grad_h = grad_h;
    A.dflags = dflags;
    return launch_queue_sweep(st, c, n, ncell, A, tune, kModeAdjoint);
}

}  // namespace pvl
