// Density sweeps (gather form: every receiver i sums over its neighbours j).
//
//   k_sweep_plain   the plain cell list of the paper's Listing 1: each receiver
//                   tests every particle of the 27 surrounding cells.
//   k_sweep_sorted  the pairs the pseudo-Verlet loop of Listing 2 tests under
//                   the loop bounds of Section 3.3, taken one receiver at a
//                   time: for each of the 26 neighbour cells only the
//                   particles whose projected separation on the cell-pair axis
//                   is below the receiver's cut-off, in the receiver's own
//                   cell those within its cut-off in x.  The predicate is
//                   evaluated on every particle of the 27 cells (no sorted
//                   lists), so the count is the bounds' by definition.
//
// Both kernels run one workgroup per receiver cell and finish in place: the
// self term is added, the sums are normalised and written in the caller's
// original particle order, so no separate finalisation pass is needed.  They
// test exactly the pairs the paper's bounds admit, one receiver per lane, and
// serve as the candidate census; the production sweeps are the tiled ones.
#include "device_util.h"

namespace pvl {

struct DensityAcc {
    float rho;   // sum m_j w(u)
    float wc;    // sum w(u)
    float dh;    // sum m_j (3 w(u) + u w'(u))
    int cnt;     // neighbours (self excluded)
};

// One candidate pair: relative position d = x_j - x_i, source mass mj.
__device__ __forceinline__ void density_pair(float dx, float dy, float dz, float mj, float H2,
                                             float invH, DensityAcc &a)
{
    float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    if (r2 < H2) {
        float u = __builtin_amdgcn_sqrtf(r2) * invH;   // v_sqrt_f32, 1 ulp
        float u2 = u * u;
        float v = 1.0f - u;
        float v2 = v * v;
        // inner piece (u < 1/2): w = 1 - 6u^2 + 6u^3, 3w + u w' = 3 - 30u^2 + 36u^3
        float wi = fmaf(u2, fmaf(6.0f, u, -6.0f), 1.0f);
        float di = fmaf(u2, fmaf(36.0f, u, -30.0f), 3.0f);
        // outer piece: w = 2 (1-u)^3, 3w + u w' = 6 (1-u)^2 (1 - 2u)
        float wo = 2.0f * v2 * v;
        float dout = 6.0f * v2 * fmaf(-2.0f, u, 1.0f);
        bool in = u < 0.5f;
        float w = in ? wi : wo;
        float d3 = in ? di : dout;
        a.rho = fmaf(mj, w, a.rho);
        a.wc += w;
        a.dh = fmaf(mj, d3, a.dh);
        a.cnt += 1;
    }
}

__device__ __forceinline__ void write_density(const DensityAcc &a, float H, float mi, int o,
                                              float *rho, float *wcount, float *drho_dh,
                                              int32_t *ncount)
{
    float invH = 1.0f / H;
    float norm = (8.0f / kPi) * invH * invH * invH;
    if (rho) rho[o] = norm * (a.rho + mi);              // self: w(0) = 1
    if (wcount) wcount[o] = norm * (a.wc + 1.0f);
    if (drho_dh) drho_dh[o] = -norm * (kGamma * invH) * (a.dh + 3.0f * mi);  // 1/h = gamma/H
    if (ncount) ncount[o] = a.cnt;
}

// Frames for the difference x_j - x_i of a receiver i in cell a and a source j
// in the neighbour at offset d, whose cell-relative coordinates differ by the
// shift s.  Per axis the operand that lies near the shared face is moved so
// the face sits at zero: the receiver (x_i - s) when d = +1, the source
// (x_j + s) when d = -1.  Both operands are then exact (Sterbenz) or far from
// the face, have opposite signs, and their difference carries no cancellation,
// so the error of every component stays near one rounding of the component
// itself however large the cell is compared with the separation.
struct PairFrame {
    float tx, ty, tz;   // receiver coordinate in the pair frame
    float ux, uy, uz;   // shift added to the source coordinate
};

__device__ __forceinline__ PairFrame pair_frame(float xi, float yi, float zi, int dx, int dy,
                                                int dz, float sx, float sy, float sz)
{
    PairFrame f;
    f.tx = dx > 0 ? xi - sx : xi;
    f.ty = dy > 0 ? yi - sy : yi;
    f.tz = dz > 0 ? zi - sz : zi;
    f.ux = dx < 0 ? sx : 0.0f;
    f.uy = dy < 0 ? sy : 0.0f;
    f.uz = dz < 0 ? sz : 0.0f;
    return f;
}

__global__ void __launch_bounds__(kBlock) k_sweep_plain(
    const BoxDesc *__restrict__ box, const int32_t *__restrict__ cell_box,
    const int32_t *__restrict__ start, const float4 *__restrict__ xyzm,
    const float *__restrict__ Hc, const int32_t *__restrict__ orig, float *rho, float *wcount,
    float *drho_dh, int32_t *ncount, const int *__restrict__ dflags,
    unsigned long long *census, int only_above)
{
    if (dflags[0]) {
        fill_error_outputs(start[gridDim.x] - start[0], rho, 1, wcount, drho_dh, ncount);
        return;
    }
    const int a = blockIdx.x;
    const int sa = start[a];
    const int na = start[a + 1] - sa;
    if (na <= 0 || na <= only_above) return;
    const BoxDesc &B = box[cell_box[a]];
    const CellGeom ga = cell_geom(B, a);
    for (int i0 = 0; i0 < na; i0 += blockDim.x) {
        const int i = i0 + threadIdx.x;
        const bool act = i < na;
        float4 pi = act ? xyzm[sa + i] : make_float4(0.f, 0.f, 0.f, 0.f);
        float Hi = act ? Hc[sa + i] : 0.0f;
        float H2 = Hi * Hi, invH = act ? 1.0f / Hi : 0.0f;
        DensityAcc acc = {0.f, 0.f, 0.f, 0};
        unsigned long long tested = 0;
        if (act) {
            for (int o = 0; o < 27; ++o) {
                int dx = o / 9 - 1, dy = (o / 3) % 3 - 1, dz = o % 3 - 1;
                float sx, sy, sz;
                int b = neighbour(B, ga, dx, dy, dz, sx, sy, sz);
                int sb = start[b], nb = start[b + 1] - sb;
                PairFrame f = pair_frame(pi.x, pi.y, pi.z, dx, dy, dz, sx, sy, sz);
                for (int j = 0; j < nb; ++j) {
                    if (b == a && j == i) continue;
                    float4 q = xyzm[sb + j];
                    density_pair((q.x + f.ux) - f.tx, (q.y + f.uy) - f.ty, (q.z + f.uz) - f.tz, q.w,
                                 H2, invH, acc);
                }
                tested += (unsigned long long)(nb - (b == a ? 1 : 0));
            }
            write_density(acc, Hi, pi.w, orig[sa + i], rho, wcount, drho_dh, ncount);
        }
        if (census && act) {
            atomicAdd(&census[0], tested);
            atomicAdd(&census[1], (unsigned long long)acc.cnt);
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_sweep_sorted(
    const BoxDesc *__restrict__ box, const int32_t *__restrict__ cell_box,
    const int32_t *__restrict__ start, const float4 *__restrict__ xyzm,
    const float *__restrict__ Hc, const int32_t *__restrict__ orig,
    const float *__restrict__ cell_dx, int64_t n, float *rho, float *wcount, float *drho_dh,
    int32_t *ncount, const int *__restrict__ dflags, unsigned long long *census, int only_above)
{
    if (dflags[0]) {
        fill_error_outputs(n, rho, 1, wcount, drho_dh, ncount);
        return;
    }
    const int a = blockIdx.x;
    const int sa = start[a];
    const int na = start[a + 1] - sa;
    if (na <= 0 || na <= only_above) return;
    const BoxDesc &B = box[cell_box[a]];
    const CellGeom ga = cell_geom(B, a);
    // pruning slack covering fp32 rounding of keys and shifts (>> the error)
    const float slack = 1.52587890625e-5f * (B.edge[0] + B.edge[1] + B.edge[2]);
    for (int i0 = 0; i0 < na; i0 += blockDim.x) {
        const int i = i0 + threadIdx.x;
        const bool act = i < na;
        float4 pi = act ? xyzm[sa + i] : make_float4(0.f, 0.f, 0.f, 0.f);
        float Hi = act ? Hc[sa + i] : 0.0f;
        float H2 = Hi * Hi, invH = act ? 1.0f / Hi : 0.0f;
        DensityAcc acc = {0.f, 0.f, 0.f, 0};
        unsigned long long tested = 0;
        if (act) {
            // own cell: the particles with |x_j - x_i| < H_i (widened by the
            // rounding slack and by twice the cell's displacement bound after
            // a drift)
            const float wx = Hi + slack + 2.0f * cell_dx[a];
            for (int j = 0; j < na; ++j) {
                if (j == i) continue;
                float4 q = xyzm[sa + j];
                if (!(fabsf(q.x - pi.x) < wx)) continue;
                ++tested;
                density_pair(q.x - pi.x, q.y - pi.y, q.z - pi.z, q.w, H2, invH, acc);
            }
            for (int o = 0; o < 27; ++o) {
                if (o == 13) continue;
                int dx = o / 9 - 1, dy = (o / 3) % 3 - 1, dz = o % 3 - 1;
                float sx, sy, sz;
                int b = neighbour(B, ga, dx, dy, dz, sx, sy, sz);
                int sb = start[b], nb = start[b + 1] - sb;
                if (nb <= 0) continue;
                int sign;
                int s = dir_canon(dx, dy, dz, &sign);
                float e[3];
                dir_axis(s, e);
                float se = fmaf(sx, e[0], fmaf(sy, e[1], sz * e[2]));
                float ki = proj_key(pi.x, pi.y, pi.z, s);
                // both cells' displacement bounds after a drift
                const float mg = cell_dx[a] + cell_dx[b];
                const float reach = Hi + slack + mg;
                PairFrame f = pair_frame(pi.x, pi.y, pi.z, dx, dy, dz, sx, sy, sz);
                for (int j = 0; j < nb; ++j) {
                    float4 q = xyzm[sb + j];
                    const float kj = proj_key(q.x, q.y, q.z, s) + se;
                    // neighbour ahead on the axis: key_j - key_i < H_i; behind:
                    // key_i - key_j < H_i
                    if (!((sign > 0 ? kj - ki : ki - kj) < reach)) continue;
                    ++tested;
                    density_pair((q.x + f.ux) - f.tx, (q.y + f.uy) - f.ty, (q.z + f.uz) - f.tz, q.w,
                                 H2, invH, acc);
                }
            }
            write_density(acc, Hi, pi.w, orig[sa + i], rho, wcount, drho_dh, ncount);
        }
        if (census && act) {
            atomicAdd(&census[0], tested);
            atomicAdd(&census[1], (unsigned long long)acc.cnt);
        }
    }
}

hipError_t launch_sweep(hipStream_t st, const DevCells &c, int64_t n, int64_t ncell, int algo,
                        float *rho, float *wcount, float *drho_dh, int32_t *ncount,
                        int *dflags, unsigned long long *census,
                        const SweepTuning &tune)
{
    if (ncell == 0 || n == 0) return hipSuccess;
    if (census) {
        // the census counts the candidates of the exact per-receiver bounds
        // (scalar kernels: one receiver per lane, no tiles), then the pair
        // slots the tiled sweep executes (its outputs replace the scalar ones)
        if (algo == PV_PLAIN_CELL)
            hipLaunchKernelGGL(k_sweep_plain, dim3((unsigned)ncell), dim3(kBlock), 0, st, c.box,
                               c.cell_box, c.cell_start, c.xyzm, c.H, c.orig, rho, wcount,
                               drho_dh, ncount, dflags, census, 0);
        else
            hipLaunchKernelGGL(k_sweep_sorted, dim3((unsigned)ncell), dim3(kBlock), 0, st, c.box,
                               c.cell_box, c.cell_start, c.xyzm, c.H, c.orig,
                               c.cell_dx, n, rho, wcount, drho_dh, ncount, dflags, census, 0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return launch_sweep_tiled(st, c, n, ncell, rho, wcount, drho_dh, ncount, dflags, tune,
                              algo == PV_PLAIN_CELL, census ? census + 2 : nullptr);
}

}  // namespace pvl
