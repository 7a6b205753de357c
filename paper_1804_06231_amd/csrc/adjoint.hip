// Adjoint of the density: dL/dx and dL/dh for an upstream gradient G = dL/drho.
//
// rho_i depends on x_k through every pair (i, k) in range of receiver i, so
//   dL/dx_k = sum_{j != k} [G_k m_j W_r(r_kj, H_k) + G_j m_k W_r(r_kj, H_j)] (x_k - x_j) / r_kj
//   dL/dh_k = G_k drho_dh_k
// with W_r(r, H) = 8 / (pi H^4) w'(r / H).  The pair set is the union
// r < max(H_k, H_j); a receiver k gathers both terms, so each output has a
// single writer.  The neighbour search is the same sorted-axis pruning as the
// forward sweep, with the receiver's cut-off widened to max(H_k, H_max of the
// neighbour cell) so that pairs decided by the neighbour's own cut-off are
// kept.
#include "device_util.h"

namespace pvl {

__global__ void k_gather_grad(int64_t n, const int32_t *__restrict__ orig,
                              const float *__restrict__ g, float *__restrict__ gcell)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) gcell[p] = g[orig[p]];
}

struct GradAcc {
    float gx, gy, gz;  // dL/dx_k
    float dh;          // sum m_j (3 w + u w') over r < H_k
};

// d = x_j - x_k.  Receiver k: Gk, mk, Hk, invHk; source j: Gj, mj, Hj.
__device__ __forceinline__ void grad_pair(float dx, float dy, float dz, float mj, float Gj,
                                          float Hj, float Gk, float mk, float Hk, float invHk,
                                          GradAcc &a)
{
    float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    float Hk2 = Hk * Hk, Hj2 = Hj * Hj;
    if ((r2 < Hk2 || r2 < Hj2) && r2 > 0.0f) {
        float invr = __builtin_amdgcn_rsqf(r2);   // v_rsq_f32, 1 ulp
        float r = r2 * invr;
        float coef = 0.0f;
        if (r2 < Hk2) {
            float u = r * invHk;
            float v = 1.0f - u;
            float dw = u < 0.5f ? u * fmaf(18.0f, u, -12.0f) : -6.0f * v * v;
            float w = u < 0.5f ? fmaf(u * u, fmaf(6.0f, u, -6.0f), 1.0f) : 2.0f * v * v * v;
            float i2 = invHk * invHk;
            coef = fmaf(Gk * mj, (8.0f / kPi) * i2 * i2 * dw, coef);
            a.dh = fmaf(mj, fmaf(u, dw, 3.0f * w), a.dh);
        }
        if (r2 < Hj2) {
            float invHj = __builtin_amdgcn_rcpf(Hj);  // v_rcp_f32, 1 ulp
            float u = r * invHj;
            float v = 1.0f - u;
            float dw = u < 0.5f ? u * fmaf(18.0f, u, -12.0f) : -6.0f * v * v;
            float i2 = invHj * invHj;
            coef = fmaf(Gj * mk, (8.0f / kPi) * i2 * i2 * dw, coef);
        }
        // (x_k - x_j) / r = -d / r
        float c = -coef * invr;
        a.gx = fmaf(c, dx, a.gx);
        a.gy = fmaf(c, dy, a.gy);
        a.gz = fmaf(c, dz, a.gz);
    }
}

__global__ void __launch_bounds__(kBlock) k_backward_sorted(
    const BoxDesc *__restrict__ box, const int32_t *__restrict__ cell_box,
    const int32_t *__restrict__ start, const float4 *__restrict__ xyzm,
    const float *__restrict__ Hc, const uint32_t *__restrict__ cell_hmax,
    const int32_t *__restrict__ orig, const uint16_t *__restrict__ sidx,
    const float *__restrict__ skey, const float *__restrict__ gcell, int64_t n,
    float *grad_pos, float *grad_h, const int *__restrict__ dflags)
{
    if (dflags[0]) return;
    const int a = blockIdx.x;
    const int sa = start[a];
    const int na = start[a + 1] - sa;
    if (na <= 0) return;
    const BoxDesc &B = box[cell_box[a]];
    int local = a - B.cell_off;
    int cz = local % B.g[2], cy = (local / B.g[2]) % B.g[1], cx = local / (B.g[2] * B.g[1]);
    float ox = (float)cx * B.edge[0], oy = (float)cy * B.edge[1], oz = (float)cz * B.edge[2];
    const float slack = 1.52587890625e-5f * (B.edge[0] + B.edge[1] + B.edge[2]);
    for (int i0 = 0; i0 < na; i0 += blockDim.x) {
        const int k = i0 + threadIdx.x;
        if (k >= na) continue;
        float4 pk = xyzm[sa + k];
        float Hk = Hc[sa + k];
        float invHk = 1.0f / Hk;
        float Gk = gcell[sa + k];
        GradAcc acc = {0.f, 0.f, 0.f, 0.f};
        for (int j = 0; j < na; ++j) {
            if (j == k) continue;
            float4 q = xyzm[sa + j];
            grad_pair(q.x - pk.x, q.y - pk.y, q.z - pk.z, q.w, gcell[sa + j], Hc[sa + j], Gk, pk.w,
                      Hk, invHk, acc);
        }
        for (int o = 0; o < 27; ++o) {
            if (o == 13) continue;
            int dx = o / 9 - 1, dy = (o / 3) % 3 - 1, dz = o % 3 - 1;
            int bx = cx + dx, by = cy + dy, bz = cz + dz;
            float wx = 0.f, wy = 0.f, wz = 0.f;
            if (bx < 0) { bx += B.g[0]; wx = -B.L[0]; } else if (bx >= B.g[0]) { bx -= B.g[0]; wx = B.L[0]; }
            if (by < 0) { by += B.g[1]; wy = -B.L[1]; } else if (by >= B.g[1]) { by -= B.g[1]; wy = B.L[1]; }
            if (bz < 0) { bz += B.g[2]; wz = -B.L[2]; } else if (bz >= B.g[2]) { bz -= B.g[2]; wz = B.L[2]; }
            float sx = ((float)bx * B.edge[0] - ox) + wx;
            float sy = ((float)by * B.edge[1] - oy) + wy;
            float sz = ((float)bz * B.edge[2] - oz) + wz;
            int b = B.cell_off + (bx * B.g[1] + by) * B.g[2] + bz;
            int sb = start[b], nb = start[b + 1] - sb;
            if (nb <= 0) continue;
            float Hreach = fmaxf(Hk, __uint_as_float(cell_hmax[b]));
            int sign;
            int s = dir_canon(dx, dy, dz, &sign);
            float e[3];
            dir_axis(s, e);
            float se = fmaf(sx, e[0], fmaf(sy, e[1], sz * e[2]));
            float ki = proj_key(pk.x, pk.y, pk.z, s);
            const float *kb = skey + (size_t)s * n + sb;
            const uint16_t *ib = sidx + (size_t)s * n + sb;
            // pair frame: the operand near the shared face is moved so the face is
            // at zero (receiver when the offset is +1, source when -1), which keeps
            // the difference free of cancellation
            float tx = dx > 0 ? pk.x - sx : pk.x, ux = dx < 0 ? sx : 0.0f;
            float ty = dy > 0 ? pk.y - sy : pk.y, uy = dy < 0 ? sy : 0.0f;
            float tz = dz > 0 ? pk.z - sz : pk.z, uz = dz < 0 ? sz : 0.0f;
            int j0, j1;
            if (sign > 0) {
                float t = (ki - se) + Hreach + slack;
                int lo = 0, hi = nb;
                while (lo < hi) { int mid = (lo + hi) >> 1; if (kb[mid] < t) lo = mid + 1; else hi = mid; }
                j0 = 0; j1 = lo;
            } else {
                float t = (ki - se) - Hreach - slack;
                int lo = 0, hi = nb;
                while (lo < hi) { int mid = (lo + hi) >> 1; if (kb[mid] <= t) lo = mid + 1; else hi = mid; }
                j0 = lo; j1 = nb;
            }
            for (int j = j0; j < j1; ++j) {
                int p = sb + ib[j];
                float4 q = xyzm[p];
                grad_pair((q.x + ux) - tx, (q.y + uy) - ty, (q.z + uz) - tz, q.w, gcell[p], Hc[p],
                          Gk, pk.w, Hk, invHk, acc);
            }
        }
        int o = orig[sa + k];
        if (grad_pos) {
            grad_pos[3 * (int64_t)o + 0] = acc.gx;
            grad_pos[3 * (int64_t)o + 1] = acc.gy;
            grad_pos[3 * (int64_t)o + 2] = acc.gz;
        }
        if (grad_h) {
            float norm = (8.0f / kPi) * invHk * invHk * invHk;
            grad_h[o] = Gk * (-norm * (kGamma * invHk) * (acc.dh + 3.0f * pk.w));
        }
    }
}

hipError_t launch_backward(hipStream_t st, const DevCells &c, int64_t n, int64_t ncell,
                           const float *grad_rho, float *grad_pos, float *grad_h,
                           const int *dflags)
{
    if (n == 0 || ncell == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_grad, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n,
                       c.orig, grad_rho, c.gcell);
    hipLaunchKernelGGL(k_backward_sorted, dim3((unsigned)ncell), dim3(kBlock), 0, st, c.box,
                       c.cell_box, c.cell_start, c.xyzm, c.H, c.cell_hmax, c.orig, c.sidx, c.skey,
                       c.gcell, n, grad_pos, grad_h, dflags);
    return hipGetLastError();
}

}  // namespace pvl
