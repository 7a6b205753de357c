// Adjoint of the density: dL/dx and dL/dh for an upstream gradient G = dL/drho.
//
// rho_i depends on x_k through every pair (i, k) in range of receiver i, so
//   dL/dx_k = sum_{j != k} [G_k m_j W_r(r_kj, H_k) + G_j m_k W_r(r_kj, H_j)] (x_k - x_j) / r_kj
//   dL/dh_k = G_k drho_dh_k
// with W_r(r, H) = 8 / (pi H^4) w'(r / H).  The pair set is the union
// r < max(H_k, H_j); a receiver k gathers both terms, so each output has a
// single writer.  The upstream gradient is first put in cell order; the sweep
// itself is the tiled work-queue sweep in its adjoint mode, whose pruning uses
// max(H_k, largest cut-off of the neighbour cell) so that pairs decided by the
// neighbour's own cut-off are kept.
#include "device_util.h"

namespace pvl {

__global__ void k_gather_grad(int64_t n, const int32_t *__restrict__ orig,
                              const float *__restrict__ g, float *__restrict__ gcell)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) gcell[p] = g[orig[p]];
}

hipError_t launch_backward(hipStream_t st, const DevCells &c, int64_t n, int64_t ncell,
                           const float *grad_rho, float *grad_pos, float *grad_h,
                           int *dflags, const SweepTuning &tune)
{
    if (n == 0 || ncell == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_grad, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n,
                       c.orig, grad_rho, c.gcell);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_backward_tiled(st, c, n, ncell, grad_pos, grad_h, dflags, tune);
}

}  // namespace pvl
