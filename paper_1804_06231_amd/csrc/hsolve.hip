// Smoothing lengths from the density: the h-iteration that wraps the density
// loop in an SPH code.  Each particle's h satisfies
//
//   rho_i(h_i) h_i^3 = m_i eta^3,
//
// where rho_i(h) uses the receiver's own cut-off gamma h (so the equations are
// independent across particles); with equal masses it is the neighbour-number
// condition (4 pi / 3) H^3 wcount = N_ngb for eta^3 = 3 N_ngb / (4 pi gamma^3).
// One Newton step per density evaluation, on g(h) = rho(h) h^3 - m eta^3 with
// g'(h) = drho_dh h^3 + 3 rho h^2 (drho_dh from the density sweep); a step is
// limited to a factor kMaxStep, and where g' is not positive the fixed-point
// update h (m eta^3 / (rho h^3))^(1/3) is taken instead.
#include "device_util.h"

namespace pvl {

constexpr float kMaxStep = 1.5f;

__global__ void __launch_bounds__(kBlock) k_h_newton(int64_t n, const float *__restrict__ rho,
                                                     const float *__restrict__ drho_dh,
                                                     const float *__restrict__ mass,
                                                     const float *__restrict__ h, float eta3,
                                                     float *__restrict__ h_next,
                                                     uint32_t *__restrict__ resid)
{
    __shared__ uint32_t red[kBlock / 64];
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float r = 0.0f;
    if (p < n) {
        const float hi = h[p], rh = rho[p];
        const float target = mass[p] * eta3;
        const float h2 = hi * hi, h3 = h2 * hi;
        const float g = fmaf(rh, h3, -target);
        const float gp = fmaf(drho_dh[p], h3, 3.0f * rh * h2);
        float hn = gp > 0.0f ? hi - g / gp : hi * cbrtf(target / (rh * h3));
        hn = fminf(fmaxf(hn, hi / kMaxStep), hi * kMaxStep);
        h_next[p] = hn;
        r = fabsf(g) / target;
        if (!(r == r)) r = INFINITY;   // a NaN residual never reads as converged
    }
    // largest relative residual (non-negative floats order as their bits)
    uint32_t v = __float_as_uint(r);
    for (int off = 32; off > 0; off >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t m = 0u;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = max(m, red[w]);
        atomicMax(resid, m);
    }
}

__global__ void k_copy_f32(int64_t n, const float *__restrict__ src, float *__restrict__ dst)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) dst[p] = src[p];
}

hipError_t launch_h_newton(hipStream_t st, int64_t n, const float *rho, const float *drho_dh,
                           const float *mass, const float *h, float eta3, float *h_next,
                           uint32_t *resid)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_h_newton, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       st, n, rho, drho_dh, mass, h, eta3, h_next, resid);
    return hipGetLastError();
}

hipError_t launch_copy_f32(hipStream_t st, int64_t n, const float *src, float *dst)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, src,
                       dst);
    return hipGetLastError();
}

}  // namespace pvl
