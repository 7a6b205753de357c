// Per-cell, per-axis sort (Section 2 of the paper: the particles of each cell
// are projected on the axis joining the cell centres and sorted along it; 13
// axes cover all 26 neighbour directions once the +- symmetry is used).
//
// One workgroup per cell.  For each axis s the key of particle r is its
// cell-relative position projected on d_s / |d_s|.  Keys are sorted ascending
// in LDS with a bitonic network on (ordered key bits, in-cell rank) pairs, so
// equal keys keep rank order and the result is deterministic.  Output per axis:
// the in-cell ranks (uint16) in key order and the keys themselves (fp32).
#include "device_util.h"

namespace pvl {

constexpr int kSortLds = PV_MAX_CELL;  // uint64 slots of LDS (32 KB)

__global__ void __launch_bounds__(kBlock) k_sort13(const int32_t *__restrict__ start,
                                                    const float4 *__restrict__ xyzm, int64_t n,
                                                    uint16_t *__restrict__ sidx,
                                                    float *__restrict__ skey)
{
    __shared__ uint64_t keys[kSortLds];
    const int c = blockIdx.x;
    const int s0 = start[c];
    const int cnt = start[c + 1] - s0;
    if (cnt <= 0 || cnt > PV_MAX_CELL) return;
    const int P2 = next_pow2(cnt);
    const int per = kSortLds / P2 < 13 ? kSortLds / P2 : 13;   // axes per pass
    for (int s_first = 0; s_first < 13; s_first += per) {
        int ns = 13 - s_first < per ? 13 - s_first : per;
        for (int t = threadIdx.x; t < ns * P2; t += blockDim.x) {
            int seg = t / P2;
            int r = t - seg * P2;
            uint64_t k = ~0ull;
            if (r < cnt) {
                float4 p = xyzm[s0 + r];
                float key = proj_key(p.x, p.y, p.z, s_first + seg);
                k = ((uint64_t)float_to_ordered(key) << 32) | (uint32_t)r;
            }
            keys[t] = k;
        }
        __syncthreads();
        bitonic_sort_segments(keys, P2, ns);
        for (int t = threadIdx.x; t < ns * P2; t += blockDim.x) {
            int seg = t / P2;
            int r = t - seg * P2;
            if (r < cnt) {
                uint64_t k = keys[t];
                size_t o = (size_t)(s_first + seg) * (size_t)n + (size_t)(s0 + r);
                sidx[o] = (uint16_t)(k & 0xffffu);
                skey[o] = ordered_to_float((uint32_t)(k >> 32));
            }
        }
        __syncthreads();
    }
}

hipError_t launch_sort13(hipStream_t st, const DevCells &c, int64_t n, int64_t ncell)
{
    if (ncell == 0 || n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sort13, dim3((unsigned)ncell), dim3(kBlock), 0, st, c.cell_start, c.xyzm,
                       n, c.sidx, c.skey);
    return hipGetLastError();
}

}  // namespace pvl
