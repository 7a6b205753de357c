// Per-cell, per-axis sort (Section 2 of the paper: the particles of each cell
// are projected on the axis joining the cell centres and sorted along it; 13
// axes cover all 26 neighbour directions once the +- symmetry is used).
//
// One workgroup per cell.  For each axis s the key of particle r is its
// cell-relative position projected on d_s / |d_s|.  The keys are bucket
// sorted in LDS: the cell's key range along the axis is cut into equal
// buckets (the bucket index is a monotone function of the key), a histogram
// and its prefix sum place every bucket, and each particle's final rank is its
// bucket's start plus the number of bucket mates with a smaller (key, in-cell
// rank) pair.  Equal keys keep in-cell order, so the result is deterministic,
// and the work is linear in the occupancy unless a bucket is crowded.
// Output per axis: the in-cell ranks (uint16) in key order and the keys (fp32).
#include "device_util.h"

namespace pvl {

constexpr int kSortLdsBytes = 48 * 1024;

__device__ __forceinline__ int sort_buckets(int cnt)
{
    if (cnt <= 256) return 128;
    int p = next_pow2(cnt);
    return cnt <= 1024 ? p >> 1 : p >> 2;
}

__global__ void __launch_bounds__(kBlock) k_sort13(const BoxDesc *__restrict__ box,
                                                    const int32_t *__restrict__ cell_box,
                                                    const int32_t *__restrict__ start,
                                                    const float4 *__restrict__ xyzm, int64_t n,
                                                    uint16_t *__restrict__ sidx,
                                                    float *__restrict__ skey)
{
    __shared__ __align__(16) unsigned char lds[kSortLdsBytes];
    const int c = blockIdx.x;
    const int s0 = start[c];
    const int cnt = start[c + 1] - s0;
    if (cnt <= 0 || cnt > PV_MAX_CELL) return;
    const BoxDesc &B = box[cell_box[c]];
    const int NB = sort_buckets(cnt);
    const int per_axis = NB * 4 + cnt * 8 + ((cnt * 2 + 15) & ~15);
    int G = kSortLdsBytes / per_axis;
    G = G > 13 ? 13 : (G < 1 ? 1 : G);

    for (int sf = 0; sf < 13; sf += G) {
        const int ng = 13 - sf < G ? 13 - sf : G;
        uint32_t *hist = reinterpret_cast<uint32_t *>(lds);                          // [ng][NB]
        uint64_t *key = reinterpret_cast<uint64_t *>(lds + (size_t)ng * NB * 4);     // [ng][cnt]
        uint16_t *order = reinterpret_cast<uint16_t *>(lds + (size_t)ng * NB * 4 + (size_t)ng * cnt * 8);
        for (int t = threadIdx.x; t < ng * NB; t += blockDim.x) hist[t] = 0u;
        __syncthreads();
        // keys, buckets, histogram
        for (int t = threadIdx.x; t < ng * cnt; t += blockDim.x) {
            int g = t / cnt, r = t - g * cnt, s = sf + g;
            float4 p = xyzm[s0 + r];
            float k = proj_key(p.x, p.y, p.z, s);
            float e[3];
            dir_axis(s, e);
            float kmin = fminf(e[0], 0.f) * B.edge[0] + fminf(e[1], 0.f) * B.edge[1] +
                         fminf(e[2], 0.f) * B.edge[2];
            float kmax = fmaxf(e[0], 0.f) * B.edge[0] + fmaxf(e[1], 0.f) * B.edge[1] +
                         fmaxf(e[2], 0.f) * B.edge[2];
            int b = (int)((k - kmin) * ((float)NB / (kmax - kmin)));
            b = b < 0 ? 0 : (b >= NB ? NB - 1 : b);
            atomicAdd(&hist[g * NB + b], 1u);
            key[t] = ((uint64_t)float_to_ordered(k) << 32) | ((uint32_t)b << 16) | (uint32_t)r;
        }
        __syncthreads();
        // exclusive scan of every axis' histogram (one wave per axis)
        {
            const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
            const int per = (NB + 63) >> 6;
            for (int g = wave; g < ng; g += (int)(blockDim.x >> 6)) {
                uint32_t *hh = hist + g * NB;
                uint32_t loc = 0;
                for (int k = 0; k < per; ++k) {
                    int q = lane * per + k;
                    if (q < NB) loc += hh[q];
                }
                uint32_t inc = loc;
                for (int off = 1; off < 64; off <<= 1) {
                    uint32_t o = (uint32_t)__shfl_up((int)inc, off);
                    if (lane >= off) inc += o;
                }
                uint32_t run = inc - loc;
                for (int k = 0; k < per; ++k) {
                    int q = lane * per + k;
                    if (q < NB) {
                        uint32_t v = hh[q];
                        hh[q] = run;
                        run += v;
                    }
                }
            }
        }
        __syncthreads();
        // list every bucket's members; afterwards hist[b] is the end of bucket b
        for (int t = threadIdx.x; t < ng * cnt; t += blockDim.x) {
            int g = t / cnt;
            int b = (int)((key[t] >> 16) & 0xffffu);
            uint32_t q = atomicAdd(&hist[g * NB + b], 1u);
            order[g * cnt + q] = (uint16_t)(t - g * cnt);
        }
        __syncthreads();
        // rank = bucket start + bucket mates ordered before this key
        for (int t = threadIdx.x; t < ng * cnt; t += blockDim.x) {
            int g = t / cnt;
            uint64_t mine = key[t];
            int b = (int)((mine >> 16) & 0xffffu);
            int q1 = (int)hist[g * NB + b];
            int q0 = b > 0 ? (int)hist[g * NB + b - 1] : 0;
            int rank = q0;
            for (int q = q0; q < q1; ++q) rank += key[g * cnt + order[g * cnt + q]] < mine;
            size_t o = (size_t)(sf + g) * (size_t)n + (size_t)(s0 + rank);
            sidx[o] = (uint16_t)(mine & 0xffffu);
            skey[o] = ordered_to_float((uint32_t)(mine >> 32));
        }
        __syncthreads();
    }
}

hipError_t launch_sort13(hipStream_t st, const DevCells &c, int64_t n, int64_t ncell)
{
    if (ncell == 0 || n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sort13, dim3((unsigned)ncell), dim3(kBlock), 0, st, c.box, c.cell_box,
                       c.cell_start, c.xyzm, n, c.sidx, c.skey);
    return hipGetLastError();
}

}  // namespace pvl
