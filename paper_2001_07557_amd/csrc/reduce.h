// Deterministic block reductions: wave64 butterfly over DPP/permute lanes,
// then a fixed-order sum of the per-wave results through LDS.  Every block
// produces the same bits for the same inputs, and the per-block partials are
// summed in index order by a single finalising block.
#pragma once

#include "lqcd_internal.h"

namespace lqcd {

constexpr int MAX_BLOCK = 512;
constexpr int MAX_WAVES = MAX_BLOCK / 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum of v over the block, valid in thread 0.  All threads must call it.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV]) {
    __shared__ double red[MAX_WAVES][NV];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) red[wave][k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = red[0][k];
            for (int w = 1; w < nw; ++w) s += red[w][k];
            v[k] = s;
        }
    }
}

}  // namespace lqcd
