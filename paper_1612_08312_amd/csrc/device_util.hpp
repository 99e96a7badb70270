// Small device helpers: deterministic block reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pyro {

constexpr int kWave = 64;

// Deterministic sum over a block (blockDim.x multiple of 64, at most 1024):
// fixed shuffle tree inside each wave, then the wave sums in wave order.
// Result valid in thread 0.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T *lds /* >= 16 entries */)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    T s = T(0);
    if (threadIdx.x == 0) {
        const int nw = blockDim.x / kWave;
        for (int w = 0; w < nw; ++w) s += lds[w];
    }
    __syncthreads();
    return s;
}

}  // namespace pyro
