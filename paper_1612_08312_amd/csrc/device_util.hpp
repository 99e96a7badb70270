// Small device helpers: lattice index products, deterministic block
// reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pyro {

constexpr int kWave = 64;

// Product of non-negative a, b below 2^24 (every lattice index product:
// L <= 406, so cell indices stay below 2^27) on the full-rate 24-bit
// multiplier; a 32-bit integer multiply is a quarter-rate instruction.
__device__ __forceinline__ int mul24(int a, int b) { return (int)__umul24((unsigned)a, (unsigned)b); }

// Index (z L + y) L + x of cell (x, y, z).
__device__ __forceinline__ int cell_index(int x, int y, int z, int L) { return mul24(mul24(z, L) + y, L) + x; }

// Deterministic sum over a block (blockDim.x multiple of 64, at most 1024):
// fixed shuffle tree inside each wave, then the wave sums in wave order.
// Result valid in thread 0.
// kReuse = false drops the closing barrier, which only protects lds from
// the block's next use of it: for a kernel's last use of its LDS.
template <typename T, bool kReuse = true>
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
    if (kReuse) __syncthreads();
    return s;
}

// block_sum of N values at once, with one barrier instead of N pairs: each
// value goes through the same shuffle tree and the same serial sum over the
// waves as in block_sum, so every result is bit for bit the one block_sum
// gives.  The sums are valid in thread 0; the kernel's last use of lds.
template <typename T, int N>
__device__ __forceinline__ void block_sum_n(T (&v)[N], T *lds /* >= 16 N entries */)
{
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) v[i] += __shfl_down(v[i], off, kWave);
        if (lane == 0) lds[16 * i + wave] = v[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = blockDim.x / kWave;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            T s = T(0);
            for (int w = 0; w < nw; ++w) s += lds[16 * i + w];
            v[i] = s;
        }
    }
}

// Block of a tile grid that this workgroup runs.  Consecutive workgroups
// are dispatched round-robin over the 8 XCDs, each with its own L2; the
// remap gives each XCD a contiguous run of blocks, i.e. of tiles, which
// are numbered x-fastest, so a tile's neighbours mostly run on its XCD and
// the label entries they share come from the same L2.  Used by the forest
// passes (unite 492 -> 475 us per launch over five L = 128 lattices); the
// tile and flip passes keep the plain order, which was 4 us faster for the
// tile pass.
__device__ __forceinline__ int xcd_block(int b, int grid)
{
    constexpr int kXcds = 8;
    const int q = grid / kXcds, r = grid % kXcds;
    const int x = b % kXcds, i = b / kXcds;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

}  // namespace pyro
