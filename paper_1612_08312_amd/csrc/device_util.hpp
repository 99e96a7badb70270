// Small device helpers: coherent loads/stores for the concurrent union-find
// and deterministic block reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pyro {

constexpr int kWave = 64;

// Device-coherent (L2) relaxed load/store: values written by other
// workgroups during the same kernel are observed.
__device__ __forceinline__ int ld_coherent(const int *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coherent(int *p, int v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x in the parent forest.  Every parent pointer points to a smaller
// index, so the walk ends; the grandparent shortcut stores only ancestors.
__device__ __forceinline__ int uf_find_coherent(int *lab, int x)
{
    int p = ld_coherent(lab + x);
    while (p != x) {
        const int gp = ld_coherent(lab + p);
        if (gp != p) st_coherent(lab + x, gp);
        x = p;
        p = gp;
    }
    return x;
}

// Union of the trees of a and b: the larger root is hooked under the smaller
// one with compare-and-swap, retried until both sides share a root.  The
// surviving root of a component is therefore its smallest site index.
__device__ __forceinline__ void uf_unite(int *lab, int a, int b)
{
    for (;;) {
        a = uf_find_coherent(lab, a);
        b = uf_find_coherent(lab, b);
        if (a == b) return;
        if (a > b) {
            const int t = a;
            a = b;
            b = t;
        }
        const int old = atomicCAS(lab + b, b, a);
        if (old == b) return;
        b = old;
    }
}

// Plain root walk, valid once no union is running.
__device__ __forceinline__ int uf_find(const int *lab, int x)
{
    int p = lab[x];
    while (p != x) {
        x = p;
        p = lab[x];
    }
    return x;
}

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
