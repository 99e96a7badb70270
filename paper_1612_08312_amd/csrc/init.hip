// Initial states and kernel names.
//   cold:   Ising +1, O(n) (1, 0, 0);
//   random: Ising spin i is -1 when bit (i mod 32) of word ((i/32) mod 4) of
//           Philox(i/128, 0, INIT) is set; O(n) spin i is the unit vector
//           drawn with counter (i, 0, INIT, attempt) (unit_vector.hpp).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"
#include "philox.hpp"
#include "unit_vector.hpp"

namespace pyro {

const char *kernel_name(int id)
{
    static const char *names[kNumKernels] = {"init", "local", "unite", "flip", "energy", "finalize", "persist", "resident"};
    return (id >= 0 && id < kNumKernels) ? names[id] : "?";
}

__global__ __launch_bounds__(kBlock) void k_init_ising(int8_t *__restrict__ s, int64_t N, int start, PhiloxKey key)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int8_t v = 1;
    if (start) {
        const uint4 w = philox4x32_10((uint32_t)(i >> 7), 0u, kStreamInit, 0u, key);
        v = ((word_of(w, (uint32_t)(i >> 5) & 3u) >> (i & 31)) & 1u) ? -1 : 1;
    }
    s[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_init_on(float *__restrict__ s, int64_t N, int n, int start,
                                                    PhiloxKey key)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    float v[3] = {1.0f, 0.0f, 0.0f};
    if (start) unit_vector((uint32_t)i, 0u, kStreamInit, n, key, v);
    for (int k = 0; k < n; ++k) s[(int64_t)k * N + i] = v[k];
}

__global__ __launch_bounds__(kBlock) void k_identity_labels(int32_t *__restrict__ label, int64_t N)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) label[i] = (int32_t)i;
}

hipError_t launch_init(const RepDesc &d, int model, int start, hipStream_t st)
{
    if (model == 1)
        k_init_ising<<<blocks_for(d.N), kBlock, 0, st>>>((int8_t *)d.spins, d.N, start, d.key);
    else
        k_init_on<<<blocks_for(d.N), kBlock, 0, st>>>((float *)d.spins, d.N, model, start, d.key);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_identity_labels<<<blocks_for(d.N), kBlock, 0, st>>>(d.label, d.N);
    return hipGetLastError();
}

}  // namespace pyro
