// Host-side launchers of the sweep kernels (one translation unit per model
// family; the C-ABI layer calls only these).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "philox.hpp"

namespace pyro {

// Record layout written by the finalize kernels; identical to pyro_sw_record.
struct DevRecord {
    int64_t sweep, bond_sum, M_int, reserved;
    double E, M[3], m2, m4;
};

constexpr int kBlock = 256;

inline int blocks_for(int64_t n, int per_block = kBlock)
{
    return (int)((n + per_block - 1) / per_block);
}

struct SweepBuffers {
    int L;
    int64_t ncell, N;
    void *spins;          // int8 [N] or float [n][N]
    int32_t *label;       // [N]
    uint64_t *mask;       // [ncell] 48 activation bits per cell
    uint32_t *flipbits;   // [4 * ceil(N/128)]
    float *sigma;         // [N] (O(n))
    float *axis;          // [4] (O(n))
    int64_t *ipart;       // integer partial sums
    double *dpart;        // floating partial sums
    DevRecord *ring;      // per-sweep records
};

struct IsingParams {
    uint32_t thr_hi;  // threshold >> 24 (256 when every parallel bond is active)
    uint32_t thr_lo;  // threshold & 0xFFFFFF
};

// Kernel ids for timing.
enum KernelId : int {
    kKInit = 0,
    kKBonds,
    kKUnion,
    kKFlipTable,
    kKFlip,
    kKEnergy,
    kKFinalize,
    kKAxis,
    kKProject,
    kNumKernels
};
const char *kernel_name(int id);

// Timing hook: the C-ABI layer brackets each launch when enabled.
struct LaunchHook {
    void (*before)(void *ctx, int kernel_id);
    void (*after)(void *ctx, int kernel_id);
    void *ctx;
};

hipError_t launch_init_ising(const SweepBuffers &b, int start, PhiloxKey key, hipStream_t s);
hipError_t launch_init_on(const SweepBuffers &b, int n, int start, PhiloxKey key, hipStream_t s);
hipError_t launch_identity_labels(const SweepBuffers &b, hipStream_t s);

// One sweep with global index t; the record goes to ring[slot].
hipError_t launch_sweep_ising(const SweepBuffers &b, IsingParams p, double J, PhiloxKey key,
                              uint32_t t, int slot, hipStream_t s, const LaunchHook &hook);
hipError_t launch_sweep_on(const SweepBuffers &b, int n, float x0, double J, PhiloxKey key,
                           uint32_t t, int slot, hipStream_t s, const LaunchHook &hook);

}  // namespace pyro
