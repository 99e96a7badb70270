// LDS-resident sweeps of small Ising lattices (resident.hip): limits, LDS
// layout and launcher.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace pyro {

constexpr int kResidentMaxL = 16;      // N = 16 L^3 <= 65536: site indices fit in 16 bits
constexpr int kResidentThreads = 1024;

// Byte offsets in the dynamic LDS of a lattice of edge L: forest (2 B per
// site), reduction scratch, cell spin masks (2 B per cell), coin words, K4
// table.  At L = 16: 147,648 B.
struct ResidentLayout {
    uint32_t pf, red, smk, cw, k4, total;
};

__host__ __device__ inline ResidentLayout resident_layout(int L)
{
    const uint32_t ncell = (uint32_t)(L * L * L), N = 16u * ncell;
    ResidentLayout r;
    r.pf = 0;
    r.red = 2u * N;  // N is a multiple of 16: 8-byte aligned
    r.smk = r.red + 16u * 8u;
    r.cw = r.smk + ((2u * ncell + 3u) & ~3u);
    r.k4 = r.cw + 4u * ((N + 31u) / 32u);
    r.total = r.k4 + 64u;
    return r;
}

// All `remaining` sweeps of every replica of the chain (each of edge
// L <= kResidentMaxL, no vacant site), one workgroup per replica, with the
// dynamic LDS of the largest edge maxL.
hipError_t launch_resident_ising(const Chain &c, int maxL, hipStream_t st, const LaunchHook &hook);

}  // namespace pyro
