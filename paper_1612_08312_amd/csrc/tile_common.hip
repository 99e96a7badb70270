// Model-independent launchers of the tiled sweep: the passes over the
// tiles' crossing lists, the canonical labels the host reads (written to a
// separate buffer), and the dispatch of one sweep of a chain to its model.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "device_util.hpp"
#include "kernels.hpp"
#include "lattice.hpp"
#include "philox.hpp"
#include "tile_common.hpp"

namespace pyro {

// Canonical label of every site into `out` (only when the host reads
// labels; the label array itself is left as the sweep built it, so the walks
// of other threads never see a rewritten entry).
__global__ __launch_bounds__(kBlock) void k_canonical_labels(const int32_t *__restrict__ label,
                                                             int32_t *__restrict__ out, int64_t N)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    out[i] = canonical_label(label, i);
}

hipError_t launch_unite(const Chain &c, hipStream_t st, const LaunchHook &hook)
{
    if (c.counts) PYRO_LAUNCH(kKUnite, k_forest<true>, c.ntile_blocks, kUniteThreads, c);
    else PYRO_LAUNCH(kKUnite, k_forest<false>, c.ntile_blocks, kUniteThreads, c);
    return hipSuccess;
}

hipError_t launch_chain_sweep(const Chain &c, hipStream_t st, const LaunchHook &hook)
{
    if (c.nreps == 0) return hipSuccess;
    return c.model == 1 ? launch_ising_sweep(c, st, hook) : launch_on_sweep(c, st, hook);
}

hipError_t launch_chain_energy_tail(const Chain &c, hipStream_t st, const LaunchHook &hook)
{
    if (c.nreps == 0) return hipSuccess;
    return c.model == 1 ? launch_ising_energy_tail(c, st, hook) : launch_on_energy_tail(c, st, hook);
}

hipError_t launch_canonical_labels(const RepDesc &d, int32_t *out, hipStream_t st)
{
    k_canonical_labels<<<blocks_for(d.N), kBlock, 0, st>>>(d.label, out, d.N);
    return hipGetLastError();
}

// Tiles of the smallest built shape bound the tile count of every shape.
static int64_t max_tiles(int L)
{
    int64_t m = 0;
    for (int s = 0; s < kNumTileShapes; ++s) {
        const TileDims t = tile_dims(s);
        m = std::max<int64_t>(m, (int64_t)((L + t.x - 1) / t.x) * ((L + t.y - 1) / t.y) * ((L + t.z - 1) / t.z));
    }
    return m;
}

int64_t max_tile_count(int L) { return max_tiles(L); }
// A tile's crossing list holds at most 3 pairs for each of the 4 down
// tetrahedra of each of its low-face cells.
int tile_list_stride(int shape)
{
    const TileDims t = tile_dims(shape);
    const int face = t.x * t.y * t.z - (t.x - 1) * (t.y - 1) * (t.z - 1);
    return 2 + 2 * 12 * face;
}

int64_t pair_list_ints(int L)
{
    int64_t m = 0;
    for (int s = 0; s < kNumTileShapes; ++s) {
        const TileDims t = tile_dims(s);
        const int64_t tiles = (int64_t)((L + t.x - 1) / t.x) * ((L + t.y - 1) / t.y) * ((L + t.z - 1) / t.z);
        m = std::max(m, tiles * tile_list_stride(s));
    }
    return m;
}

int64_t ipart_count(int L) { return 2 * max_tiles(L) + blocks_for((int64_t)L * L * L); }
int64_t dpart_count(int L) { return 4 * max_tiles(L) + blocks_for((int64_t)L * L * L); }

}  // namespace pyro
