// Device-side description of the lattices a launch works on, and the
// host-side launchers of the sweep kernels.
//
// Every sweep kernel handles a *chain*: a set of lattices (replicas) of one
// model.  Each replica has a descriptor (geometry, device buffers, constants
// of its run) and a small mutable state (sweep index, sweeps still to run,
// record ring position) that lives in device memory, so that one captured
// graph can replay sweeps for any set of replicas: the kernels read the
// sweep index and skip replicas with nothing left to run, and the last
// kernel of a sweep advances the state.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "philox.hpp"

namespace pyro {

// Store `msg` as the calling thread's last error (pyro_sw_last_error) and
// return `status`.
int record_error(int status, const char *msg);

// Record layout written by the finalize kernels; identical to pyro_sw_record.
struct DevRecord {
    int64_t sweep, bond_sum, M_int, reserved;
    double E, M[3], m2, m4;
};

constexpr int kBlock = 256;  // threads of the per-cell and per-call kernels
constexpr int kFinalizeThreads = 1024;  // one workgroup per replica sums its partials

__host__ __device__ inline int blocks_for(int64_t n, int per_block = kBlock) { return (int)((n + per_block - 1) / per_block); }

// Tile shapes (cells per tile edge) the library is built for.
enum TileShape : int { kTile884 = 0, kTile844 = 1, kTile444 = 2, kTile888 = 3, kTile1688 = 4, kNumTileShapes };
struct TileDims {
    int x, y, z;
};
inline TileDims tile_dims(int shape)
{
    static const TileDims d[kNumTileShapes] = {{8, 8, 4}, {8, 4, 4}, {4, 4, 4}, {8, 8, 8}, {16, 8, 8}};
    return d[shape];
}

struct RepDesc {
    // geometry
    int L, ntx, nty, ntz;  // tiles per axis for the chain's tile shape
    int lgL;               // log2 L when L is a power of two that every tile edge divides, else -1
    int divisible;         // 1 when every tile edge divides L and L >= 2 x the largest edge
    int64_t ncell, N;
    // device buffers owned by the replica
    void *spins;       // int8 [N] or float [n][N]
    int32_t *label;    // [N]
    int64_t *ipart;    // integer partial sums
    double *dpart;     // FP64 partial sums
    DevRecord *ring;   // per-sweep records
    int *pairs;        // per-tile crossing lists: pair count, root count (set by the unite pass), then
                       // (name, name) pairs, replaced by the distinct local roots when the root count is > 0
    int list_stride;   // ints per tile list (tile shape dependent)
    const uint64_t *present;  // Ising site dilution: [ncell] masks of the cell's 48 bonds whose two sites
                              // are occupied (bit j = bond 48 cell + j), or null when no site is vacant
    // constants of the run
    uint32_t thr_hi, thr_lo;  // Ising threshold split at bit 24
    float x0;                 // O(n): (float)(2J/T)
    double J;
    PhiloxKey key;
    int ring_cap;
    int mpart_off;  // per-tile magnetisation partials start here in ipart / dpart
    int tail_off;   // per-cell-block partials of the energy tail start here
    // first block of this replica in each grid of its chain
    int tile_base, cblk_base;
};

struct RepState {
    uint32_t t;         // global index of the next sweep
    int32_t remaining;  // sweeps still to run in the current call
    int32_t ring_used;  // records in the ring
    int32_t e_pending;  // ring slot whose energy is not reduced yet, or -1
};

// What every chain kernel receives: descriptors, states and the block ->
// replica maps of the two grids.
struct Chain {
    const RepDesc *desc;
    RepState *const *state;  // state of each replica (in its own workspace)
    const int *tile_rep;  // tile grid
    const int *cblk_rep;  // 256-cell blocks
    int nreps;
    int shape;            // TileShape of the tile grid
    int model;            // 1, 2, 3
    int ntile_blocks, ncell_blocks;
    unsigned long long *counts;  // null, or [2]: compare-and-swaps of the unite pass tried, and that hooked
};

// Kernel ids for timing (names in init.hip).
enum KernelId : int {
    kKInit = 0,
    kKLocal,     // tile pass
    kKUnite,     // forest unite pass
    kKFlip,      // settle and flip
    kKEnergy,    // energy tail
    kKFinalize,
    kKPersist,   // persistent fused sweep (all sweeps of a call)
    kKResident,  // LDS-resident small lattices (all sweeps of a call)
    kNumKernels
};
const char *kernel_name(int id);

// Optional timing hook around each launch (the C-ABI layer brackets
// launches with HIP events when timing is enabled).
struct LaunchHook {
    void (*before)(void *ctx, int kernel_id);
    void (*after)(void *ctx, int kernel_id);
    void *ctx;
};

// Initial state of one replica.
hipError_t launch_init(const RepDesc &d, int model, int start, hipStream_t st);
// One sweep of every replica of the chain with remaining > 0.
hipError_t launch_chain_sweep(const Chain &c, hipStream_t st, const LaunchHook &hook);
// Energy of the current state into the pending record of every replica of
// the chain, then mark it complete.
hipError_t launch_chain_energy_tail(const Chain &c, hipStream_t st, const LaunchHook &hook);
// Persistent fused Ising sweep: every sweep of a call for all replicas of the
// chain in one launch of `grid` workgroups (control words: kPersistStride
// ints per replica plus one line; see ising_tiled.hip).
constexpr int kPersistStride = 32;
constexpr int kPersistSpin = 1 << 22;  // polls of a wait (about 1 us each) before the launch gives up
hipError_t launch_ising_persistent(const Chain &c, int *ctl, int grid, hipStream_t st, const LaunchHook &hook);
hipError_t ising_persistent_blocks_per_cu(int shape, int *blocks_per_cu);

// Canonical label (smallest site index of the cluster) of every site of one
// replica into the device array out[N].
hipError_t launch_canonical_labels(const RepDesc &d, int32_t *out, hipStream_t st);

// Sizes of the per-replica partial-sum buffers (any tile shape):
// ipart = [E per tile][M per tile][tail per 256-cell block],
// dpart = [E per tile][M per tile x 3][tail per 256-cell block].
int64_t max_tile_count(int L);
// Ints per tile of the crossing lists for a tile shape, and ints of all
// lists of one lattice for the shape that needs most.
int tile_list_stride(int shape);
int64_t pair_list_ints(int L);
int64_t ipart_count(int L);
int64_t dpart_count(int L);

#define PYRO_LAUNCH(id, kernel, grid, block, ...)               \
    do {                                                        \
        if ((grid) > 0) {                                       \
            if (hook.before) hook.before(hook.ctx, id);         \
            kernel<<<(grid), (block), 0, st>>>(__VA_ARGS__);    \
            if (hook.after) hook.after(hook.ctx, id);           \
            hipError_t e_ = hipGetLastError();                  \
            if (e_ != hipSuccess) return e_;                    \
        }                                                       \
    } while (0)

}  // namespace pyro
