// Ising Swendsen-Wang sweep on gfx950 with LDS-tiled cluster labeling, for a
// chain of lattices (kernels.hpp).
//
// One sweep (method of Sec. 1-2 of the paper; random draws as documented in
// ising_cell.hpp):
//   k_local_ising  one workgroup per tile: stage the 16-bit spin masks of the
//                  tile in LDS, activate the 48 bonds of every cell, merge
//                  each up tetrahedron with a K4 component table, unite the
//                  down-tetrahedron bonds inside the tile in an LDS forest,
//                  write every site's tile-local root as a global site index
//                  and list the tile's crossing pairs (tile_components).  The
//                  parallel-bond count is the energy of the incoming state.
//   k_forest       unite and store passes over the crossing lists
//                  (tile_common.hpp); the store pass writes each merged
//                  cluster's smallest site and flip coin into its local roots.
//   k_flip_ising   one workgroup per tile: the coin of every site's cluster
//                  from an LDS copy of the tile's labels and the tile's own
//                  coins, XOR flip of the int8 spins, magnetisation of the new
//                  state.
//   k_finalize_ising  fixed-order sums of the partials into the records,
//                  then advance the replica's state.
// Local site order inside a tile follows the global order, so a tile-local
// root is the smallest site index of its local component, and the canonical
// passes make every label the smallest site index of its cluster.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_util.hpp"
#include "ising_cell.hpp"
#include "kernels.hpp"
#include "lattice.hpp"
#include "philox.hpp"
#include "tile_common.hpp"

namespace pyro {

template <int TX, int TY, int TZ>
__global__ __launch_bounds__(TX *TY *TZ) void k_local_ising(Chain c)
{
    constexpr int NC = TX * TY * TZ;
    __shared__ uint32_t P[kForestSlots<NC>];
    __shared__ uint32_t SM[NC];
    __shared__ uint32_t U[kUnionsPerCell * NC];
    __shared__ uint8_t K4[64];
    __shared__ int64_t red[16];

    const int rep = c.tile_rep[blockIdx.x];
    const RepState st = *c.state[rep];
    if (st.remaining <= 0) return;
    const RepDesc &d = c.desc[rep];
    const int tile = blockIdx.x - d.tile_base;
    const TileIdx<TX, TY, TZ> ti = TileIdx<TX, TY, TZ>::of(tile, d);
    const int8_t *__restrict__ s = (const int8_t *)d.spins;
    const int tid = threadIdx.x;
    const int L = d.L;
    const int lcid = tid;  // local cell of the thread
    const int lx = lcid % TX, ly = (lcid / TX) % TY, lz = lcid / (TX * TY);
    const int x = ti.bx * TX + lx, y = ti.by * TY + ly, z = ti.bz * TZ + lz;
    const bool valid = x < L && y < L && z < L;
    const int cell = cell_index(x, y, z, L);

    if (tid < 64) {
        constexpr K4Table k4 = make_k4();
        K4[tid] = k4.v[tid];
    }
    uint32_t m = 0;
    if (valid) m = spin_mask16(reinterpret_cast<const int4 *>(s)[cell]);
    SM[lcid] = m;
    __syncthreads();

    uint64_t act = 0;
    int aligned_count = 0, nbonds = 48;
    int lc[kNCellCodes];
#pragma unroll
    for (int q = 0; q < kNCellCodes; ++q) lc[q] = -1;
    if (valid) {
        NbrCell nb[kNCellCodes];
        ti.neighbours(x, y, z, cell, lcid, nb);
        // Spins of the neighbour cells outside the tile: every lane issues all
        // six loads (its own cell, a cache hit, where the neighbour is in the
        // tile), so they are in flight together instead of one divergent
        // branch at a time.
        int4 gv[kNCellCodes];
#pragma unroll
        for (int q = 1; q < kNCellCodes; ++q)
            gv[q] = reinterpret_cast<const int4 *>(s)[nb[q].lcell >= 0 ? cell : nb[q].gcell];
        uint32_t nm[kNCellCodes];
        nm[kSelf] = m;
#pragma unroll
        for (int q = 0; q < kNCellCodes; ++q) {
            lc[q] = nb[q].lcell;
            if (q > 0) nm[q] = nb[q].lcell >= 0 ? SM[nb[q].lcell] : spin_mask16(gv[q]);
        }
        const uint32_t dm = down_mask16(m, nm[kMx], nm[kMy], nm[kMz], nm[kMyMz], nm[kMxMz], nm[kMxMy]);
        uint64_t al = aligned48(m, dm);
        if (d.present) {  // a bond with a vacant end is neither a candidate nor counted in E
            const uint64_t pm = d.present[cell];
            al &= pm;
            nbonds = (int)__popcll(pm);
        }
        aligned_count = (int)__popcll(al);
        act = ising_activate(al, (uint32_t)cell, st.t, d.key, IsingParams{d.thr_hi, d.thr_lo});
    }
    tile_components<TX, TY, TZ>(d, ti, tile, tid, lcid, valid, cell, act, lc, P, U, SM, K4);
    const int64_t bsum = block_sum<int64_t>(valid ? (int64_t)(2 * aligned_count - nbonds) : 0, red);
    if (tid == 0) d.ipart[tile] = bsum;
}

// One workgroup per tile: the labels of the tile's sites and the coins of
// its own clusters are staged in LDS, so the coin of every site's cluster
// (site -> local root -> stored encoding or the root's own coin) costs no
// scattered global read; then flips and the magnetisation of the new state.
template <int TX, int TY, int TZ>
__global__ __launch_bounds__(TX *TY *TZ) void k_flip_ising(Chain c)
{
    constexpr int NC = TX * TY * TZ;
    __shared__ int LAB[16 * NC];
    __shared__ uint32_t CB[NC];
    __shared__ int64_t red[16];
    const int rep = c.tile_rep[blockIdx.x];
    const RepState st = *c.state[rep];
    if (st.remaining <= 0) return;
    const RepDesc &d = c.desc[rep];
    const int tile = blockIdx.x - d.tile_base;
    const TileIdx<TX, TY, TZ> ti = TileIdx<TX, TY, TZ>::of(tile, d);
    const int tid = threadIdx.x;
    const int L = d.L;
    const int lx = tid % TX, ly = (tid / TX) % TY, lz = tid / (TX * TY);
    const int x = ti.bx * TX + lx, y = ti.by * TY + ly, z = ti.bz * TZ + lz;
    const bool valid = x < L && y < L && z < L;
    const int cell = cell_index(x, y, z, L);
    int lab[16];
    if (valid) {
        const int4 *L4 = reinterpret_cast<const int4 *>(d.label + 16 * cell);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int4 v = L4[q];
            lab[4 * q] = v.x;
            lab[4 * q + 1] = v.y;
            lab[4 * q + 2] = v.z;
            lab[4 * q + 3] = v.w;
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) LAB[k * NC + tid] = lab[k];
    }
    CB[tid] = valid ? cell_coins(cell, st.t, d.key) : 0u;
    __syncthreads();
    int mag = 0;
    if (valid) {
        const uint32_t flipmask = cell_flip_mask<NC>(lab, LAB, CB, ti, st.t, d.key);
        int4 *S4 = reinterpret_cast<int4 *>(d.spins);
        const int4 sv = S4[cell];
        uint32_t w[4] = {(uint32_t)sv.x, (uint32_t)sv.y, (uint32_t)sv.z, (uint32_t)sv.w};
        int down = 0, occupied = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t f4 = (flipmask >> (4 * q)) & 15u;
            // +1 (0x01) <-> -1 (0xFF) is XOR 0xFE on the flipped bytes; a
            // vacant site (0x00) is left alone
            const uint32_t nz = (((w[q] & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | w[q]) & 0x80808080u;
            const uint32_t fx = (((f4 & 1u) * 0xFEu) | ((f4 >> 1 & 1u) * 0xFE00u) | ((f4 >> 2 & 1u) * 0xFE0000u) |
                                 ((f4 >> 3 & 1u) * 0xFE000000u)) & ((nz >> 7) * 0xFEu);
            w[q] ^= fx;
            down += (int)__popc(w[q] & 0x80808080u);
            occupied += (int)__popc(nz);
        }
        S4[cell] = make_int4((int)w[0], (int)w[1], (int)w[2], (int)w[3]);
        mag = occupied - 2 * down;
    }
    const int64_t msum = block_sum<int64_t>((int64_t)mag, red);
    if (tid == 0) d.ipart[d.mpart_off + tile] = msum;
}

// Records and state: energy partials (state before this sweep) into the
// pending record, magnetisation of the new state into a new record.
__global__ __launch_bounds__(kFinalizeThreads) void k_finalize_ising(Chain c)
{
    __shared__ int64_t red[16];
    const int rep = blockIdx.x;
    const RepState st = *c.state[rep];
    if (st.remaining <= 0) return;
    const RepDesc &d = c.desc[rep];
    const int ntiles = d.ntx * d.nty * d.ntz;
    int64_t E = 0, M = 0;
    for (int k = threadIdx.x; k < ntiles; k += blockDim.x) {
        E += d.ipart[k];
        M += d.ipart[d.mpart_off + k];
    }
    E = block_sum<int64_t>(E, red);
    M = block_sum<int64_t>(M, red);
    if (threadIdx.x == 0) {
        if (st.e_pending >= 0) {
            d.ring[st.e_pending].bond_sum = E;
            d.ring[st.e_pending].E = -d.J * (double)E;
        }
        const int slot = st.ring_used;
        if (slot < d.ring_cap) {
            DevRecord r;
            r.sweep = st.t;
            r.bond_sum = 0;
            r.M_int = M;
            r.reserved = 0;
            r.E = 0.0;
            r.M[0] = (double)M;
            r.M[1] = 0.0;
            r.M[2] = 0.0;
            const double mm = (double)M / (double)d.N;
            r.m2 = mm * mm;
            r.m4 = r.m2 * r.m2;
            d.ring[slot] = r;
        }
        RepState ns;
        ns.t = st.t + 1;
        ns.remaining = st.remaining - 1;
        ns.ring_used = slot + 1;
        ns.e_pending = slot < d.ring_cap ? slot : -1;
        *c.state[rep] = ns;
    }
}

// Energy of the current state for replicas whose last record is pending.
__global__ __launch_bounds__(kBlock) void k_energy_ising(Chain c)
{
    __shared__ int64_t red[16];
    const int rep = c.cblk_rep[blockIdx.x];
    if (c.state[rep]->e_pending < 0) return;
    const RepDesc &d = c.desc[rep];
    const int blk = blockIdx.x - d.cblk_base;
    const int64_t cl = (int64_t)blk * kBlock + threadIdx.x;
    int64_t B = 0;
    if (cl < d.ncell) {
        const int cell = (int)cl;
        const CellNbrs nb = cell_neighbours(cell, d.L);
        const int4 *S4 = reinterpret_cast<const int4 *>(d.spins);
        const uint32_t m = spin_mask16(S4[cell]);
        const uint32_t dm = down_mask16(m, spin_mask16(S4[nb.c[kMx]]), spin_mask16(S4[nb.c[kMy]]),
                                        spin_mask16(S4[nb.c[kMz]]), spin_mask16(S4[nb.c[kMyMz]]),
                                        spin_mask16(S4[nb.c[kMxMz]]), spin_mask16(S4[nb.c[kMxMy]]));
        uint64_t al = aligned48(m, dm);
        int nbonds = 48;
        if (d.present) {
            const uint64_t pm = d.present[cell];
            al &= pm;
            nbonds = (int)__popcll(pm);
        }
        B = 2 * (int64_t)__popcll(al) - nbonds;
    }
    const int64_t bsum = block_sum<int64_t>(B, red);
    if (threadIdx.x == 0) d.ipart[d.tail_off + blk] = bsum;
}

__global__ __launch_bounds__(kBlock) void k_energy_tail_finalize_ising(Chain c)
{
    __shared__ int64_t red[16];
    const int rep = blockIdx.x;
    const RepState st = *c.state[rep];
    if (st.e_pending < 0) return;
    const RepDesc &d = c.desc[rep];
    const int ncb = blocks_for(d.ncell);
    int64_t E = 0;
    for (int k = threadIdx.x; k < ncb; k += blockDim.x) E += d.ipart[d.tail_off + k];
    E = block_sum<int64_t>(E, red);
    if (threadIdx.x == 0) {
        d.ring[st.e_pending].bond_sum = E;
        d.ring[st.e_pending].E = -d.J * (double)E;
        c.state[rep]->e_pending = -1;
    }
}

struct IsingLocal {
    template <int TX, int TY, int TZ>
    static hipError_t run(const Chain &c, hipStream_t st, const LaunchHook &hook)
    {
        PYRO_LAUNCH(kKLocal, (k_local_ising<TX, TY, TZ>), c.ntile_blocks, TX * TY * TZ, c);
        return hipSuccess;
    }
};

struct IsingFlip {
    template <int TX, int TY, int TZ>
    static hipError_t run(const Chain &c, hipStream_t st, const LaunchHook &hook)
    {
        PYRO_LAUNCH(kKFlip, (k_flip_ising<TX, TY, TZ>), c.ntile_blocks, TX * TY * TZ, c);
        return hipSuccess;
    }
};

hipError_t launch_ising_sweep(const Chain &c, hipStream_t st, const LaunchHook &hook)
{
    hipError_t e = with_tile_shape<IsingLocal>(c.shape, c, st, hook);
    if (e == hipSuccess) e = launch_merge(c, st, hook);
    if (e == hipSuccess) e = with_tile_shape<IsingFlip>(c.shape, c, st, hook);
    if (e != hipSuccess) return e;
    PYRO_LAUNCH(kKFinalize, k_finalize_ising, c.nreps, kFinalizeThreads, c);
    return hipSuccess;
}

hipError_t launch_ising_energy_tail(const Chain &c, hipStream_t st, const LaunchHook &hook)
{
    PYRO_LAUNCH(kKEnergy, k_energy_ising, c.ncell_blocks, kBlock, c);
    PYRO_LAUNCH(kKFinalize, k_energy_tail_finalize_ising, c.nreps, kBlock, c);
    return hipSuccess;
}

}  // namespace pyro
