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
//   k_forest      unite pass over the crossing lists (tile_common.hpp): the
//                  global forest over the tiles' local roots.
//   k_settle_flip_ising  one workgroup per tile: settle the tile's hooked
//                  local roots (their cluster's smallest site and flip
//                  coin), then the coin of every site's cluster from an LDS
//                  copy of the tile's labels and the tile's own coins, XOR
//                  flip of the int8 spins, magnetisation of the new state.
//                  (The persistent kernel runs the store pass of
//                  tile_common.hpp and ising_flip_pass instead.)
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

// LDS of the tile pass and of the flip of one tile.
template <int TX, int TY, int TZ>
struct IsingTileLds {
    uint32_t P[kForestSlots<TX * TY * TZ>];     // tile forest
    uint32_t SM[TX * TY * TZ];                  // spin masks of the cells
    uint32_t U[kIsingUnionsPerCell<TX * TY * TZ> * TX * TY * TZ];  // union list
    uint8_t K4[64];
    int64_t red[16];
};

template <int TX, int TY, int TZ>
struct IsingFlipLds {
    alignas(16) int LAB[16 * TX * TY * TZ];  // labels of the tile's sites
    alignas(16) uint32_t CB[TX * TY * TZ];   // coins of the tile's sites
    int64_t red[16];
};

// kLast: the pass is the kernel's last use of its LDS (k_local_ising, not
// the persistent kernel).
template <int TX, int TY, int TZ, bool kLast = false>
__device__ __forceinline__ void ising_tile_pass(const RepDesc &d, const RepState &st, int tile, int tid,
                                                IsingTileLds<TX, TY, TZ> &S)
{
    constexpr int NC = TX * TY * TZ;
    uint32_t *P = S.P, *SM = S.SM, *U = S.U;
    uint8_t *K4 = S.K4;
    int64_t *red = S.red;
    const TileIdx<TX, TY, TZ> ti = TileIdx<TX, TY, TZ>::of(tile, d);
    const int8_t *__restrict__ s = (const int8_t *)d.spins;
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
    tile_components<TX, TY, TZ, kIsingUnionsPerCell<NC>>(d, ti, tile, tid, lcid, valid, cell, act, lc, P, U, SM, K4);
    const int64_t bsum = block_sum<int64_t, !kLast>(valid ? (int64_t)(2 * aligned_count - nbonds) : 0, red);
    if (tid == 0) d.ipart[tile] = bsum;
}

template <int TX, int TY, int TZ>
__global__ __launch_bounds__(TX *TY *TZ) void k_local_ising(Chain c)
{
    __shared__ IsingTileLds<TX, TY, TZ> S;
    const int blk = blockIdx.x;
    const int rep = c.tile_rep[blk];
    const RepState st = *c.state[rep];
    if (st.remaining <= 0) return;
    const RepDesc &d = c.desc[rep];
    ising_tile_pass<TX, TY, TZ, true>(d, st, blk - d.tile_base, threadIdx.x, S);
}

// XOR flip of the int8 spins of `cell` selected by `flipmask` (bit k = site
// 16 cell + k); returns the magnetisation of the cell's new state.
__device__ __forceinline__ int flip_cell(void *spins, int cell, uint32_t flipmask)
{
    int4 *S4 = reinterpret_cast<int4 *>(spins);
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
    return occupied - 2 * down;
}

// One workgroup per tile: the labels of the tile's sites and the coins of
// its own clusters are staged in LDS, so the coin of every site's cluster
// (site -> local root -> stored encoding or the root's own coin) costs no
// scattered global read; then flips and the magnetisation of the new state.
template <int TX, int TY, int TZ>
__device__ __forceinline__ void ising_flip_pass(const RepDesc &d, const RepState &st, int tile, int tid,
                                                IsingFlipLds<TX, TY, TZ> &S)
{
    constexpr int NC = TX * TY * TZ;
    int *LAB = S.LAB;
    uint32_t *CB = S.CB;
    int64_t *red = S.red;
    const TileIdx<TX, TY, TZ> ti = TileIdx<TX, TY, TZ>::of(tile, d);
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
    if (valid) mag = flip_cell(d.spins, cell, cell_flip_mask<NC>(lab, LAB, CB, ti, cell, tid, st.t, d.key));
    const int64_t msum = block_sum<int64_t>((int64_t)mag, red);
    if (tid == 0) d.ipart[d.mpart_off + tile] = msum;
}

// LDS of the settle-and-flip pass: the flip's, plus the list of the tile's
// hooked local roots.
template <int TX, int TY, int TZ>
struct IsingSettleLds {
    IsingFlipLds<TX, TY, TZ> f;
    uint16_t HL[kSettleListPerCell * TX * TY * TZ];  // local keys of the tile's hooked local roots
    int wtot[TX * TY * TZ / 64];
};

// Settle and flip, one workgroup per tile, once every unite is done: the
// settle step (settle_tile_roots), then the flip as in ising_flip_pass
// (MODE = kFlipGeneral), or, when the tile edges divide L and TX >= 8
// (FlipMode), with the labels staged by local key, the coin words drawn
// once per FLIP block and each site's coin found without a branch.
template <int TX, int TY, int TZ, int MODE>
__device__ __forceinline__ void ising_settle_flip_pass(const RepDesc &d, const RepState &st, int tile, int tid,
                                                       IsingSettleLds<TX, TY, TZ> &S)
{
    constexpr int NC = TX * TY * TZ;
    constexpr bool ALIGNED = MODE != kFlipGeneral;  // labels staged by local key, every thread has a cell
    int *LAB = S.f.LAB;
    uint32_t *CB = S.f.CB;
    const TileIdx<TX, TY, TZ> ti = TileIdx<TX, TY, TZ>::of(tile, d);
    const int L = d.L;
    const int lx = tid % TX, ly = (tid / TX) % TY, lz = tid / (TX * TY);
    const int x = ti.bx * TX + lx, y = ti.by * TY + ly, z = ti.bz * TZ + lz;
    const bool valid = ALIGNED || (x < L && y < L && z < L);
    const int cell = cell_index(x, y, z, L);
    int lab[16];
    const uint32_t hm = valid ? stage_cell_labels<NC, ALIGNED>(d.label, cell, tid, lab, LAB) : 0u;
    if constexpr (ALIGNED) {
        if (tid < NC / 8) reinterpret_cast<uint4 *>(CB)[tid] = aligned_coin_words<TX, TY, TZ>(ti, tid, st.t, d.key);
    } else {
        CB[tid] = valid ? cell_coins(cell, st.t, d.key) : 0u;
    }
    settle_tile_roots<TX, TY, TZ, ALIGNED>(d, st, ti, tid, cell, hm, LAB, S.HL, S.wtot);
    int mag = 0;
    if (valid) {
        uint32_t flipmask;
        if constexpr (ALIGNED) flipmask = cell_flip_mask_keyed<TX, TY, TZ, MODE>(lab, LAB, CB, d.lgL, ti, cell, tid);
        else flipmask = cell_flip_mask<NC>(lab, LAB, CB, ti, cell, tid, st.t, d.key);
        mag = flip_cell(d.spins, cell, flipmask);
    }
    const int64_t msum = block_sum<int64_t, false>((int64_t)mag, S.f.red);
    if (tid == 0) d.ipart[d.mpart_off + tile] = msum;
}

template <int TX, int TY, int TZ>
__global__ __launch_bounds__(TX *TY *TZ) void k_settle_flip_ising(Chain c)
{
    __shared__ IsingSettleLds<TX, TY, TZ> S;
    const int blk = blockIdx.x;
    const int rep = c.tile_rep[blk];
    const RepState st = *c.state[rep];
    if (st.remaining <= 0) return;
    const RepDesc &d = c.desc[rep];
    if constexpr (TX % 8 == 0) {
        if (d.lgL >= 0) {
            ising_settle_flip_pass<TX, TY, TZ, kFlipPow2>(d, st, blk - d.tile_base, threadIdx.x, S);
            return;
        }
        if (d.divisible) {
            ising_settle_flip_pass<TX, TY, TZ, kFlipDivisible>(d, st, blk - d.tile_base, threadIdx.x, S);
            return;
        }
    }
    ising_settle_flip_pass<TX, TY, TZ, kFlipGeneral>(d, st, blk - d.tile_base, threadIdx.x, S);
}

// Records and state: energy partials (state before this sweep) into the
// pending record, magnetisation of the new state into a new record (a block
// of NT threads; the sums are exact integers).
template <int NT>
__device__ __forceinline__ void ising_finalize(const RepDesc &d, const RepState &st, RepState *stp, int tid,
                                               int64_t *red)
{
    const int ntiles = d.ntx * d.nty * d.ntz;
    int64_t E = 0, M = 0;
    for (int k = tid; k < ntiles; k += NT) {
        E += d.ipart[k];
        M += d.ipart[d.mpart_off + k];
    }
    E = block_sum<int64_t>(E, red);
    M = block_sum<int64_t>(M, red);
    if (tid == 0) {
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
        *stp = ns;
    }
}

__global__ __launch_bounds__(kFinalizeThreads) void k_finalize_ising(Chain c)
{
    __shared__ int64_t red[16];
    const int rep = blockIdx.x;
    const RepState st = *c.state[rep];
    if (st.remaining <= 0) return;
    ising_finalize<kFinalizeThreads>(c.desc[rep], st, c.state[rep], threadIdx.x, red);
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
        PYRO_LAUNCH(kKFlip, (k_settle_flip_ising<TX, TY, TZ>), c.ntile_blocks, TX * TY * TZ, c);
        return hipSuccess;
    }
};

hipError_t launch_ising_sweep(const Chain &c, hipStream_t st, const LaunchHook &hook)
{
    hipError_t e = with_tile_shape<IsingLocal>(c.shape, c, st, hook);
    if (e == hipSuccess) e = launch_unite(c, st, hook);
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

// ------------------------------------------------ persistent fused sweep ---
// All sweeps of a call for every replica of an Ising chain in one launch:
// a fixed grid of workgroups takes work items, each one phase of one tile of
// one replica (tile pass, unite, store, flip; the last flip item of a sweep
// also finalises the record), until no item is left.  Items of a replica
// are numbered k = (4 s + phase) T + tile (T tiles, sweep s of the call) and
// handed out in that order by the replica's cursor, so an item depends only
// on items handed out before it: it waits until the replica's completed-item
// count reaches 4 s T + phase T (the previous phase complete), which is
// deadlock-free whatever the number of resident workgroups, since every
// item handed out is held by a running workgroup.  A workgroup prefers a
// replica whose next phase is ready, so replicas drift apart and the
// issue-bound passes (tile, flip) of some run beside the latency-bound
// passes (unite, store) of others on the same compute units.
//
// Visibility between phases: after an item its writes are released to agent
// scope (L2 written back) before the completed count is raised; a waiting
// item acquires at agent scope (caches invalidated) after the count is
// reached.  Every wait is bounded: past kPersistSpin polls the error flag is
// raised and every workgroup leaves (the host reports the error).
//
// Control words (ints, one 128-byte line per replica; cleared by
// k_persist_reset before each launch): ctl[0] error flag; for replica r at
// kPersistStride (r + 1): cursor, done, flips arrived this sweep, sweeps of
// the call, items of the call.
__device__ __forceinline__ int *persist_ctl(int *ctl, int r) { return ctl + kPersistStride * (r + 1); }

__global__ void k_persist_reset(Chain c, int *ctl)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r == 0) ctl[0] = 0;
    if (r >= c.nreps) return;
    const RepDesc &d = c.desc[r];
    const int S = max(c.state[r]->remaining, 0);
    int *q = persist_ctl(ctl, r);
    q[0] = 0;
    q[1] = 0;
    q[2] = 0;
    q[3] = S;
    q[4] = 4 * S * d.ntx * d.nty * d.ntz;
}

__device__ __forceinline__ int ld_agent(const int *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

template <int TX, int TY, int TZ>
__global__ __launch_bounds__(TX *TY *TZ) void k_persist_ising(Chain c, int *ctl)
{
    constexpr int NC = TX * TY * TZ;
    __shared__ union {
        IsingTileLds<TX, TY, TZ> tile;
        UniteLds unite;
        int HK[kTileRoots];
        IsingFlipLds<TX, TY, TZ> flip;
        int64_t red[16];
    } S;
    __shared__ int take[3];  // replica (-1: nothing left), item, last flip of the sweep
    const int R = c.nreps;
    int next = blockIdx.x % R;  // replica to try first (thread 0)
    for (;;) {
        // The thread index is laundered on every item, so that nothing derived
        // from it is hoisted out of the item loop: each item is independent,
        // and values kept live across items would only raise register
        // pressure (occupancy).
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        if (tid == 0) {
            int r_take = -1, k = 0;
            // a replica whose next item is ready, among the next few
            for (int probe = 0; probe < 4 && probe < R && r_take < 0; ++probe) {
                const int r = (next + probe) % R;
                int *q = persist_ctl(ctl, r);
                const int total = q[4], T = total / max(4 * q[3], 1);
                const int cur = ld_agent(&q[0]);
                if (cur >= total || ld_agent(&q[1]) < (cur / T) * T) continue;
                k = atomicAdd(&q[0], 1);
                if (k < total) r_take = r;
            }
            // otherwise any replica with items left (the item may wait)
            for (int probe = 0; probe < R && r_take < 0; ++probe) {
                const int r = (next + probe) % R;
                int *q = persist_ctl(ctl, r);
                if (ld_agent(&q[0]) >= q[4]) continue;
                k = atomicAdd(&q[0], 1);
                if (k < q[4]) r_take = r;
            }
            if (ld_agent(&ctl[0])) r_take = -1;
            take[0] = r_take;
            take[1] = k;
            if (r_take >= 0) {
                next = (r_take + 1) % R;
                // wait for the previous phase of this replica
                int *q = persist_ctl(ctl, r_take);
                const int T = q[4] / (4 * q[3]);
                const int need = (k / T) * T;
                for (int spin = 0; ld_agent(&q[1]) < need; ++spin) {
                    if (spin >= kPersistSpin || ld_agent(&ctl[0])) {
                        atomicOr(&ctl[0], 1);
                        take[0] = -1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
        }
        __syncthreads();
        // the item is the same for every lane: keep it in scalar registers
        const int r = __builtin_amdgcn_readfirstlane(take[0]), k = __builtin_amdgcn_readfirstlane(take[1]);
        if (r < 0) return;
        const RepDesc &d = c.desc[r];
        const int T = d.ntx * d.nty * d.ntz;
        const int seg = k / T, tile = k - seg * T, phase = seg & 3;
        const RepState st = *c.state[r];
        if (phase == 0) ising_tile_pass<TX, TY, TZ>(d, st, tile, tid, S.tile);
        else if (phase == 1) unite_tile<NC>(d, tile, tid, S.unite);
        else if (phase == 2) store_tile<NC>(d, st, tile, tid, S.HK);
        else ising_flip_pass<TX, TY, TZ>(d, st, tile, tid, S.flip);
        __syncthreads();
        int *q = persist_ctl(ctl, r);
        if (phase == 3) {
            if (tid == 0) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                const int old = atomicAdd(&q[2], 1);
                take[2] = (old + 1) % T == 0;
                if (take[2]) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            __syncthreads();
            if (__builtin_amdgcn_readfirstlane(take[2])) ising_finalize<NC>(d, st, c.state[r], tid, S.red);
            __syncthreads();
        }
        if (tid == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            atomicAdd(&q[1], 1);
        }
    }
}

struct IsingPersist {
    template <int TX, int TY, int TZ>
    static hipError_t run(const Chain &c, int *ctl, int grid, hipStream_t st, const LaunchHook &hook)
    {
        k_persist_reset<<<blocks_for(c.nreps), kBlock, 0, st>>>(c, ctl);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        PYRO_LAUNCH(kKPersist, (k_persist_ising<TX, TY, TZ>), grid, TX * TY * TZ, c, ctl);
        return hipSuccess;
    }
    template <int TX, int TY, int TZ>
    static hipError_t grid(int *blocks_per_cu)
    {
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, (const void *)k_persist_ising<TX, TY, TZ>,
                                                            TX * TY * TZ, 0);
    }
};

struct IsingPersistGrid {
    template <int TX, int TY, int TZ>
    static hipError_t run(int *blocks_per_cu) { return IsingPersist::grid<TX, TY, TZ>(blocks_per_cu); }
};

hipError_t launch_ising_persistent(const Chain &c, int *ctl, int grid, hipStream_t st, const LaunchHook &hook)
{
    if (c.nreps == 0) return hipSuccess;
    return with_tile_shape<IsingPersist>(c.shape, c, ctl, grid, st, hook);
}

hipError_t ising_persistent_blocks_per_cu(int shape, int *blocks_per_cu)
{
    return with_tile_shape<IsingPersistGrid>(shape, blocks_per_cu);
}

}  // namespace pyro
