// Tile machinery shared by the Ising and O(n) sweeps: the LDS cluster forest
// of one tile, tile indexing, and the merge of tile-crossing bonds into the
// global forest.
//
// A tile is a box of TX x TY x TZ cells handled by one workgroup (one thread
// per cell).  Tiles at the high end of an axis are ragged when the tile edge
// does not divide L; when L is smaller than the tile edge the tile spans the
// whole axis and its periodic bonds wrap onto itself.
//
// After the tile pass every site's label is its tile-local root (a global
// site index) and local roots point at themselves.  The merge unites local
// roots only, always hooking the larger root under the smaller one, so the
// entries of ordinary sites keep pointing at their local root and every
// final root is the smallest site index of its cluster.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_util.hpp"
#include "kernels.hpp"
#include "lattice.hpp"

namespace pyro {

// The tile forest is keyed by the canonical local index key = 16 c + k (cell
// c of the tile, site k), whose order follows the global site order, but is
// stored at position k * NC + c so that the lanes of a wave, which own
// consecutive cells, touch consecutive LDS banks.
template <int NC>
__device__ __forceinline__ int lds_pos(int key)
{
    return (key & 15) * NC + (key >> 4);
}

template <int NC>
__device__ __forceinline__ int lds_find(volatile int *P, int x)
{
    int p = P[lds_pos<NC>(x)];
    while (p != x) {
        const int gp = P[lds_pos<NC>(p)];
        if (gp != p) P[lds_pos<NC>(x)] = gp;
        x = p;
        p = gp;
    }
    return x;
}

// Union in an LDS forest: the larger root is lowered to the smaller one with
// atomicMin; if it had been re-parented meanwhile, continue with its new
// parent.  Parent values only decrease, so every loop ends.
template <int NC>
__device__ __forceinline__ void lds_unite(int *P, int a, int b)
{
    volatile int *V = P;
    for (;;) {
        a = lds_find<NC>(V, a);
        b = lds_find<NC>(V, b);
        if (a == b) return;
        if (a < b) {
            const int tmp = a;
            a = b;
            b = tmp;
        }
        const int old = atomicMin(P + lds_pos<NC>(a), b);
        if (old == a) return;
        a = old;
    }
}

struct NbrCell {
    int gcell;  // global cell index
    int lcell;  // local cell index in the tile, or -1 if outside
};

template <int TX, int TY, int TZ>
struct TileIdx {
    int L, bx, by, bz;

    __device__ __forceinline__ static TileIdx of(int tile, const RepDesc &d)
    {
        TileIdx t;
        t.L = d.L;
        t.bx = tile % d.ntx;
        tile /= d.ntx;
        t.by = tile % d.nty;
        t.bz = tile / d.nty;
        return t;
    }
    __device__ __forceinline__ NbrCell at(int x, int y, int z) const
    {
        NbrCell c;
        c.gcell = (z * L + y) * L + x;
        const int tx = x - bx * TX, ty = y - by * TY, tz = z - bz * TZ;
        const bool in = (unsigned)tx < (unsigned)TX && (unsigned)ty < (unsigned)TY && (unsigned)tz < (unsigned)TZ;
        c.lcell = in ? (tz * TY + ty) * TX + tx : -1;
        return c;
    }
    // Global site index of local key l = 16 c + k.
    __device__ __forceinline__ int global_site(int l) const
    {
        const int lc = l >> 4;
        const int x = bx * TX + lc % TX, y = by * TY + (lc / TX) % TY, z = bz * TZ + lc / (TX * TY);
        return 16 * ((z * L + y) * L + x) + (l & 15);
    }
    // The seven cells the bonds of cell (x, y, z) touch (periodic wrap).
    __device__ __forceinline__ void neighbours(int x, int y, int z, int cell, int lcell,
                                              NbrCell nb[kNCellCodes]) const
    {
        const int xm = x == 0 ? L - 1 : x - 1, ym = y == 0 ? L - 1 : y - 1, zm = z == 0 ? L - 1 : z - 1;
        nb[kSelf] = NbrCell{cell, lcell};
        nb[kMx] = at(xm, y, z);
        nb[kMy] = at(x, ym, z);
        nb[kMz] = at(x, y, zm);
        nb[kMyMz] = at(x, ym, zm);
        nb[kMxMz] = at(xm, y, zm);
        nb[kMxMy] = at(xm, ym, z);
    }
};

// Only cells on a low face of a tile own bonds that leave the tile.
__device__ __forceinline__ bool is_face_cell(int lx, int ly, int lz, const RepDesc &d)
{
    return (lx == 0 && d.ntx > 1) || (ly == 0 && d.nty > 1) || (lz == 0 && d.ntz > 1);
}

// Hash-set size of the merge for a tile shape: a power of two above the
// number of crossing bonds a tile can own (24 per face cell).
template <int TX, int TY, int TZ>
struct MergeHash {
    static constexpr int faces = TX * TY * TZ - (TX - 1) * (TY - 1) * (TZ - 1);
    static constexpr int need = 24 * faces;
    static constexpr int value = need <= 1024 ? 1024 : need <= 2048 ? 2048 : 4096;
    static_assert(need <= 4096, "tile too large for the merge hash set");
};

// One workgroup per tile: gather the (local root, local root) pairs of the
// tile's crossing bonds, drop duplicates in an LDS hash set, and unite each
// distinct pair once in the global forest.  Many crossing bonds of one
// cluster join the same two local roots.
template <int TX, int TY, int TZ>
__global__ __launch_bounds__(TX *TY *TZ) void k_merge(Chain c)
{
    constexpr int NC = TX * TY * TZ;
    constexpr int HASH = MergeHash<TX, TY, TZ>::value;
    __shared__ unsigned long long H[HASH];
    __shared__ unsigned long long U[HASH];
    __shared__ int n_unique;
    const int rep = c.tile_rep[blockIdx.x];
    if (c.state[rep]->remaining <= 0) return;
    const RepDesc &d = c.desc[rep];
    const TileIdx<TX, TY, TZ> ti = TileIdx<TX, TY, TZ>::of(blockIdx.x - d.tile_base, d);
    const int tid = threadIdx.x;
    const int L = d.L;
    int32_t *label = d.label;
    for (int k = tid; k < HASH; k += NC) H[k] = ~0ull;
    if (tid == 0) n_unique = 0;
    __syncthreads();
    const int lx = tid % TX, ly = (tid / TX) % TY, lz = tid / (TX * TY);
    const int x = ti.bx * TX + lx, y = ti.by * TY + ly, z = ti.bz * TZ + lz;
    if (x < L && y < L && z < L && is_face_cell(lx, ly, lz, d)) {
        const int cell = (z * L + y) * L + x;
        const uint64_t m = d.xmask[cell];
        if (m) {
            const CellNbrs nb = cell_neighbours(cell, L);
            const uint32_t down = (uint32_t)(m >> 24);
#pragma unroll
            for (int jj = 0; jj < 24; ++jj) {
                if (!((down >> jj) & 1u)) continue;
                const SiteRef A = bond_end_a(24 + jj), B = bond_end_b(24 + jj);
                int ra = label[16 * nb.c[A.cell] + A.site];
                int rb = label[16 * nb.c[B.cell] + B.site];
                if (ra > rb) {
                    const int tmp = ra;
                    ra = rb;
                    rb = tmp;
                }
                const unsigned long long key = ((unsigned long long)(unsigned)ra << 32) | (unsigned)rb;
                uint32_t h = ((uint32_t)ra * 0x9E3779B1u) ^ ((uint32_t)rb * 0x85EBCA77u);
                h ^= h >> 15;
                for (int probe = 0; probe < HASH; ++probe) {
                    const int slot = (int)((h + (uint32_t)probe) & (HASH - 1));
                    const unsigned long long prev = atomicCAS(&H[slot], ~0ull, key);
                    if (prev == ~0ull) {
                        U[atomicAdd(&n_unique, 1)] = key;
                        break;
                    }
                    if (prev == key) break;
                }
            }
        }
    }
    __syncthreads();
    const int nu = n_unique;
    for (int k = tid; k < nu; k += NC) {
        const unsigned long long key = U[k];
        uf_unite(label, (int)(key >> 32), (int)(key & 0xFFFFFFFFu));
    }
}

// After the merge: point every local root that was hooked straight at its
// final root.  Every node the merge touched is the local root of an
// endpoint of some crossing bond, so afterwards every site reaches its root
// in at most two reads.  One thread per cell.
template <int TX, int TY, int TZ>
__global__ __launch_bounds__(kBlock) void k_compress_roots(Chain c)
{
    const int rep = c.cblk_rep[blockIdx.x];
    if (c.state[rep]->remaining <= 0) return;
    const RepDesc &d = c.desc[rep];
    const int64_t c64 = (int64_t)(blockIdx.x - d.cblk_base) * kBlock + threadIdx.x;
    if (c64 >= d.ncell) return;
    const int L = d.L;
    const int cell = (int)c64;
    const int x = cell % L, y = (cell / L) % L, z = cell / (L * L);
    if (!is_face_cell(x % TX, y % TY, z % TZ, d)) return;
    const uint64_t m = d.xmask[cell];
    if (!m) return;
    int32_t *label = d.label;
    const CellNbrs nb = cell_neighbours(cell, L);
    const uint32_t down = (uint32_t)(m >> 24);
#pragma unroll
    for (int jj = 0; jj < 24; ++jj) {
        if (!((down >> jj) & 1u)) continue;
        const SiteRef A = bond_end_a(24 + jj), B = bond_end_b(24 + jj);
        const int ra = label[16 * nb.c[A.cell] + A.site];
        const int rb = label[16 * nb.c[B.cell] + B.site];
        const int root = uf_find_coherent(label, ra);
        st_coherent(label + ra, root);
        st_coherent(label + rb, root);
    }
}

// Shape dispatch: calls F::template run<TX, TY, TZ>(args...).
template <typename F, typename... Args>
hipError_t with_tile_shape(int shape, Args &&...args)
{
    switch (shape) {
    case kTile844: return F::template run<8, 4, 4>(args...);
    case kTile444: return F::template run<4, 4, 4>(args...);
    case kTile888: return F::template run<8, 8, 8>(args...);
    default: return F::template run<8, 8, 4>(args...);
    }
}

// Launchers of the model-independent kernels (tile_common.hip).
hipError_t launch_merge(const Chain &c, hipStream_t st, const LaunchHook &hook);
hipError_t launch_coins(const Chain &c, hipStream_t st, const LaunchHook &hook);

// Per-model chain launchers (ising_tiled.hip, on_tiled.hip).
hipError_t launch_ising_sweep(const Chain &c, hipStream_t st, const LaunchHook &hook);
hipError_t launch_ising_energy_tail(const Chain &c, hipStream_t st, const LaunchHook &hook);
hipError_t launch_on_sweep(const Chain &c, hipStream_t st, const LaunchHook &hook);
hipError_t launch_on_energy_tail(const Chain &c, hipStream_t st, const LaunchHook &hook);

}  // namespace pyro
