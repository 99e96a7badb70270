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

// Every walk below is capped far above any reachable depth (a forest over n
// nodes has depth below n), so a damaged forest can only give a wrong label,
// never a kernel that does not finish.
constexpr int kWalkCap = 1 << 22;

template <int NC>
__device__ __forceinline__ int lds_find(volatile int *P, int x)
{
    int p = P[lds_pos<NC>(x)];
    for (int it = 0; p != x && it < 16 * NC; ++it) {
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
    for (int it = 0; it < 16 * NC; ++it) {
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
    // Local key 16 c + k of a global site index known to lie in this tile.
    __device__ __forceinline__ int local_key(int site) const
    {
        const int cell = site >> 4;
        const int x = cell % L, y = (cell / L) % L, z = cell / (L * L);
        return 16 * (((z - bz * TZ) * TY + (y - by * TY)) * TX + (x - bx * TX)) + (site & 15);
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

// Endpoints of the 24 down-tetrahedron bonds of a cell (bond 24 + jj):
// bytes (cell code of A, site of A, cell code of B, site of B).
struct DownEnds {
    uint32_t v[24];
};
__host__ __device__ constexpr DownEnds make_down_ends()
{
    DownEnds t{};
    for (int jj = 0; jj < 24; ++jj) {
        const SiteRef A = bond_end_a(24 + jj), B = bond_end_b(24 + jj);
        t.v[jj] = (uint32_t)A.cell | (uint32_t)A.site << 8 | (uint32_t)B.cell << 16 | (uint32_t)B.site << 24;
    }
    return t;
}
static __constant__ DownEnds kDownEnds = make_down_ends();

// Only cells on a low face of a tile own bonds that leave the tile.
__device__ __forceinline__ bool is_face_cell(int lx, int ly, int lz, const RepDesc &d)
{
    return (lx == 0 && d.ntx > 1) || (ly == 0 && d.nty > 1) || (lz == 0 && d.ntz > 1);
}

// ---------------------------------------------------------------- merge ---
// The global forest lives in the label entries of tile-local roots (the
// entries of ordinary sites keep pointing at their local root).  Entry
// encodings of a local root r:
//   r                   r is a root of the merged forest
//   kTag | p            r was hooked under p
//   kCanonBase + c      r is a merged root after the minimum pass: c is the
//                       smallest site index of r's cluster
// Site indices are below 2^30 (L <= 406), so the three forms are distinct and
// the local root of any site is decodable at any time (endpoint_root), even
// while other threads hook roots or store canonical labels.
//
// Roots are linked by a fixed pseudo-random priority (a bijective hash of
// the site index): a root is always hooked under the root of smaller
// priority, so trees stay shallow (expected logarithmic depth) even when one
// cluster spans every tile, whereas linking by index builds chains through
// the tiles.  The smallest index of each merged cluster is then stored in
// its tree root by the minimum pass and copied into every local root of the
// cluster by the store pass.
constexpr int kTag = 1 << 30;
constexpr int kIdxMask = kTag - 1;
constexpr int kCanonBase = INT32_MIN;  // canonical index c is stored as kCanonBase + c

__device__ __forceinline__ uint32_t link_priority(int x)
{
    const uint32_t h = (uint32_t)x * 0x9E3779B1u;
    return h ^ (h >> 16);
}

__device__ __forceinline__ int lab_load(const int32_t *lab, int x)
{
    return __hip_atomic_load(lab + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void lab_store(int32_t *lab, int x, int v)
{
    __hip_atomic_store(lab + x, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Local root of site e.  The entry of an ordinary site never changes during
// the global phase, and every value a local root's entry can hold decodes to
// the site itself, so a plain (possibly stale) load is exact.
__device__ __forceinline__ int endpoint_root(const int32_t *lab, int e)
{
    const int v = lab[e];
    return (v < 0 || (v & kTag) || v == e) ? e : v;
}

// Root of local root x in the forest while hooking runs (shortcuts store
// tagged grandparents, which are ancestors).
__device__ __forceinline__ int forest_find(int32_t *lab, int x)
{
    for (int it = 0; it < kWalkCap; ++it) {
        const int v = lab_load(lab, x);
        if (v == x) return x;
        const int p = v & kIdxMask;
        const int w = lab_load(lab, p);
        if (w != p) lab_store(lab, x, w);
        x = p;
    }
    return x;
}

__device__ __forceinline__ void forest_unite(int32_t *lab, int a, int b)
{
    for (int it = 0; it < kWalkCap; ++it) {
        a = forest_find(lab, a);
        b = forest_find(lab, b);
        if (a == b) return;
        if (link_priority(a) < link_priority(b)) {
            const int tmp = a;
            a = b;
            b = tmp;
        }
        const int old = atomicCAS(lab + a, a, kTag | b);
        if (old == a) return;
        a = old & kIdxMask;
    }
}


// Site `site` of the neighbour cell `code` (lattice.hpp codes) of the cell
// at (x, y, z); xm, ym, zm are the wrapped lower coordinates.  Bit 0/1/2 of
// the 3-bit field of a code says whether the neighbour is one cell lower in
// x/y/z.
__device__ __forceinline__ int nbr_site(int code, int site, int x, int y, int z, int xm, int ym, int zm, int L)
{
    constexpr uint32_t kLowerAxes = 0u | 1u << 3 | 2u << 6 | 4u << 9 | 6u << 12 | 5u << 15 | 3u << 18;
    const uint32_t mk = (kLowerAxes >> (3 * code)) & 7u;
    const int cx = (mk & 1u) ? xm : x, cy = (mk & 2u) ? ym : y, cz = (mk & 4u) ? zm : z;
    return 16 * ((cz * L + cy) * L + cx) + site;
}

// Visit the (local root, local root) pairs of the active crossing bonds owned
// by one face cell.
template <typename F>
__device__ __forceinline__ void for_cross_pairs(const RepDesc &d, int cell, uint64_t m, F &&f)
{
    const int L = d.L;
    const int x = cell % L, y = (cell / L) % L, z = cell / (L * L);
    const int xm = x == 0 ? L - 1 : x - 1, ym = y == 0 ? L - 1 : y - 1, zm = z == 0 ? L - 1 : z - 1;
    uint32_t down = (uint32_t)(m >> 24);
    while (down) {
        const int jj = __ffs(down) - 1;
        down &= down - 1;
        const uint32_t e = kDownEnds.v[jj];
        const int sa = nbr_site(e & 0xFF, (e >> 8) & 0xFF, x, y, z, xm, ym, zm, L);
        const int sb = nbr_site((e >> 16) & 0xFF, e >> 24, x, y, z, xm, ym, zm, L);
        f(endpoint_root(d.label, sa), endpoint_root(d.label, sb));
    }
}

// Root of local root x in the merged forest (no hooking runs any more); a
// root holds itself, or an encoded minimum once the minimum pass reached it.
__device__ __forceinline__ int merged_root(const int32_t *lab, int x)
{
    for (int it = 0; it < kWalkCap; ++it) {
        const int v = lab_load(lab, x);
        if (v == x || v < 0) return x;
        x = v & kIdxMask;
    }
    return x;
}

// Encoded canonical index of the cluster of local root x (after the
// minimum pass).  Only negative values are stored by the store pass, and
// walks stop at the first negative value, so no walk can loop.
__device__ __forceinline__ int encoded_canon(const int32_t *lab, int x)
{
    for (int it = 0; it < kWalkCap; ++it) {
        const int v = lab_load(lab, x);
        if (v < 0) return v;
        if (v == x) return kCanonBase + x;
        x = v & kIdxMask;
    }
    return kCanonBase + x;
}

// Canonical label (smallest site index of the cluster) of any site once the
// store pass is done: site -> local root -> itself or its encoding.
__device__ __forceinline__ int canonical_label(const int32_t *label, int64_t i)
{
    const int v = label[i];
    if (v < 0) return v - kCanonBase;
    const int r = v & kIdxMask;
    const int w = label[r];
    return w < 0 ? w - kCanonBase : (w & kIdxMask);
}

enum GlobalPass : int { kPassUnite = 0, kPassMin = 1, kPassStore = 2 };

// Per-tile list of the distinct (local root, local root) pairs joined by the
// tile's active crossing bonds, written by the unite pass for the two later
// passes: word 0 = count (or -1 when the list overflowed; the later passes
// then gather the pairs again), then `kPairCap` pairs (low, high).
constexpr int kPairCap = 256;
constexpr int kPairListInts = 1 + 2 * kPairCap;

// One workgroup per tile, three passes (three launches, each seeing the
// previous one complete):
//   kPassUnite  unite every distinct (root, root) pair in the global forest;
//   kPassMin    lower each merged root to the encoding of the smallest local
//               root of its cluster (= the smallest site of the cluster);
//   kPassStore  store that encoding in every local root of the cluster.
// The unite pass reads the labels of the tile's face cells and of the halo
// cells below them into LDS with row-coalesced loads, finds the local root
// of every crossing-bond endpoint there, and drops repeated pairs in an LDS
// hash set (a cluster usually crosses a face through many bonds but few
// local roots).  Items that do not fit the set are processed directly.
template <int TX, int TY, int TZ, int PASS>
__global__ __launch_bounds__(TX *TY *TZ) void k_global(Chain c)
{
    constexpr int NC = TX * TY * TZ;
    constexpr int EX = TX + 1, EY = TY + 1, EZ = TZ + 1, NE = EX * EY * EZ;  // tile + low halo
    constexpr int HASH = 1024;
    __shared__ unsigned long long H[HASH];
    __shared__ unsigned long long U[HASH];
    __shared__ int n_unique;
    __shared__ int LABS[PASS == kPassUnite ? 16 * NE : 1];
    const int rep = c.tile_rep[blockIdx.x];
    if (c.state[rep]->remaining <= 0) return;
    const RepDesc &d = c.desc[rep];
    const int tile = blockIdx.x - d.tile_base;
    const TileIdx<TX, TY, TZ> ti = TileIdx<TX, TY, TZ>::of(tile, d);
    const int tid = threadIdx.x;
    const int L = d.L;
    int32_t *lab = d.label;
    int *plist = d.pairs + (int64_t)tile * kPairListInts;
    for (int k = tid; k < HASH; k += NC) H[k] = ~0ull;
    if (tid == 0) n_unique = 0;

    const int x0 = ti.bx * TX, y0 = ti.by * TY, z0 = ti.bz * TZ;
    // extended-box coordinate of a neighbour coordinate (wrapped) on one axis
    auto ext = [&](int v, int v0, int nt) { return (nt > 1 && v == (v0 == 0 ? L - 1 : v0 - 1)) ? 0 : v - v0 + 1; };

    if (PASS == kPassUnite) {
        // labels of the face layer and the halo below it (interior cells are
        // never crossing-bond endpoints)
        for (int e = tid; e < NE; e += NC) {
            const int ex = e % EX, ey = (e / EX) % EY, ez = e / (EX * EY);
            if (ex > 1 && ey > 1 && ez > 1) continue;
            int gx = x0 + ex - 1, gy = y0 + ey - 1, gz = z0 + ez - 1;
            if (gx >= L || gy >= L || gz >= L) continue;  // beyond a ragged tile
            if (ex == 0 && d.ntx == 1) continue;          // no halo along a single-tile axis
            if (ey == 0 && d.nty == 1) continue;
            if (ez == 0 && d.ntz == 1) continue;
            if (gx < 0) gx += L;
            if (gy < 0) gy += L;
            if (gz < 0) gz += L;
            const int4 *src = reinterpret_cast<const int4 *>(lab + 16 * ((gz * L + gy) * L + gx));
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int4 v = src[q];
                LABS[(4 * q) * NE + e] = v.x;
                LABS[(4 * q + 1) * NE + e] = v.y;
                LABS[(4 * q + 2) * NE + e] = v.z;
                LABS[(4 * q + 3) * NE + e] = v.w;
            }
        }
    }
    __syncthreads();

    auto process = [&](unsigned long long key) {
        if (PASS == kPassUnite) {
            forest_unite(lab, (int)(key >> 32), (int)(key & 0xFFFFFFFFu));
        } else if (PASS == kPassMin) {
            const int r = (int)key;
            const int root = merged_root(lab, r);
            if (lab_load(lab, root) > kCanonBase + r) atomicMin(lab + root, kCanonBase + r);
        } else {
            const int r = (int)key;
            lab_store(lab, r, encoded_canon(lab, r));
        }
    };
    auto insert = [&](unsigned long long key) {
        uint32_t h = ((uint32_t)(key >> 32) * 0x9E3779B1u) ^ ((uint32_t)key * 0x85EBCA77u);
        h ^= h >> 15;
        for (int probe = 0; probe < 32; ++probe) {
            const int slot = (int)((h + (uint32_t)probe) & (HASH - 1));
            const unsigned long long prev = atomicCAS(&H[slot], ~0ull, key);
            if (prev == ~0ull) {
                U[atomicAdd(&n_unique, 1)] = key;
                return;
            }
            if (prev == key) return;
        }
        process(key);  // set too crowded: no deduplication for this item
    };
    auto add_pair = [&](int ra, int rb) {
        if (PASS == kPassUnite) {
            if (ra == rb) return;
            const int lo = ra < rb ? ra : rb, hi = ra < rb ? rb : ra;
            insert(((unsigned long long)(unsigned)lo << 32) | (unsigned)hi);
        } else {
            insert((unsigned)ra);
            if (rb != ra) insert((unsigned)rb);
        }
    };

    // Pairs of this tile: from the list of the unite pass when it fits,
    // otherwise from the crossing bonds themselves.
    const int listed = PASS == kPassUnite ? -1 : plist[0];
    if (listed >= 0) {
        for (int k = tid; k < listed; k += NC) add_pair(plist[1 + 2 * k], plist[2 + 2 * k]);
    } else {
        const int lx = tid % TX, ly = (tid / TX) % TY, lz = tid / (TX * TY);
        const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
        if (x < L && y < L && z < L && is_face_cell(lx, ly, lz, d)) {
            const int cell = (z * L + y) * L + x;
            const uint64_t m = d.xmask[cell];
            if (m) {
                if (PASS == kPassUnite) {
                    const int xm = x == 0 ? L - 1 : x - 1, ym = y == 0 ? L - 1 : y - 1, zm = z == 0 ? L - 1 : z - 1;
                    uint32_t down = (uint32_t)(m >> 24);
                    while (down) {
                        const int jj = __ffs(down) - 1;
                        down &= down - 1;
                        const uint32_t e = kDownEnds.v[jj];
                        int rts[2];
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            const uint32_t code = (e >> (16 * h)) & 0xFF, site = (e >> (16 * h + 8)) & 0xFF;
                            constexpr uint32_t kLowerAxes =
                                0u | 1u << 3 | 2u << 6 | 4u << 9 | 6u << 12 | 5u << 15 | 3u << 18;
                            const uint32_t mk = (kLowerAxes >> (3 * code)) & 7u;
                            const int cx = (mk & 1u) ? xm : x, cy = (mk & 2u) ? ym : y, cz = (mk & 4u) ? zm : z;
                            const int ecell = (ext(cz, z0, d.ntz) * EY + ext(cy, y0, d.nty)) * EX + ext(cx, x0, d.ntx);
                            const int v = LABS[site * NE + ecell];
                            const int gsite = 16 * ((cz * L + cy) * L + cx) + (int)site;
                            rts[h] = (v < 0 || (v & kTag) || v == gsite) ? gsite : v;
                        }
                        add_pair(rts[0], rts[1]);
                    }
                } else {
                    for_cross_pairs(d, cell, m, add_pair);
                }
            }
        }
    }
    __syncthreads();
    const int nu = n_unique;
    if (PASS == kPassUnite && tid == 0) plist[0] = nu <= kPairCap ? nu : -1;
    for (int k = tid; k < nu; k += NC) {
        const unsigned long long key = U[k];
        if (PASS == kPassUnite && nu <= kPairCap) {
            plist[1 + 2 * k] = (int)(key >> 32);
            plist[2 + 2 * k] = (int)(key & 0xFFFFFFFFu);
        }
        process(key);
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
