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
// c of the tile, site k), whose order follows the global site order.  Node
// key sits at slot key + c = 17 c + k of the forest array: the slot order is
// the key order, and the 16 nodes of consecutive cells, which the lanes of a
// wave touch together, are 17 words apart and so never share an LDS bank.
// Each entry holds the byte offset (4 x slot) of its parent, so a step of a
// walk is one load with no index arithmetic.
template <int NC>
constexpr int kForestSlots = 17 * NC;

__device__ __forceinline__ uint32_t node_off(int key)
{
    return 4u * (uint32_t)(key + (key >> 4));
}

// Key of the node at byte offset off: slot - slot / 17, the quotient by a
// 24-bit multiply and shift (exact for every slot below 2^16).
__device__ __forceinline__ int node_key(uint32_t off)
{
    const uint32_t slot = off >> 2, c = __umul24(slot, 61681u) >> 20;
    return (int)(slot - c);
}

// Entry at byte offset off of the forest array, addressed in the LDS
// address space (a 32-bit offset, no generic-pointer arithmetic).
typedef __attribute__((address_space(3))) volatile uint32_t lds_word;
typedef __attribute__((address_space(3))) volatile char lds_byte;

__device__ __forceinline__ lds_word &node(volatile uint32_t *P, uint32_t off)
{
    return *(lds_word *)((lds_byte *)P + off);
}

// Every walk in the global forest below is capped far above any reachable
// depth (a forest over n nodes has depth below n), so a damaged forest can
// only give a wrong label, never a kernel that does not finish.
constexpr int kWalkCap = 1 << 22;

// In the tile forest a parent's offset is never above its child's (roots
// hold their own offset): initial parents are the smallest vertex of an up
// tetrahedron's component, unions lower a root to a smaller one, and path
// splitting stores ancestors.  Walks therefore step only while the parent is
// strictly smaller, which bounds them by the forest size whatever the
// entries hold.

// Root of node x (byte offsets), with path splitting.  The store is
// unconditional: x is not a root, and any ancestor is a valid parent.
__device__ __forceinline__ uint32_t lds_find(volatile uint32_t *P, uint32_t x)
{
    uint32_t p = node(P, x);
    while (p < x) {
        const uint32_t gp = node(P, p);
        node(P, x) = gp;
        x = p;
        p = gp;
    }
    return x;
}

// Union in an LDS forest: the larger root is lowered to the smaller one with
// atomicMin; if it had been re-parented meanwhile (to a smaller node),
// continue from there.  The larger root strictly decreases on every retry.
__device__ __forceinline__ void lds_unite(uint32_t *P, uint32_t a, uint32_t b)
{
    volatile uint32_t *V = P;
    for (;;) {
        a = lds_find(V, a);
        b = lds_find(V, b);
        if (a == b) return;
        if (a < b) {
            const uint32_t tmp = a;
            a = b;
            b = tmp;
        }
        const uint32_t old = __hip_atomic_fetch_min((__attribute__((address_space(3))) uint32_t *)((lds_byte *)P + a), b,
                                                    __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (old >= a) return;
        a = old;
    }
}

// Label staging of the flip kernels: the label of local key 16 c + k is kept
// at k * NC + c, so the lanes of a wave, which own consecutive cells, touch
// consecutive LDS banks.
template <int NC>
__device__ __forceinline__ int lds_pos(int key)
{
    return (int)(((unsigned)key & 15u) * NC + ((unsigned)key >> 4));
}

struct NbrCell {
    int gcell;  // global cell index
    int lcell;  // local cell index in the tile, or -1 if outside
};

// Quotient a / b for 0 <= a < 2^24 and b >= 1 with a small quotient: a
// float reciprocal gives it to within one, an integer check corrects it.
__device__ __forceinline__ int small_div(int a, int b, float inv_b)
{
    int q = (int)((float)a * inv_b);
    if (mul24(q, b) > a) --q;
    else if (mul24(q + 1, b) <= a) ++q;
    return q;
}

template <int TX, int TY, int TZ>
struct TileIdx {
    int L, bx, by, bz;
    int base;            // global index of the tile's first cell
    float inv_L, inv_LL; // 1/L and 1/L^2

    __device__ __forceinline__ static TileIdx of(int tile, const RepDesc &d)
    {
        TileIdx t;
        t.L = d.L;
        t.bx = tile % d.ntx;
        tile /= d.ntx;
        t.by = tile % d.nty;
        t.bz = tile / d.nty;
        t.base = ((t.bz * TZ) * t.L + t.by * TY) * t.L + t.bx * TX;
        t.inv_L = 1.0f / (float)t.L;
        t.inv_LL = 1.0f / (float)(t.L * t.L);
        return t;
    }
    __device__ __forceinline__ NbrCell at(int x, int y, int z) const
    {
        NbrCell c;
        c.gcell = cell_index(x, y, z, L);
        const int tx = x - bx * TX, ty = y - by * TY, tz = z - bz * TZ;
        const bool in = (unsigned)tx < (unsigned)TX && (unsigned)ty < (unsigned)TY && (unsigned)tz < (unsigned)TZ;
        c.lcell = in ? (tz * TY + ty) * TX + tx : -1;
        return c;
    }
    // Global site index of the first site of local row `row` = lz TY + ly of
    // the tile (its cells x = bx TX .. bx TX + TX - 1 are consecutive).
    __device__ __forceinline__ int row_base(int row) const
    {
        const int lz = row / TY, ly = row % TY;
        return 16 * (base + mul24(mul24(lz, L) + ly, L));
    }
    // Global site index of local key l = 16 c + k.
    __device__ __forceinline__ int global_site(int l) const
    {
        const unsigned lc = (unsigned)l >> 4;  // keys are non-negative; unsigned keeps % and / to masks and shifts
        const int lx = (int)(lc % TX), ly = (int)((lc / TX) % TY), lz = (int)(lc / (TX * TY));
        return 16 * (base + cell_index(lx, ly, lz, L)) + (l & 15);
    }
    // Local key 16 c + k of a global site index known to lie in this tile
    // (offsets from the tile's first cell are below TZ L^2 < 2^24).
    __device__ __forceinline__ int local_key(int site) const
    {
        const int off = (site >> 4) - base;
        const int LL = L * L;
        const int lz = small_div(off, LL, inv_LL);
        const int rem = off - mul24(lz, LL);
        const int ly = small_div(rem, L, inv_L);
        const int lx = rem - mul24(ly, L);
        return 16 * ((lz * TY + ly) * TX + lx) + (site & 15);
    }
    // Local key of a site of this tile from the thread's own cell (global
    // index `cell`, local index `lcell`): the cell offset dc = dz L^2 + dy L
    // + dx has |dx| < TX, |dy| < TY, |dz| < TZ, so when L >= 2 max(TX, TY,
    // TZ) (near_decodable) dz and dy are the nearest integers of dc / L^2 and
    // of the remainder / L (each more than 0.03 away from a half-integer).
    __device__ __forceinline__ bool near_decodable() const { return L >= 2 * (TX > TY ? (TX > TZ ? TX : TZ) : (TY > TZ ? TY : TZ)); }
    __device__ __forceinline__ int local_key_near(int site, int cell, int lcell) const
    {
        const int dc = (site >> 4) - cell;
        const int dz = (int)rintf((float)dc * inv_LL);
        const int r1 = dc - __mul24(dz, L * L);
        const int dy = (int)rintf((float)r1 * inv_L);
        const int dx = r1 - __mul24(dy, L);
        return 16 * (lcell + dx + dy * TX + dz * (TX * TY)) + (site & 15);
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

// ---------------------------------------------------------------- merge ---
// The global forest lives in the label entries of tile-local roots (the
// entries of ordinary sites keep pointing at their local root).  Entry
// encodings of a local root r:
//   r                   r is a root of the merged forest
//   kTag | p            r was hooked under p
//   kCanonBase + c (| kCoinBit)  written by the settle step of the flip
//                       kernels (or the persistent kernel's store phase): c is
//                       the smallest site index of r's cluster, and kCoinBit
//                       is set when that cluster flips in this sweep
// Site indices are below 2^30 (L <= 406), so the three forms are distinct and
// the local root of any site is decodable at any time, even while other
// threads hook roots or store canonical labels: an entry that is negative,
// tagged or equal to the site's own index names the site itself.
//
// A root is always hooked under the smaller of the two roots, so every tree
// root is the smallest local root of its tree, i.e. the smallest site of
// its cluster, and settling a hooked local root only has to copy it (with
// its coin) into the root's entry.  The unite pass hooks each tile's group
// of roots under its smallest member in one step, which keeps the trees
// shallow.
constexpr int kTag = 1 << 30;
constexpr int kIdxMask = kTag - 1;
constexpr int kCanonBase = INT32_MIN;  // canonical index c is stored as kCanonBase + c
constexpr int kCoinBit = 1 << 30;      // flip coin of the cluster, in a stored encoding

// Flip coin of the cluster whose smallest site is r in sweep t: bit (r mod
// 32) of word ((r/32) mod 4) of FLIP(r/128).
__device__ __forceinline__ uint32_t cluster_coin(int r, uint32_t t, PhiloxKey key)
{
    const uint4 w = philox4x32_10((uint32_t)r >> 7, t, kStreamFlip, 0u, key);
    return (word_of(w, ((uint32_t)r >> 5) & 3u) >> (r & 31)) & 1u;
}

// The coins of the 16 sites of a cell (bit k = site 16 cell + k) in sweep t:
// sites of one cell are 16 consecutive bits of one word of FLIP(cell/8).
__device__ __forceinline__ uint32_t cell_coins(int cell, uint32_t t, PhiloxKey key)
{
    const uint4 w = philox4x32_10((uint32_t)cell >> 3, t, kStreamFlip, 0u, key);
    return (word_of(w, ((uint32_t)cell >> 1) & 3u) >> (16 * (cell & 1))) & 0xFFFFu;
}

// Forest entries are read and written with relaxed workgroup-scope atomics,
// which the caches may serve stale within a launch (agent-scope loads would
// go past the per-XCD L2 on every step of every walk).  A stale value is an
// older value of the same entry, and every value an entry ever holds is an
// ancestor of the node in the final forest (hooks link roots, shortcuts
// store ancestors, the settle step writes only encodings that end a walk),
// so a stale walk is only longer, never wrong; the updates that decide the
// forest (hook CAS) are device-wide atomics and return the current value.  Launch boundaries make all writes visible.
__device__ __forceinline__ int lab_load(const int32_t *lab, int x)
{
    return __hip_atomic_load(lab + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void lab_store(int32_t *lab, int x, int v)
{
    __hip_atomic_store(lab + x, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
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

// Union of the trees of local roots a and b.  Every parent is smaller than
// its child (hooks put the larger root under a smaller node, shortcuts store
// ancestors), so a root may be hooked under any node smaller than itself:
// that node cannot lie in the root's own tree.  Hence a's root is walked
// first and, when it is larger than b, hooked under b by CAS without walking
// b; otherwise b's root is walked and the larger of the two roots is hooked
// under the smaller.  A lost CAS continues from the value it returned.
template <bool COUNT = false>
__device__ __forceinline__ void forest_unite(int32_t *lab, int a, int b, unsigned long long *counts)
{
    for (int it = 0; it < kWalkCap; ++it) {
        a = forest_find(lab, a);
        if (a == b) return;
        if (a < b) {
            b = forest_find(lab, b);
            if (a == b) return;
            if (a < b) {
                const int tmp = a;
                a = b;
                b = tmp;
            }
        }
        const int old = atomicCAS(lab + a, a, kTag | b);
        if (COUNT) {  // measurement runs only (a kernel of its own)
            atomicAdd(&counts[0], 1ull);
            if (old == a) atomicAdd(&counts[1], 1ull);
        }
        if (old == a) return;
        a = old & kIdxMask;
    }
}

// Tree root of local root x after the unite pass, or the first encoding a
// settle step has already written on the way (a negative value).  The tree
// root's index is the cluster's smallest site.
__device__ __forceinline__ int root_or_encoding(const int32_t *lab, int x)
{
    for (int it = 0; it < kWalkCap; ++it) {
        const int v = lab_load(lab, x);
        if (v < 0 || v == x) return v;
        x = v & kIdxMask;
    }
    return x;
}

// Encoding stored for the cluster of local root x in sweep t: its smallest
// site and its flip coin.
__device__ __forceinline__ int canon_encoding(const int32_t *lab, int x, uint32_t t, PhiloxKey key)
{
    const int v = root_or_encoding(lab, x);
    if (v < 0) return v;
    return kCanonBase + v + (int)(cluster_coin(v, t, key) << 30);
}

// Canonical label (smallest site index of the cluster) of any site once the
// sweep is done: site -> local root -> itself (a tree root) or its settled
// encoding (a walk from a still-hooked local root is kept as a safeguard).
__device__ __forceinline__ int canonical_label(const int32_t *label, int64_t i)
{
    const int v = label[i];
    if (v < 0) return v & kIdxMask;
    const int r = (v & kTag) ? (int)i : v;
    const int w = label[r];
    if (w < 0) return w & kIdxMask;
    if (w & kTag) {
        const int e = root_or_encoding(label, r);
        return e < 0 ? (e & kIdxMask) : e;
    }
    return r;
}

// Flip mask (bit k = site k) of the cell of a flip kernel's thread, from the
// labels of its 16 sites (lab), the tile's labels staged in LDS (LAB, laid
// out by lds_pos) and the coins of the tile's own sites (CB, one 16-bit word
// per cell).  A site's label is its tile-local root r; r's entry holds the
// stored encoding (canonical site and coin) when r's cluster leaves the tile,
// else r itself, whose coin is the tile's.  Only LDS is read.
template <int NC, int TX, int TY, int TZ>
__device__ __forceinline__ uint32_t cell_flip_mask(const int (&lab)[16], const int *LAB, const uint32_t *CB,
                                                  const TileIdx<TX, TY, TZ> &ti, int cell, int lcell, uint32_t t,
                                                  PhiloxKey key)
{
    const bool near = ti.near_decodable();  // uniform
    int last_in = -1;
    uint32_t last_coin = 0, mask = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int r0 = lab[k];  // tile-local root, or an encoding (the site is a merged local root)
        uint32_t coin;
        if (r0 < 0) {
            coin = ((uint32_t)r0 >> 30) & 1u;
        } else if (r0 & kTag) {
            coin = cluster_coin(r0 & kIdxMask, t, key);  // not produced by a complete sweep; kept in range
        } else if (r0 == last_in) {
            coin = last_coin;
        } else {
            const int key16 = near ? ti.local_key_near(r0, cell, lcell) : ti.local_key(r0);
            const int v = LAB[lds_pos<NC>(key16)];
            if (v < 0) coin = ((uint32_t)v >> 30) & 1u;
            else if (v & kTag) coin = cluster_coin(v & kIdxMask, t, key);  // as above
            else coin = (CB[key16 >> 4] >> (key16 & 15)) & 1u;
            last_in = r0;
            last_coin = coin;
        }
        mask |= coin << k;
    }
    return mask;
}

constexpr int const_log2(int v) { return v <= 1 ? 0 : 1 + const_log2(v >> 1); }

// Aligned tiling: the lattice edge is L = 2^lg and every tile edge divides
// it, so each tile starts at a multiple of its edges and a site index
// 16 (x + L y + L^2 z) + k of the tile has its local cell coordinates in
// fixed bit fields.  The local key 16 (lx + TX ly + TX TY lz) + k is then
// a few bit-field extracts, whatever value is decoded (an encoding yields
// some key of the tile, never one outside it).
template <int TX, int TY, int TZ>
__device__ __forceinline__ int aligned_local_key(int site, int lg)
{
    constexpr int lTX = const_log2(TX), lTY = const_log2(TY);
    const uint32_t u = (uint32_t)site;
    const uint32_t ly = __builtin_amdgcn_ubfe(u, (uint32_t)(4 + lg), (uint32_t)const_log2(TY));
    const uint32_t lz = __builtin_amdgcn_ubfe(u, (uint32_t)(4 + 2 * lg), (uint32_t)const_log2(TZ));
    return (int)((u & (16u * TX - 1u)) | (ly << (4 + lTX)) | (lz << (4 + lTX + lTY)));
}

// How a flip kernel finds a site's local root in its tile: kFlipGeneral
// stages the labels at lds_pos and decodes with branches (cell_flip_mask);
// the keyed modes stage them by local key and decode without a branch, for
// tilings whose tile edges divide L (every thread has a cell, TX >= 8): by
// bit fields when L is a power of two (kFlipPow2, aligned_local_key), else
// by rounding the cell offset (kFlipDivisible, TileIdx::local_key_near,
// exact for L >= 2 x the largest tile edge).
enum FlipMode : int { kFlipGeneral = 0, kFlipPow2 = 1, kFlipDivisible = 2 };

// Flip mask of a flip kernel's cell for a keyed mode.  LAB holds the
// tile's labels by local key; CB holds the coin words of the tile's cells,
// two cells per word as the flip stream draws them (bit (key & 31) of word
// key >> 5 is the coin of local key `key`).  The same rule as
// cell_flip_mask: a stored encoding, in the site's own entry or in its
// local root's, gives the coin; otherwise the local root's own coin.  No
// branch: both LDS words are read for every site, and the key decoded from
// an encoding, which is not used, is masked into the tile's key range.
template <int TX, int TY, int TZ, int MODE>
__device__ __forceinline__ uint32_t cell_flip_mask_keyed(const int (&lab)[16], const int *LAB, const uint32_t *CB,
                                                        int lg, const TileIdx<TX, TY, TZ> &ti, int cell, int lcell)
{
    constexpr int NC = TX * TY * TZ;
    static_assert(MODE == kFlipPow2 || MODE == kFlipDivisible, "a keyed mode");
    static_assert((NC & (NC - 1)) == 0, "tile keys fill a power of two");
    uint32_t mask = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int r = lab[k];
        const int key = MODE == kFlipPow2 ? aligned_local_key<TX, TY, TZ>(r, lg)
                                          : (ti.local_key_near(r, cell, lcell) & (16 * NC - 1));
        const int u = r < 0 ? r : LAB[key];
        const bool enc = u < 0;
        const uint32_t word = enc ? (uint32_t)u : CB[key >> 5];
        mask |= __builtin_amdgcn_ubfe(word, enc ? 30u : (uint32_t)key & 31u, 1u) << k;
    }
    return mask;
}

// Coin words of a keyed tile (NC / 8 threads, thread j): local cells
// 8j .. 8j + 7 are eight consecutive cells of one x row starting at a
// multiple of 8 (TX >= 8), i.e. exactly the cells of one FLIP block, whose
// four words cover two cells each (cell_coins).
template <int TX, int TY, int TZ>
__device__ __forceinline__ uint4 aligned_coin_words(const TileIdx<TX, TY, TZ> &ti, int j, uint32_t t, PhiloxKey key)
{
    static_assert(TX % 8 == 0, "a FLIP block is 8 cells of one x row");
    const int c0 = 8 * j;
    const int gcell = cell_index(ti.bx * TX + c0 % TX, ti.by * TY + (c0 / TX) % TY, ti.bz * TZ + c0 / (TX * TY), ti.L);
    return philox4x32_10((uint32_t)gcell >> 3, t, kStreamFlip, 0u, key);
}

// ------------------------------------------------------- settle step ---
// The flip kernels settle their tile's own hooked local roots (entries
// kTag | p) once every unite is done: the walk from p ends at the
// cluster's tree root, its smallest site, or at an encoding that another
// settle wrote on the way, and the root's entry becomes the stored encoding
// (smallest site and coin) in the label array, for later walks and the
// host's labels, and in the LDS copy of the tile's labels.  A local root
// that is a tree root keeps its own index: its cluster's coin is the
// tile's own coin of that site (the same bit of the same FLIP word).  Only
// a root's own tile settles it, so no other workgroup changes an entry a
// tile has staged.
constexpr int kSettleListPerCell = 4;  // list room per cell; roots beyond it settle in place

// Loads the 16 labels of a flip kernel's cell into lab and copies them into
// LAB (by local key in a keyed FlipMode, else at lds_pos).  Returns the
// mask of the sites that are hooked local roots; their lab value becomes
// the site's own index, so that the flip reads the site's settled entry.
template <int NC, bool ALIGNED>
__device__ __forceinline__ uint32_t stage_cell_labels(const int32_t *label, int cell, int tid, int (&lab)[16], int *LAB)
{
    const int4 *L4 = reinterpret_cast<const int4 *>(label + 16 * cell);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int4 v = L4[q];
        if (ALIGNED) reinterpret_cast<int4 *>(LAB)[4 * tid + q] = v;
        lab[4 * q] = v.x;
        lab[4 * q + 1] = v.y;
        lab[4 * q + 2] = v.z;
        lab[4 * q + 3] = v.w;
    }
    uint32_t hm = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (!ALIGNED) LAB[k * NC + tid] = lab[k];
        const bool hooked = ((uint32_t)lab[k] >> 30) == 1u;  // kTag | p
        hm |= (uint32_t)hooked << k;
        lab[k] = hooked ? 16 * cell + k : lab[k];
    }
    return hm;
}

// The settle step of a flip kernel (all NC threads of the tile, after
// stage_cell_labels; hm is the thread's mask, 0 for a thread without a
// cell).  The hooked roots are listed in HL (kSettleListPerCell NC
// entries; the list places follow the threads' counts, by five ballots
// and the wave totals in wtot, NC / 64 ints) and settled by all threads.
template <int TX, int TY, int TZ, bool ALIGNED>
__device__ __forceinline__ void settle_tile_roots(const RepDesc &d, const RepState &st, const TileIdx<TX, TY, TZ> &ti,
                                                  int tid, int cell, uint32_t hm, int *LAB, uint16_t *HL, int *wtot)
{
    constexpr int NC = TX * TY * TZ;
    constexpr int kCapHL = kSettleListPerCell * NC;
    static_assert(16 * NC <= 65536, "local keys fit 16 bits");
    auto pos = [](int key) { return ALIGNED ? key : lds_pos<NC>(key); };
    const uint32_t cnt = (uint32_t)__popc(hm);
    uint32_t below = 0, wt = 0;
#pragma unroll
    for (int bit = 0; bit < 5; ++bit) {
        const uint64_t b = __ballot((cnt >> bit) & 1u);
        below += __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u)) << bit;
        wt += (uint32_t)__popcll(b) << bit;
    }
    const int wave = tid >> 6;
    if ((tid & 63) == 0) wtot[wave] = (int)wt;
    __syncthreads();
    int at = (int)below, nh = 0;
    for (int w = 0; w < NC / 64; ++w) {
        const int t = wtot[w];
        at += w < wave ? t : 0;
        nh += t;
    }
    if (hm) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            if (!((hm >> k) & 1u)) continue;
            const int key = 16 * tid + k;
            if (at < kCapHL) {
                HL[at] = (uint16_t)key;
            } else {  // beyond the list: settled by the thread that found it
                const int e = canon_encoding(d.label, LAB[pos(key)] & kIdxMask, st.t, d.key);
                lab_store(d.label, 16 * cell + k, e);
                LAB[pos(key)] = e;
            }
            ++at;
        }
    }
    __syncthreads();
    const int nl = min(nh, kCapHL);
    for (int j = tid; j < nl; j += NC) {
        const int key = HL[j];
        const int e = canon_encoding(d.label, LAB[pos(key)] & kIdxMask, st.t, d.key);
        lab_store(d.label, ti.global_site(key), e);
        LAB[pos(key)] = e;
    }
    __syncthreads();
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
    return 16 * cell_index(cx, cy, cz, L) + site;
}

// Local root of site e (a plain, possibly stale load is exact: the entry of
// an ordinary site does not change during the global phase, and any value a
// local root's entry takes decodes to the root itself).
__device__ __forceinline__ int endpoint_root(const int32_t *lab, int e)
{
    const int v = lab[e];
    return (v < 0 || (v & kTag) || v == e) ? e : v;
}

// Local root named by a crossing-list entry: a tagged name is a local root
// already; a site index is looked up (endpoint_root).
__device__ __forceinline__ int name_root(const int32_t *lab, int name)
{
    return (name & kTag) ? (name & kIdxMask) : endpoint_root(lab, name);
}

// Crossing-pair emission items of a tile shape: one per (low-face cell c,
// down tetrahedron f) whose tetrahedron can have a vertex outside the tile
// (f = 0 on every low face, f = 1/2/3 on the face x/y/z = 0), packed as
// 4 c + f and sorted by f, so the lanes of a wave mostly share f.  Whether a
// vertex is outside is decided at run time (an axis with a single tile
// wraps onto itself).
template <int TX, int TY, int TZ>
struct EmitItems {
    uint16_t v[4 * TX * TY * TZ];
    int n;
};
template <int TX, int TY, int TZ>
__host__ __device__ constexpr EmitItems<TX, TY, TZ> make_emit_items()
{
    EmitItems<TX, TY, TZ> t{};
    t.n = 0;
    for (int f = 0; f < 4; ++f)
        for (int c = 0; c < TX * TY * TZ; ++c) {
            const bool fx = c % TX == 0, fy = (c / TX) % TY == 0, fz = c / (TX * TY) == 0;
            const bool use = f == 0 ? (fx || fy || fz) : (f == 1 ? fx : (f == 2 ? fy : fz));
            if (use) t.v[t.n++] = (uint16_t)(4 * c + f);
        }
    return t;
}
template <int TX, int TY, int TZ>
__constant__ EmitItems<TX, TY, TZ> kEmitItems = make_emit_items<TX, TY, TZ>();

// Vertex mu of down tetrahedron f as (cell code << 4 | site), byte 4 f + mu.
__host__ __device__ constexpr uint64_t down_vertex_bytes(int half)
{
    uint64_t w = 0;
    for (int k = 0; k < 8; ++k) {
        const SiteRef R = down_vertex(2 * half + k / 4, k % 4);
        w |= (uint64_t)(R.cell << 4 | R.site) << (8 * k);
    }
    return w;
}

// ------------------------------------------------------ tile components ---
// Union-list entries per cell of a tile of NC cells (the UPC argument of
// tile_components); unions beyond the list are done by the thread that
// found them.  The Ising tile pass keeps one entry per cell for tiles of
// 512 cells or more: the smaller list lets four 8x8x8 tile workgroups share
// a CU's LDS instead of three, which pays more than the balance of a longer
// list (tile pass 598 -> 569 us per launch over five L = 128 lattices).
// Its smaller tiles keep eight (one per cell made L = 48 sweeps with 8x8x4
// tiles 3-4% slower), and so does the O(n) tile pass, whose 8x8x8 tiles
// were 3-4% slower with one.
template <int NC>
constexpr int kIsingUnionsPerCell = NC >= 512 ? 1 : 8;
constexpr int kOnUnionsPerCell = 8;

// Second half of both models' tile pass (every thread of the block calls
// it; `act` is 0 for threads without a cell, lc[] holds the local index of
// each neighbour cell of the thread's cell, or -1 outside the tile; DA is
// LDS for one word per cell): the components of the tile's sites from the
// active bonds of its cells, written as every site's tile-local root, and
// the tile's crossing list.
//
// Inside the tile, each down tetrahedron contributes the spanning edges of
// the components of its active bonds whose two ends lie in the tile (at most
// 3, from the K4 table); all threads then process the tile's list of such
// unions evenly, so one busy cell does not hold up its wave.
//
// Every site is a vertex of exactly one down tetrahedron, owned by one cell,
// so the crossing bonds of different cells never join the same pair of
// sites.  For each down tetrahedron with a vertex outside the tile, each
// vertex is named by its tile-local root with the tag bit set (inside) or
// by its site index (outside), and per component of the tetrahedron's
// active bonds the edges from the component's smallest vertex to the others
// whose name differs are emitted: at most 3 pairs per tetrahedron, none
// repeated.  These tetrahedra belong to the cells of the low faces; they
// are handed out to all threads as a table of (cell, tetrahedron) items.
template <int TX, int TY, int TZ, int UPC>
__device__ __forceinline__ void tile_components(const RepDesc &d, const TileIdx<TX, TY, TZ> &ti, int tile, int tid,
                                                int lcid, bool valid, int cell, uint64_t act,
                                                const int (&lc)[kNCellCodes], uint32_t *P, uint32_t *U, uint32_t *DA,
                                                const uint8_t *K4)
{
    constexpr int NC = TX * TY * TZ;
    static_assert(NC % 64 == 0, "tiles are whole waves");
    constexpr int kCap = UPC * NC - NC / 64;  // union list; its wave totals follow it in U
    uint32_t *WT = U + kCap;
    // local key of vertex mu of down tetrahedron f (-1 when outside the tile)
    auto vkey = [&](int f, int mu) {
        const SiteRef R = down_vertex(f, mu);
        const int l = R.cell == kSelf ? lcid : lc[R.cell];
        return l >= 0 ? 16 * l + R.site : -1;
    };
    // Up tetrahedra: components from the table, roots at the smallest vertex.
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const uint32_t code = K4[(uint32_t)(act >> (6 * f)) & 63u];
        const uint32_t base = node_off(16 * lcid + 4 * f);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) node(P, base + 4 * mu) = base + 4 * ((code >> (2 * mu)) & 3);
    }
    // No barrier here: the down tetrahedra below read only registers and K4,
    // and the forest is first read after the barrier of the list placement.
    // Down tetrahedra, inside the tile: spanning edges, packed as two 16-bit
    // forest slots (17 NC < 2^16).
    uint32_t un[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) un[k] = 0xFFFFFFFFu;  // no union (also for threads without a cell)
    unsigned nun = 0;
    if (valid) {
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const int k0 = vkey(f, 0), k1 = vkey(f, 1), k2 = vkey(f, 2), k3 = vkey(f, 3);
            uint32_t inside = 0;  // bonds with both ends in the tile
#pragma unroll
            for (int e = 0; e < 6; ++e) {
                const int a = pair_a(e), b = pair_b(e);
                const int ka = a == 0 ? k0 : (a == 1 ? k1 : k2), kb = b == 1 ? k1 : (b == 2 ? k2 : k3);
                inside |= (uint32_t)(ka >= 0 && kb >= 0) << e;
            }
            const uint32_t code = K4[(uint32_t)(act >> (24 + 6 * f)) & inside];
#pragma unroll
            for (int mu = 1; mu < 4; ++mu) {
                const int rp = (code >> (2 * mu)) & 3;
                const int kr = rp == 0 ? k0 : (rp == 1 ? k1 : k2);
                const int km = mu == 1 ? k1 : (mu == 2 ? k2 : k3);
                const bool use = rp != mu;
                un[3 * f + mu - 1] = use ? (node_off(kr) << 14 | node_off(km) >> 2) : 0xFFFFFFFFu;
                nun += use;
            }
        }
    }
    // The thread's unions go after those of the lanes below it (four ballots
    // of its 0..12 count) and of the lower waves (totals in WT, past the
    // list's room in U; DA may still be read by a slower thread's bond
    // activation, which is why it does not hold them).
    uint32_t below = 0, wtot = 0;
#pragma unroll
    for (int bit = 0; bit < 4; ++bit) {
        const uint64_t b = __ballot((nun >> bit) & 1u);
        below += __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u)) << bit;
        wtot += (uint32_t)__popcll(b) << bit;
    }
    const int wave = tid >> 6;
    if ((tid & 63) == 0) WT[wave] = wtot;
    __syncthreads();
    int ntotal = 0;
    unsigned at = below;
    for (int w = 0; w < NC / 64; ++w) {
        const int t = (int)WT[w];
        at += w < wave ? t : 0;
        ntotal += t;
    }
    if (nun) {
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            if (un[k] == 0xFFFFFFFFu) continue;
            if (at < (unsigned)kCap) U[at] = un[k];
            else lds_unite(P, (un[k] >> 14) & ~3u, (un[k] & 0xFFFFu) << 2);
            ++at;
        }
    }
    __syncthreads();
    // Each thread takes a contiguous run of the list: a cell's unions sit
    // together in it, so the lanes of a wave work on different cells' roots.
    {
        const int nlist = min(ntotal, kCap);
        const int per = (nlist + NC - 1) / NC;
        const int kb = min(tid * per, nlist), ke = min(kb + per, nlist);
        for (int k = kb; k < ke; ++k) lds_unite(P, (U[k] >> 14) & ~3u, (U[k] & 0xFFFFu) << 2);
    }
    __syncthreads();
    // Tile-local roots of the thread's sites, as global site indices: into
    // the labels, and into the forest entries, where the emission below
    // reads the root of any site of the tile.  A key's global index is the
    // base of its row (a table in U, free after the unions) plus its offset
    // in the row, 16 lx + k.
    static_assert((TX & (TX - 1)) == 0 && TX * TY * TZ <= 1024, "power-of-two rows");
    constexpr int kRowShift = 4 + (TX == 4 ? 2 : (TX == 8 ? 3 : 4));
    for (int row = tid; row < TY * TZ; row += NC) U[row] = (uint32_t)ti.row_base(row);
    int r[16];
    if (valid) {
        const uint32_t base = node_off(16 * lcid);
#pragma unroll
        for (int k = 0; k < 16; ++k) r[k] = node_key(lds_find(P, base + 4 * k));
    }
    __syncthreads();
    if (valid) {
        const uint32_t base = node_off(16 * lcid);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            r[k] = (int)U[(uint32_t)r[k] >> kRowShift] + (r[k] & (16 * TX - 1));
            node(P, base + 4 * k) = (uint32_t)r[k];
        }
        int4 *out = reinterpret_cast<int4 *>(d.label + 16 * cell);
#pragma unroll
        for (int q = 0; q < 4; ++q) out[q] = make_int4(r[4 * q], r[4 * q + 1], r[4 * q + 2], r[4 * q + 3]);
    }
    DA[lcid] = (uint32_t)(act >> 24);  // active bonds of the cell's down tetrahedra
    __syncthreads();
    // Crossing pairs, one item (cell, down tetrahedron) per thread and round.
    // Each round places its pairs in item order: a lane's offset is the
    // number of pairs of the lanes below it (two ballots of the 0..3 pair
    // count), plus the totals of the lower waves, kept in U (free by now).
    const int L = d.L;
    int2 *list = reinterpret_cast<int2 *>(d.pairs + (int64_t)tile * d.list_stride) + 1;
    constexpr uint64_t kVert0 = down_vertex_bytes(0), kVert1 = down_vertex_bytes(1);
    constexpr uint32_t kLowerAxes = 0u | 1u << 3 | 2u << 6 | 4u << 9 | 6u << 12 | 5u << 15 | 3u << 18;
    constexpr int kItems = make_emit_items<TX, TY, TZ>().n;
    int placed = 0;  // pairs listed so far (the same in every thread)
    for (int jb = 0; jb < kItems; jb += NC) {
        const int j = jb + tid;
        int2 q[3];
        bool e[3] = {false, false, false};
        if (j < kItems) {
            const int item = kEmitItems<TX, TY, TZ>.v[j];
            const int c = item >> 2, f = item & 3;
            const int ix = c % TX, iy = (c / TX) % TY, iz = c / (TX * TY);
            const int cx = ti.bx * TX + ix, cy = ti.by * TY + iy, cz = ti.bz * TZ + iz;
            if (cx < L && cy < L && cz < L) {
                const int xm = cx == 0 ? L - 1 : cx - 1, ym = cy == 0 ? L - 1 : cy - 1, zm = cz == 0 ? L - 1 : cz - 1;
                const uint64_t vb = (f < 2) ? kVert0 : kVert1;
                bool outside = false;
                int id[4];
#pragma unroll
                for (int mu = 0; mu < 4; ++mu) {
                    const uint32_t v = (uint32_t)(vb >> (8 * (4 * (f & 1) + mu))) & 0xFFu;
                    const int code = (int)(v >> 4), site = (int)(v & 15u);
                    const uint32_t mk = (kLowerAxes >> (3 * code)) & 7u;
                    const int nx = (mk & 1u) ? xm : cx, ny = (mk & 2u) ? ym : cy, nz = (mk & 4u) ? zm : cz;
                    const NbrCell nb = ti.at(nx, ny, nz);
                    if (nb.lcell >= 0) {
                        id[mu] = (int)node(P, node_off(16 * nb.lcell + site)) | kTag;
                    } else {
                        id[mu] = 16 * nb.gcell + site;
                        outside = true;
                    }
                }
                if (outside) {
                    const uint32_t code = K4[(DA[c] >> (6 * f)) & 63u];
#pragma unroll
                    for (int mu = 1; mu < 4; ++mu) {
                        const int rp = (code >> (2 * mu)) & 3;
                        const int rid = rp == 0 ? id[0] : (rp == 1 ? id[1] : id[2]);
                        e[mu - 1] = rp != mu && rid != id[mu];
                        q[mu - 1] = make_int2(rid, id[mu]);
                    }
                }
            }
        }
        const uint32_t npair = (uint32_t)e[0] + (uint32_t)e[1] + (uint32_t)e[2];
        const uint64_t b0 = __ballot(npair & 1u), b1 = __ballot(npair & 2u);
        const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(b0 >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b0, 0u)) +
                               2u * __builtin_amdgcn_mbcnt_hi((uint32_t)(b1 >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b1, 0u));
        const int wave = tid >> 6;
        if ((tid & 63) == 0) U[wave] = (uint32_t)(__popcll(b0) + 2 * __popcll(b1));
        __syncthreads();
        int at = placed + (int)below, total = 0;
        for (int w = 0; w < NC / 64; ++w) {
            const int t = (int)U[w];
            at += w < wave ? t : 0;
            total += t;
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (e[k]) list[at] = q[k];
            at += e[k];
        }
        placed += total;
        if (jb + NC < kItems) __syncthreads();  // U[wave] is rewritten by the next round
    }
    if (tid == 0) d.pairs[(int64_t)tile * d.list_stride] = placed;
}

// ------------------------------------------------------- forest passes ---
// Work on the tiles' crossing lists, one workgroup per tile:
//   unite  unite the local roots of the two names of every pair (the unite
//          pass of every chain, and a phase of the persistent kernel);
//   store  store the encoded root of its tree (the cluster's smallest site
//          and its flip coin) in every local root of the list (walks stop
//          at the first stored encoding, so they shorten as the pass
//          proceeds); only the persistent kernel runs it, the chains
//          settle their roots in the flip pass instead.

// Unite pass of one tile (kBlock threads).  The pairs of a tile mostly share
// a few local roots, so hooking them one by one makes the tile's threads
// race for the same roots.  Instead, the distinct local roots of the list
// are grouped by the list's pairs in an LDS union-find, and every member of
// a group is united with the group's smallest member: the hooks of one tile
// then target distinct roots.  Pairs beyond the LDS tables are united
// directly.
//
// When a store phase follows (keep_roots: the persistent kernel), the
// tile's list is then replaced by its distinct local roots, which is all
// the store phase needs: it skips resolving names again.  With room for it
// (list_stride >= 2 + 2 H), head[1] = -m and the m roots from head[2] on are
// followed, from head[2 + H] on, by the list position of each root's group
// representative, so the store phase walks once per group.  Otherwise
// head[1] = m and only the roots are written.  head[1] = 0 keeps the pairs
// (some root did not fit in the table).  A local root that occurs only in
// pairs whose two names resolve to it is left out: it is never hooked nor
// hooked under, and its entry (itself) is already its canonical form.
constexpr int kTileRoots = 1024;  // LDS root table of the unite pass

constexpr int kUniteThreads = 256;   // threads per tile in the unite pass (its CAS chains are latency bound;
                                     // smaller workgroups let more tiles run at once)

// LDS words that other threads of the workgroup change concurrently (root
// tables and parent slots of the unite pass and the store phase) are read and
// written with relaxed workgroup-scope atomics, so that no load is hoisted
// out of a retry loop or served from a register copy.
__device__ __forceinline__ int lds_ld(const int *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); }
__device__ __forceinline__ void lds_st(int *p, int v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); }

// LDS of the unite pass of one tile.
struct UniteLds {
    static constexpr int kMaxListed = 1024;  // pairs kept in LDS
    int HK[kTileRoots];           // local root of the slot, -1 if free
    int HP[kTileRoots];           // LDS parent slot
    uint64_t BEST[kTileRoots];    // per group: smallest member << 10 | its slot
    int16_t PA[kMaxListed], PB[kMaxListed];
    int nroots, missed;
};

template <int NT, bool COUNT = false>
__device__ __forceinline__ void unite_tile_pairs(int32_t *lab, int *head, int n, int list_stride, int tid, UniteLds &S,
                                                 unsigned long long *counts, bool keep_roots)
{
    constexpr int H = kTileRoots;                    // root slots
    constexpr int kMaxListed = UniteLds::kMaxListed;  // pairs kept in LDS
    const int2 *list = reinterpret_cast<const int2 *>(head) + 1;
    for (int k = tid; k < H; k += NT) {
        S.HK[k] = -1;
        S.HP[k] = k;
        S.BEST[k] = ~0ull;
    }
    if (tid == 0) {
        S.nroots = 0;
        S.missed = 0;
    }
    __syncthreads();
    auto insert = [&](int key) {
        uint32_t h = (uint32_t)key * 0x9E3779B1u;
        h ^= h >> 15;
        for (int probe = 0; probe < 32; ++probe) {
            const int slot = (int)((h + (uint32_t)probe) & (H - 1));
            int prev = lds_ld(&S.HK[slot]);
            if (prev == -1) prev = atomicCAS(&S.HK[slot], -1, key);
            if (prev == -1 || prev == key) return slot;
        }
        return -1;
    };
    // Four of the thread's pairs at a time: their names are resolved with all
    // label loads in flight together, then entered in the table.
    constexpr int kBatch = 4;
    for (int k0 = tid; k0 < n; k0 += kBatch * NT) {
        int ra[kBatch], rb[kBatch];
#pragma unroll
        for (int i = 0; i < kBatch; ++i) {
            const int k = k0 + i * NT;
            const int2 p = k < n ? list[k] : make_int2(kTag, kTag);
            ra[i] = name_root(lab, p.x);
            rb[i] = name_root(lab, p.y);
        }
#pragma unroll
        for (int i = 0; i < kBatch; ++i) {
            const int k = k0 + i * NT;
            if (k >= n) break;
            const int sa = ra[i] == rb[i] ? -1 : insert(ra[i]), sb = ra[i] == rb[i] ? -1 : insert(rb[i]);
            const bool listed = k < kMaxListed && sa >= 0 && sb >= 0;
            if (!listed && ra[i] != rb[i]) forest_unite<COUNT>(lab, ra[i], rb[i], counts);
            if (ra[i] != rb[i] && (sa < 0 || sb < 0)) S.missed = 1;
            if (k < kMaxListed) {
                S.PA[k] = (int16_t)(listed ? sa : -1);
                S.PB[k] = (int16_t)(listed ? sb : -1);
            }
        }
    }
    __syncthreads();
    auto slot_find = [&](int x) {
        for (int it = 0; it < H; ++it) {
            const int p = lds_ld(&S.HP[x]);
            if (p == x) return x;
            const int gp = lds_ld(&S.HP[p]);
            if (gp != p) lds_st(&S.HP[x], gp);
            x = p;
        }
        return x;
    };
    const int nl = min(n, kMaxListed);
    for (int k = tid; k < nl; k += NT) {
        int a = S.PA[k], b = S.PB[k];
        if (a < 0) continue;
        for (int it = 0; it < H; ++it) {
            a = slot_find(a);
            b = slot_find(b);
            if (a == b) break;
            if (a < b) {
                const int t = a;
                a = b;
                b = t;
            }
            const int old = atomicMin(&S.HP[a], b);
            if (old == a) break;
            a = old;
        }
    }
    __syncthreads();
    for (int s = tid; s < H; s += NT) {
        if (S.HK[s] < 0) continue;
        atomicMin(&S.BEST[slot_find(s)], (uint64_t)S.HK[s] << 10 | (uint64_t)s);
    }
    __syncthreads();
    // The pairs are read: overwrite them with the distinct local roots (at
    // most 2n of them, so they fit where the pairs were); PA now holds each
    // slot's list position.
    const bool with_reps = keep_roots && list_stride >= 2 + 2 * H;
    if (keep_roots && !S.missed) {
        for (int s = tid; s < H; s += NT) {
            if (S.HK[s] < 0) continue;
            const int j = atomicAdd(&S.nroots, 1);
            S.PA[s] = (int16_t)j;
            head[2 + j] = S.HK[s];
        }
    }
    __syncthreads();
    // Each member of a group other than its smallest is hooked under the
    // smallest (a smaller node, so a valid parent for a root).  A member that
    // is still a root of the global forest is hooked by one compare-and-swap,
    // without a walk, and the thread's compare-and-swaps are in flight
    // together; one that finds the member already hooked continues the union
    // from the parent it returned.
    constexpr int kSlotsPerThread = (H + NT - 1) / NT;
    constexpr int kHookBatch = kSlotsPerThread < 4 ? kSlotsPerThread : 4;
    for (int i0 = 0; i0 < kSlotsPerThread; i0 += kHookBatch) {
        int ha[kHookBatch], hb[kHookBatch], old[kHookBatch];
#pragma unroll
        for (int i = 0; i < kHookBatch; ++i) {
            const int s = tid + (i0 + i) * NT;
            ha[i] = -1;
            hb[i] = -1;
            if (s < H && S.HK[s] >= 0) {
                const int rs = (int)(S.BEST[slot_find(s)] & (uint64_t)(H - 1));
                if (!S.missed && with_reps) head[2 + H + S.PA[s]] = S.PA[rs];
                if (rs != s) {
                    ha[i] = S.HK[s];
                    hb[i] = S.HK[rs];
                }
            }
        }
#pragma unroll
        for (int i = 0; i < kHookBatch; ++i) old[i] = ha[i] >= 0 ? atomicCAS(lab + ha[i], ha[i], kTag | hb[i]) : -1;
#pragma unroll
        for (int i = 0; i < kHookBatch; ++i) {
            if (ha[i] < 0) continue;
            if (COUNT) {  // measurement runs only (a kernel of its own)
                atomicAdd(&counts[0], 1ull);
                if (old[i] == ha[i]) atomicAdd(&counts[1], 1ull);
            }
            if (old[i] != ha[i]) forest_unite<COUNT>(lab, old[i] & kIdxMask, hb[i], counts);
        }
    }
    if (tid == 0 && keep_roots) head[1] = S.missed ? 0 : (with_reps ? -S.nroots : S.nroots);
}

// Store phase of one tile in the persistent kernel (NT threads; HK:
// kTileRoots ints of LDS).
template <int NT>
__device__ __forceinline__ void store_tile(const RepDesc &d, const RepState &st, int tile, int tid, int *HK)
{
    constexpr int H = kTileRoots;
    int *head = d.pairs + (int64_t)tile * d.list_stride;
    const int2 *list = reinterpret_cast<const int2 *>(head) + 1;
    const int n = head[0];
    int32_t *lab = d.label;
    if (n == 0) return;
    const int nroots = head[1];  // != 0: the list holds the tile's distinct local roots
    if (nroots < 0) {
        // with group representatives: one walk per group, then plain stores
        const int m = -nroots;
        const int *rp = head + 2 + H;
        for (int k = tid; k < m; k += NT) {
            if (rp[k] != k) continue;
            const int r = head[2 + k];
            const int e = canon_encoding(lab, r, st.t, d.key);
            HK[k] = e;
            lab_store(lab, r, e);
        }
        __syncthreads();
        for (int k = tid; k < m; k += NT)
            if (rp[k] != k) lab_store(lab, head[2 + k], HK[rp[k]]);
        return;
    }
    if (nroots > 0) {
        for (int k = tid; k < nroots; k += NT) {
            const int r = head[2 + k];
            lab_store(lab, r, canon_encoding(lab, r, st.t, d.key));
        }
        return;
    }
    // The list kept its pairs: store once per distinct local root, found
    // through an LDS hash table (a full table stores directly).
    for (int k = tid; k < H; k += NT) HK[k] = -1;
    __syncthreads();
    auto add = [&](int key) {
        uint32_t h = (uint32_t)key * 0x9E3779B1u;
        h ^= h >> 15;
        for (int probe = 0; probe < 32; ++probe) {
            const int slot = (int)((h + (uint32_t)probe) & (H - 1));
            int prev = lds_ld(&HK[slot]);
            if (prev == -1) prev = atomicCAS(&HK[slot], -1, key);
            if (prev == -1 || prev == key) return;
        }
        lab_store(lab, key, canon_encoding(lab, key, st.t, d.key));
    };
    for (int k = tid; k < 2 * n; k += NT) {
        const int2 p = list[k >> 1];
        add(name_root(lab, (k & 1) ? p.y : p.x));
    }
    __syncthreads();
    for (int k = tid; k < H; k += NT) {
        const int key = HK[k];
        if (key >= 0) lab_store(lab, key, canon_encoding(lab, key, st.t, d.key));
    }
}

// Unite pass of one tile (NT threads).
template <int NT, bool COUNT = false>
__device__ __forceinline__ void unite_tile(const RepDesc &d, int tile, int tid, UniteLds &S,
                                           unsigned long long *counts = nullptr, bool keep_roots = true)
{
    int *head = d.pairs + (int64_t)tile * d.list_stride;
    unite_tile_pairs<NT, COUNT>(d.label, head, head[0], d.list_stride, tid, S, counts, keep_roots);
}

// The unite pass of a chain.  COUNT: it counts its compare-and-swaps into
// c.counts (measurement runs).  The chains settle their roots in the flip
// pass and run no store pass, so the lists are left as they are.
template <bool COUNT = false>
__global__ __launch_bounds__(kUniteThreads) void k_forest(Chain c)
{
    __shared__ UniteLds S;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int rep = c.tile_rep[blk];
    const RepState st = *c.state[rep];
    if (st.remaining <= 0) return;
    const RepDesc &d = c.desc[rep];
    unite_tile<kUniteThreads, COUNT>(d, blk - d.tile_base, threadIdx.x, S, c.counts, false);
}

// Shape dispatch: calls F::template run<TX, TY, TZ>(args...).
template <typename F, typename... Args>
hipError_t with_tile_shape(int shape, Args &&...args)
{
    switch (shape) {
    case kTile844: return F::template run<8, 4, 4>(args...);
    case kTile444: return F::template run<4, 4, 4>(args...);
    case kTile888: return F::template run<8, 8, 8>(args...);
    case kTile1688: return F::template run<16, 8, 8>(args...);
    default: return F::template run<8, 8, 4>(args...);
    }
}

// Launcher of the model-independent unite pass (tile_common.hip).
hipError_t launch_unite(const Chain &c, hipStream_t st, const LaunchHook &hook);

// Per-model chain launchers (ising_tiled.hip, on_tiled.hip).
hipError_t launch_ising_sweep(const Chain &c, hipStream_t st, const LaunchHook &hook);
hipError_t launch_ising_energy_tail(const Chain &c, hipStream_t st, const LaunchHook &hook);
hipError_t launch_on_sweep(const Chain &c, hipStream_t st, const LaunchHook &hook);
hipError_t launch_on_energy_tail(const Chain &c, hipStream_t st, const LaunchHook &hook);

}  // namespace pyro
