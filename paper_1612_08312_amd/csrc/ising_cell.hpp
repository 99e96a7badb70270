// Per-cell pieces of the Ising sweep shared by the tiled and batched kernels:
// spin bit masks, bond alignment, the bond activation decision and the
// connected components of one tetrahedron.
//
// Bond j (0..47) of a cell belongs to tetrahedron j/6 (0..3 up, 4..7 down)
// and joins its vertices (0,1),(0,2),(0,3),(1,2),(1,3),(2,3) for j mod 6.
// The activation of bond b = 48 cell + j uses r32(b) = (byte (j mod 16) of
// Philox(3 cell + j/16, t, BOND)) << 24 | low 24 bits of word (j mod 4) of
// Philox(12 cell + j/4, t, BOND_LO); the bond is active iff its spins are
// equal and r32 < thr.  Comparing the top byte decides every bond except a
// tie with thr >> 24 (probability 1/256), for which the low call is made.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"
#include "lattice.hpp"
#include "philox.hpp"

namespace pyro {

// Activation threshold thr = floor((1 - exp(-2J/T)) 2^32), split at bit 24
// (thr_hi = 256 when every parallel bond is active).
struct IsingParams {
    uint32_t thr_hi;
    uint32_t thr_lo;
};

// Byte flags of four words (each byte 0x80 when set, 0 otherwise) -> 16 bits,
// bit 4k + b = the flag of byte b of word k.  v_dot4_u32_u8 sums the four
// byte products with the weights 2^b (word 0, 2) or 2^(b+4) (word 1, 3), so
// each pair of words lands as a byte shifted left by 7: full-rate dot
// instructions instead of quarter-rate multiplies.
__device__ __forceinline__ uint32_t gather_flags16(uint32_t f0, uint32_t f1, uint32_t f2, uint32_t f3)
{
    const uint32_t lo = __builtin_amdgcn_udot4(f1, 0x80402010u, __builtin_amdgcn_udot4(f0, 0x08040201u, 0u, false), false);
    const uint32_t hi = __builtin_amdgcn_udot4(f3, 0x80402010u, __builtin_amdgcn_udot4(f2, 0x08040201u, 0u, false), false);
    return (lo >> 7) | (hi << 1);
}

// 16 int8 spins (+1 = 0x01, -1 = 0xFF) -> 16-bit mask, bit k set when spin k
// is -1 (the byte's sign bit).
__device__ __forceinline__ uint32_t spin_mask16(int4 v)
{
    return gather_flags16((uint32_t)v.x & 0x80808080u, (uint32_t)v.y & 0x80808080u, (uint32_t)v.z & 0x80808080u,
                          (uint32_t)v.w & 0x80808080u);
}

// Mask of the 16 down-tetrahedron vertices, bit 4f + mu = vertex mu of the
// down tetrahedron of FCC point f (see down_vertex in lattice.hpp), from the
// masks of the owning cell and its six lower neighbours.
__device__ __forceinline__ uint32_t down_mask16(uint32_t m, uint32_t nx, uint32_t ny, uint32_t nz,
                                                uint32_t nyz, uint32_t nxz, uint32_t nxy)
{
    auto bit = [](uint32_t v, int k) { return (v >> k) & 1u; };
    return bit(m, 0) | bit(nyz, 5) << 1 | bit(nxz, 10) << 2 | bit(nxy, 15) << 3 |
           bit(m, 4) << 4 | bit(m, 1) << 5 | bit(nx, 14) << 6 | bit(nx, 11) << 7 |
           bit(m, 8) << 8 | bit(ny, 13) << 9 | bit(m, 2) << 10 | bit(ny, 7) << 11 |
           bit(m, 12) << 12 | bit(nz, 9) << 13 | bit(nz, 6) << 14 | bit(m, 3) << 15;
}

// 6-bit mask of the antiparallel vertex pairs of a tetrahedron whose four
// vertex spins are the bits of v (pair order as above).  Table of all 16
// vertex patterns packed in two 64-bit words (8 patterns x 6 bits each).
struct Anti6Table {
    uint64_t w[2];
};
__host__ __device__ constexpr Anti6Table make_anti6()
{
    Anti6Table t{{0, 0}};
    for (int v = 0; v < 16; ++v) {
        uint64_t code = 0;
        for (int e = 0; e < 6; ++e) {
            const int a = pair_a(e), b = pair_b(e);
            if (((v >> a) ^ (v >> b)) & 1) code |= 1ull << e;
        }
        t.w[v >> 3] |= code << (6 * (v & 7));
    }
    return t;
}

__device__ __forceinline__ uint32_t anti6(uint32_t v)
{
    constexpr Anti6Table t = make_anti6();
    const uint64_t w = (v & 8u) ? t.w[1] : t.w[0];
    return (uint32_t)(w >> (6 * (v & 7u))) & 63u;
}

// 48-bit mask of the parallel (aligned) bonds of a cell.
__device__ __forceinline__ uint64_t aligned48(uint32_t m, uint32_t dm)
{
    uint64_t anti = 0;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        anti |= (uint64_t)anti6((m >> (4 * f)) & 15u) << (6 * f);
        anti |= (uint64_t)anti6((dm >> (4 * f)) & 15u) << (24 + 6 * f);
    }
    return ~anti & 0xFFFFFFFFFFFFull;
}

// Per-byte flags of four bytes x against one byte value c (replicated in C):
// x < c and x == c, as 0x80 in each byte where the comparison holds.
__device__ __forceinline__ uint32_t bytes_lt(uint32_t x, uint32_t C)
{
    // d: top bit of each byte = (x mod 128) >= (c mod 128), no cross-byte borrow
    const uint32_t d = (x | 0x80808080u) - (C & 0x7F7F7F7Fu);
    return ((~x & C) | (~(x ^ C) & ~d)) & 0x80808080u;
}

__device__ __forceinline__ uint32_t bytes_eq(uint32_t x, uint32_t C)
{
    const uint32_t t = x ^ C;
    const uint32_t nz = ((t & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | t;
    return ~nz & 0x80808080u;
}

// Active bonds of cell `cell` in sweep t, given its aligned-bond mask.
__device__ __forceinline__ uint64_t ising_activate(uint64_t aligned, uint32_t cell, uint32_t t, PhiloxKey key,
                                                   IsingParams p)
{
    if (aligned == 0) return 0;
    uint64_t acc = 0, tie = 0;
    if (p.thr_hi >= 256u) {
        acc = ~0ull;
    } else {
        const uint32_t C = p.thr_hi * 0x01010101u;
        uint32_t lt[3], eq[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const uint4 r = philox4x32_10(3u * cell + q, t, kStreamBond, 0u, key);
            lt[q] = gather_flags16(bytes_lt(r.x, C), bytes_lt(r.y, C), bytes_lt(r.z, C), bytes_lt(r.w, C));
            eq[q] = gather_flags16(bytes_eq(r.x, C), bytes_eq(r.y, C), bytes_eq(r.z, C), bytes_eq(r.w, C));
        }
        acc = (uint64_t)(lt[0] | lt[1] << 16) | (uint64_t)lt[2] << 32;
        tie = (uint64_t)(eq[0] | eq[1] << 16) | (uint64_t)eq[2] << 32;
    }
    uint64_t act = aligned & acc;
    uint64_t amb = aligned & tie;
    while (amb) {
        const int j = __ffsll((unsigned long long)amb) - 1;
        amb &= amb - 1;
        const uint4 lo = philox4x32_10(12u * cell + (uint32_t)(j >> 2), t, kStreamBondLo, 0u, key);
        if ((word_of(lo, j & 3) & 0xFFFFFFu) < p.thr_lo) act |= 1ull << j;
    }
    return act;
}

// Components of a tetrahedron (K4) for each of the 64 active-edge patterns:
// 2 bits per vertex = smallest vertex of its component.
struct K4Table {
    uint8_t v[64];
};
__host__ __device__ constexpr K4Table make_k4()
{
    K4Table t{};
    for (int u = 0; u < 64; ++u) {
        int root[4] = {0, 1, 2, 3};
        for (int it = 0; it < 4; ++it)
            for (int e = 0; e < 6; ++e) {
                if (!((u >> e) & 1)) continue;
                const int ra = root[pair_a(e)], rb = root[pair_b(e)];
                const int lo = ra < rb ? ra : rb;
                for (int q = 0; q < 4; ++q)
                    if (root[q] == ra || root[q] == rb) root[q] = lo;
            }
        t.v[u] = (uint8_t)(root[0] | root[1] << 2 | root[2] << 4 | root[3] << 6);
    }
    return t;
}

}  // namespace pyro
