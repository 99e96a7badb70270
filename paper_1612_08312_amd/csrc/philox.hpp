// Philox4x32-10 counter-based generator for gfx950.
//
// Written from the description in Salmon, Moraes, Dror, Shaw, "Parallel
// random numbers: as easy as 1, 2, 3" (SC'11): a 128-bit counter and a
// 64-bit key; each of the ten rounds multiplies counter words 0 and 2 by two
// fixed odd 32-bit constants, recombines the high halves with words 1 and 3
// and the round key by XOR, and the two key words advance by two Weyl
// constants between rounds.  The 32x32->64 products map to v_mad_u64_u32.
//
// Counter layout used by this library: (unit, sweep, stream, attempt); key
// = (seed mod 2^32, seed >> 32).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pyro {

enum : uint32_t {
    kStreamBond = 0,    // bond activation, top byte (Ising) / full word (O(n))
    kStreamFlip = 1,    // cluster flip coins
    kStreamInit = 2,    // random initial state
    kStreamAxis = 3,    // embedding axis of each sweep
    kStreamBondLo = 4,  // bond activation, low 24 bits (Ising)
};

struct PhiloxKey {
    uint32_t k0, k1;
};

__host__ __device__ inline PhiloxKey philox_key(uint64_t seed)
{
    return PhiloxKey{(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
}

__device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                               uint32_t c3, PhiloxKey key)
{
    uint32_t k0 = key.k0, k1 = key.k1;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        // three-way XORs as one v_bitop3_b32 each (truth table 0x96)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

__device__ __forceinline__ uint32_t word_of(const uint4 &v, uint32_t k)
{
    return k == 0 ? v.x : k == 1 ? v.y : k == 2 ? v.z : v.w;
}

}  // namespace pyro
