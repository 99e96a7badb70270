// LDS-resident Swendsen-Wang sweeps of small Ising lattices (L <= 16): one
// workgroup holds a whole lattice in LDS and runs all of its sweeps of a call
// in one launch, with only workgroup barriers between the steps.  The method
// is the one of the tiled sweep (Sec. 1-2 of the paper: bond activation,
// cluster labeling, flip of each cluster with probability 1/2, moments of
// Eq. 2) with the same random draws, so every record, spin and label is
// identical to the tiled path's.
//
// LDS of a lattice of N = 16 L^3 sites (N <= 65536, so a site index fits in
// 16 bits; offsets in resident.hpp):
//   PF   uint16 [N]       forest: parent site of each site; roots are the
//                         smallest site of their component (hooks put the
//                         larger root under the smaller)
//   SMK  uint16 [L^3]     spin mask of each cell (bit k: site k is -1)
//   CW   uint32 [N/32]    flip coins of the sweep: bit (r mod 32) of word
//                         r/32 is the coin of the cluster rooted at r
// At L = 16 that is 128 + 8 + 8 KiB.  One sweep:
//   1. each cell's 48 bonds are activated (ising_activate) and the
//      components of its four up tetrahedra seed the forest (K4 table);
//   2. the spanning edges of the components of each down tetrahedron are
//      united (every bond of the lattice is inside the workgroup);
//   3. the coins: one Philox block per 128 sites;
//   4. every site finds its root and flips with the root's coin (the labels
//      are written out after the last sweep);
//   5. magnetisation and bond sum of the new state, one record.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_util.hpp"
#include "ising_cell.hpp"
#include "kernels.hpp"
#include "lattice.hpp"
#include "philox.hpp"
#include "resident.hpp"

namespace pyro {

namespace {

typedef __attribute__((address_space(3))) volatile uint16_t lds_u16;
typedef __attribute__((address_space(3))) uint32_t lds_u32;

constexpr int kCellsPerThread = (kResidentMaxL * kResidentMaxL * kResidentMaxL + kResidentThreads - 1) / kResidentThreads;

// Root of site x with path halving (parents never exceed their children, so
// the walk steps to strictly smaller sites and ends).
__device__ __forceinline__ uint32_t find16(lds_u16 *PF, uint32_t x)
{
    uint32_t p = PF[x];
    while (p < x) {
        const uint32_t gp = PF[p];
        PF[x] = (uint16_t)gp;
        x = p;
        p = gp;
    }
    return x;
}

// Union of the components of sites a and b: the larger root is hooked under
// the smaller by a compare-and-swap of the 32-bit word holding its entry
// (the other half of the word may change meanwhile; the swap then fails and
// is retried on the word's new value).
__device__ __forceinline__ void unite16(lds_u16 *PF, uint32_t a, uint32_t b)
{
    for (;;) {
        a = find16(PF, a);
        b = find16(PF, b);
        if (a == b) return;
        if (a < b) {
            const uint32_t t = a;
            a = b;
            b = t;
        }
        lds_u32 *w = (lds_u32 *)((__attribute__((address_space(3))) char *)PF + 2 * (a & ~1u));
        const uint32_t sh = 16u * (a & 1u);
        uint32_t old = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        bool hooked = false;
        for (;;) {
            const uint32_t pa = (old >> sh) & 0xFFFFu;
            if (pa != a) {  // a was hooked meanwhile: continue from its new parent
                a = pa;
                break;
            }
            const uint32_t nw = (old & ~(0xFFFFu << sh)) | (b << sh);
            const uint32_t got = atomicCAS((uint32_t *)w, old, nw);
            if (got == old) {
                hooked = true;
                break;
            }
            old = got;
        }
        if (hooked) return;
    }
}

}  // namespace

// One workgroup of kResidentThreads threads per replica of the chain (all of
// edge L <= kResidentMaxL, no vacant sites): `remaining` sweeps, records into
// the ring, then the state is advanced as the tiled finalize would.
__global__ __launch_bounds__(kResidentThreads) void k_resident_ising(Chain c)
{
    extern __shared__ __align__(16) char lds[];
    const int rep = blockIdx.x;
    const RepState st = *c.state[rep];
    if (st.remaining <= 0) return;
    const RepDesc &d = c.desc[rep];
    const int L = d.L;
    const int ncell = (int)d.ncell;
    const int N = (int)d.N;
    const int tid = threadIdx.x;
    constexpr int NT = kResidentThreads;
    const ResidentLayout ly = resident_layout(L);
    __attribute__((address_space(3))) char *base = (__attribute__((address_space(3))) char *)lds;
    lds_u16 *PF = (lds_u16 *)(base + ly.pf);
    lds_u16 *SMK = (lds_u16 *)(base + ly.smk);
    lds_u32 *CW = (lds_u32 *)(base + ly.cw);
    __attribute__((address_space(3))) uint8_t *K4 = (__attribute__((address_space(3))) uint8_t *)(base + ly.k4);
    int64_t *red = (int64_t *)(lds + ly.red);

    if (tid < 64) {
        constexpr K4Table k4 = make_k4();
        K4[tid] = k4.v[tid];
    }
    // The six lower neighbour cells of each of the thread's cells.
    int nbc[kCellsPerThread][kNCellCodes];
#pragma unroll
    for (int j = 0; j < kCellsPerThread; ++j) {
        const int c0 = tid + j * NT;
        if (c0 < ncell) {
            const CellNbrs nb = cell_neighbours(c0, L);
#pragma unroll
            for (int q = 0; q < kNCellCodes; ++q) nbc[j][q] = nb.c[q];
            SMK[c0] = (uint16_t)spin_mask16(reinterpret_cast<const int4 *>(d.spins)[c0]);
        } else {
#pragma unroll
            for (int q = 0; q < kNCellCodes; ++q) nbc[j][q] = 0;
        }
    }
    __syncthreads();
    const IsingParams prm{d.thr_hi, d.thr_lo};
#define PYRO_DOWN_OF(j, m)                                                                                   \
    down_mask16((m), SMK[nbc[j][kMx]], SMK[nbc[j][kMy]], SMK[nbc[j][kMz]], SMK[nbc[j][kMyMz]],             \
                SMK[nbc[j][kMxMz]], SMK[nbc[j][kMxMy]])
    for (int s = 0; s < st.remaining; ++s) {
        const uint32_t t = st.t + (uint32_t)s;
        // 1. activation; up tetrahedra seed the forest
        uint64_t act[kCellsPerThread];
#pragma unroll
        for (int j = 0; j < kCellsPerThread; ++j) {
            const int c0 = tid + j * NT;
            act[j] = 0;
            if (c0 < ncell) {
                const uint32_t m = SMK[c0];
                act[j] = ising_activate(aligned48(m, PYRO_DOWN_OF(j, m)), (uint32_t)c0, t, d.key, prm);
#pragma unroll
                for (int f = 0; f < 4; ++f) {
                    const uint32_t code = K4[(uint32_t)(act[j] >> (6 * f)) & 63u];
                    const uint32_t base = 16u * (uint32_t)c0 + 4u * f;
#pragma unroll
                    for (int mu = 0; mu < 4; ++mu) PF[base + mu] = (uint16_t)(base + ((code >> (2 * mu)) & 3u));
                }
            }
        }
        __syncthreads();
        // 2. down tetrahedra: spanning edges of their components
#pragma unroll
        for (int j = 0; j < kCellsPerThread; ++j) {
            const int c0 = tid + j * NT;
            if (c0 >= ncell) continue;
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                const uint32_t code = K4[(uint32_t)(act[j] >> (24 + 6 * f)) & 63u];
                if (code == 0xE4u) continue;  // four single vertices
                uint32_t v[4];
#pragma unroll
                for (int mu = 0; mu < 4; ++mu) {
                    const SiteRef R = down_vertex(f, mu);
                    v[mu] = 16u * (uint32_t)(R.cell == kSelf ? c0 : nbc[j][R.cell]) + R.site;
                }
#pragma unroll
                for (int mu = 1; mu < 4; ++mu) {
                    const uint32_t rp = (code >> (2 * mu)) & 3u;
                    if (rp != (uint32_t)mu) unite16(PF, v[rp], v[mu]);
                }
            }
        }
        // 3. coins of the sweep
        for (int g = tid; g < (N + 127) / 128; g += NT) {
            const uint4 w = philox4x32_10((uint32_t)g, t, kStreamFlip, 0u, d.key);
            CW[4 * g] = w.x;
            if (4 * g + 1 < (N + 31) / 32) CW[4 * g + 1] = w.y;
            if (4 * g + 2 < (N + 31) / 32) CW[4 * g + 2] = w.z;
            if (4 * g + 3 < (N + 31) / 32) CW[4 * g + 3] = w.w;
        }
        __syncthreads();
        // 4. roots, coins and flips (labels after the last sweep)
        const bool last = s + 1 == st.remaining;
        uint32_t nm[kCellsPerThread];
#pragma unroll
        for (int j = 0; j < kCellsPerThread; ++j) {
            const int c0 = tid + j * NT;
            nm[j] = 0;
            if (c0 >= ncell) continue;
            uint32_t flip = 0, last_r = 0xFFFFFFFFu, last_coin = 0;
            for (int k = 0; k < 16; ++k) {
                const uint32_t r = find16(PF, 16u * (uint32_t)c0 + k);
                if (r != last_r) {
                    last_r = r;
                    last_coin = (CW[r >> 5] >> (r & 31u)) & 1u;
                }
                flip |= last_coin << k;
                if (last) d.label[16 * c0 + k] = (int)r;
            }
            nm[j] = SMK[c0] ^ flip;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kCellsPerThread; ++j)
            if (tid + j * NT < ncell) SMK[tid + j * NT] = (uint16_t)nm[j];
        __syncthreads();
        // 5. moments of the new state
        int64_t bsum = 0, down = 0;
#pragma unroll
        for (int j = 0; j < kCellsPerThread; ++j) {
            const int c0 = tid + j * NT;
            if (c0 >= ncell) continue;
            bsum += 2 * (int64_t)__popcll(aligned48(nm[j], PYRO_DOWN_OF(j, nm[j]))) - 48;
            down += __popc(nm[j]);
        }
        const int64_t B = block_sum<int64_t>(bsum, red);
        const int64_t D = block_sum<int64_t>(down, red);
        if (tid == 0) {
            const int slot = st.ring_used + s;
            if (slot < d.ring_cap) {
                const int64_t M = (int64_t)N - 2 * D;
                DevRecord rec;
                rec.sweep = t;
                rec.bond_sum = B;
                rec.M_int = M;
                rec.reserved = 0;
                rec.E = -d.J * (double)B;
                rec.M[0] = (double)M;
                rec.M[1] = 0.0;
                rec.M[2] = 0.0;
                const double mm = (double)M / (double)d.N;
                rec.m2 = mm * mm;
                rec.m4 = rec.m2 * rec.m2;
                d.ring[slot] = rec;
            }
        }
    }
#undef PYRO_DOWN_OF
    // spins back to HBM (+1 = 0x01, -1 = 0xFF)
#pragma unroll
    for (int j = 0; j < kCellsPerThread; ++j) {
        const int c0 = tid + j * NT;
        if (c0 >= ncell) continue;
        const uint32_t m = SMK[c0];
        uint32_t w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            w[q] = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) w[q] |= (((m >> (4 * q + b)) & 1u) ? 0xFFu : 0x01u) << (8 * b);
        }
        reinterpret_cast<int4 *>(d.spins)[c0] = make_int4((int)w[0], (int)w[1], (int)w[2], (int)w[3]);
    }
    if (tid == 0) {
        RepState ns;
        ns.t = st.t + (uint32_t)st.remaining;
        ns.remaining = 0;
        ns.ring_used = st.ring_used + st.remaining;
        ns.e_pending = -1;
        *c.state[rep] = ns;
    }
}

hipError_t launch_resident_ising(const Chain &c, int maxL, hipStream_t st, const LaunchHook &hook)
{
    if (c.nreps == 0) return hipSuccess;
    if (maxL < 1 || maxL > kResidentMaxL) return hipErrorInvalidValue;
    static const hipError_t attr = hipFuncSetAttribute(
        (const void *)k_resident_ising, hipFuncAttributeMaxDynamicSharedMemorySize, (int)resident_layout(kResidentMaxL).total);
    if (attr != hipSuccess) return attr;
    const size_t lds = resident_layout(maxL).total;
    if (hook.before) hook.before(hook.ctx, kKResident);
    k_resident_ising<<<c.nreps, kResidentThreads, lds, st>>>(c);
    if (hook.after) hook.after(hook.ctx, kKResident);
    return hipGetLastError();
}

}  // namespace pyro
