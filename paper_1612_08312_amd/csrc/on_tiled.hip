// XY (n = 2) and Heisenberg (n = 3) Swendsen-Wang sweep on gfx950, with
// Wolff's embedding (Sec. 2 of the paper): every spin is projected on the
// sweep's random unit axis r, sigma = s . r; the Ising-like cluster
// construction runs on the projections, and flipped clusters are reflected
// through the plane normal to r.
//
// Same tile structure and chain of lattices as the Ising sweep
// (tile_common.hpp, kernels.hpp).  Arithmetic that
// decides bonds or moves spins is FP32 in a fixed operation order with
// explicit fused multiply-adds:
//   sigma = fmaf(s_z, r_z, fmaf(s_y, r_y, s_x * r_x))      (XY: no z term)
//   x     = (x0 * sigma_a) * sigma_b,   x0 = (float)(2 J / T)
//   bond active iff (double)x > -log1p(-u), u = (r32 + 0.5) 2^-32, r32 =
//   word (b mod 4) of Philox(b/4, t, BOND)
//   reflection s_k <- fmaf(-2 sigma, r_k, s_k)
// The FP64 log1p is evaluated only when x lies within 1e-4 (1 + t) of
// t = -ln(1 - u) computed in FP32 with the native base-2 logarithm: that
// margin exceeds the FP32 error by orders of magnitude, so outside it the FP32
// comparison gives the same answer as the exact one.  Energies and
// magnetisations are FP64 sums of the FP32 spins.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "device_util.hpp"
#include "ising_cell.hpp"
#include "kernels.hpp"
#include "lattice.hpp"
#include "on_bond.hpp"
#include "philox.hpp"
#include "tile_common.hpp"
#include "unit_vector.hpp"

namespace pyro {

// Embedding axis of sweep t.  Both passes that use it draw it themselves:
// the inputs are uniform, so every lane computes the same value, at the cost
// of a few dozen instructions per wave instead of a kernel of its own (about
// 6 us per sweep, most of it launch latency).
template <int NV>
__device__ __forceinline__ void sweep_axis(const RepDesc &d, uint32_t t, float (&r)[NV])
{
    float a[3];
    unit_vector(0u, t, kStreamAxis, NV, d.key, a);
#pragma unroll
    for (int k = 0; k < NV; ++k) r[k] = a[k];
}


// Four waves per SIMD, so at most 128 VGPRs: left alone, the Heisenberg pass
// takes 139 and only three 8x8x4 workgroups share a CU (60 -> 51 us per
// L = 64 sweep with the cap, despite a few spills).  XY takes 113 either way;
// a cap of five waves made its pass slower (43 -> 48 us).
template <int NV, int TX, int TY, int TZ>
__global__ __launch_bounds__(TX *TY *TZ) __attribute__((amdgpu_waves_per_eu(4))) void k_local_on(Chain c)
{
    constexpr int NC = TX * TY * TZ;
    __shared__ uint32_t P[kForestSlots<NC>];
    __shared__ uint32_t U[kOnUnionsPerCell * NC];
    __shared__ uint32_t DA[NC];
    __shared__ uint8_t K4[64];
    __shared__ double red[16];

    const int blk = blockIdx.x;
    const int rep = c.tile_rep[blk];
    const RepState st = *c.state[rep];
    if (st.remaining <= 0) return;
    const RepDesc &d = c.desc[rep];
    const int tile = blk - d.tile_base;
    const TileIdx<TX, TY, TZ> ti = TileIdx<TX, TY, TZ>::of(tile, d);
    const float *__restrict__ s = (const float *)d.spins;
    const int64_t N = d.N;
    const float x0 = d.x0;
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

    uint64_t act = 0;
    double esum = 0.0;
    int lc[kNCellCodes];
    NbrCell nb[kNCellCodes];
    float own[NV][16];
#pragma unroll
    for (int q = 0; q < kNCellCodes; ++q) lc[q] = -1;
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int q = 0; q < 16; ++q) own[k][q] = 0.0f;
    if (valid) {
        ti.neighbours(x, y, z, cell, lcid, nb);
#pragma unroll
        for (int q = 0; q < kNCellCodes; ++q) lc[q] = nb[q].lcell;
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const float4 *S4 = reinterpret_cast<const float4 *>(s + (int64_t)k * N) + 4 * (int64_t)cell;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float4 v = S4[q];
                own[k][4 * q] = v.x;
                own[k][4 * q + 1] = v.y;
                own[k][4 * q + 2] = v.z;
                own[k][4 * q + 3] = v.w;
            }
        }
    }
    // Down-tetrahedron vertices: those in the tile are read from the tile's
    // spins, staged one component at a time in the forest array (free until
    // the tile components start; site q of local cell c at q NC + c), those
    // outside the tile from global memory.
    float dv[NV][16];
    float *SP = reinterpret_cast<float *>(P);
#pragma unroll
    for (int k = 0; k < NV; ++k) {
#pragma unroll
        for (int q = 0; q < 16; ++q) SP[q * NC + lcid] = own[k][q];
        __syncthreads();
        if (valid) {
#pragma unroll
            for (int f = 0; f < 4; ++f)
#pragma unroll
                for (int mu = 0; mu < 4; ++mu) {
                    const SiteRef R = down_vertex(f, mu);
                    float v;
                    if (R.cell == kSelf) {
                        v = own[k][R.site];
                    } else {
                        const int l = lc[R.cell];
                        if (l >= 0) v = SP[R.site * NC + l];
                        else v = s[(int64_t)k * N + 16 * nb[R.cell].gcell + R.site];
                    }
                    dv[k][4 * f + mu] = v;
                }
        }
        __syncthreads();
    }
    if (valid) {
        float r[NV];
        sweep_axis<NV>(d, st.t, r);
        float sig_own[16], sig_dv[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            float a[NV], b[NV];
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                a[k] = own[k][q];
                b[k] = dv[k][q];
            }
            sig_own[q] = project<NV>(a, r);
            sig_dv[q] = project<NV>(b, r);
        }
#pragma unroll
        for (int qg = 0; qg < 12; ++qg) {
            float xs[4];
            bool any = false;
#pragma unroll
            for (int k4 = 0; k4 < 4; ++k4) {
                const int j = 4 * qg + k4;
                const int tet = j / 6, e = j % 6;
                const int ia = 4 * (tet & 3) + pair_a(e), ib = 4 * (tet & 3) + pair_b(e);
                const float sa = tet < 4 ? sig_own[ia] : sig_dv[ia];
                const float sb = tet < 4 ? sig_own[ib] : sig_dv[ib];
                xs[k4] = __fmul_rn(__fmul_rn(x0, sa), sb);
                any |= xs[k4] > 0.0f;
                double dd = 0.0;
#pragma unroll
                for (int k = 0; k < NV; ++k) {
                    const float va = tet < 4 ? own[k][ia] : dv[k][ia];
                    const float vb = tet < 4 ? own[k][ib] : dv[k][ib];
                    dd += (double)va * (double)vb;
                }
                esum += dd;
            }
            if (any) {
                const uint4 rnd = philox4x32_10(12u * (uint32_t)cell + qg, st.t, kStreamBond, 0u, d.key);
#pragma unroll
                for (int k4 = 0; k4 < 4; ++k4)
                    if (on_bond_active(xs[k4], word_of(rnd, k4))) act |= 1ull << (4 * qg + k4);
            }
        }
    }
    tile_components<TX, TY, TZ, kOnUnionsPerCell>(d, ti, tile, tid, lcid, valid, cell, act, lc, P, U, DA, K4);
    const double b = block_sum<double, false>(esum, red);
    if (tid == 0) d.dpart[tile] = b;
}

// LDS of the O(n) settle-and-flip pass.
template <int TX, int TY, int TZ>
struct OnFlipLds {
    alignas(16) int LAB[16 * TX * TY * TZ];  // labels of the tile's sites
    alignas(16) uint32_t CB[TX * TY * TZ];   // coins of the tile's sites
    uint16_t HL[kSettleListPerCell * TX * TY * TZ];  // local keys of the tile's hooked local roots
    int wtot[TX * TY * TZ / 64];
    double red[16];
};

// One workgroup per tile, once every unite is done: the settle step
// (settle_tile_roots), cluster coins from the LDS copy of the tile's labels
// and the tile's own coins (as in the Ising flip; MODE as there),
// reflections, FP64 magnetisation.
template <int NV, int TX, int TY, int TZ, int MODE>
__device__ __forceinline__ void on_settle_flip_pass(const RepDesc &d, const RepState &st, int tile, int tid,
                                                    OnFlipLds<TX, TY, TZ> &S)
{
    constexpr int NC = TX * TY * TZ;
    constexpr bool ALIGNED = MODE != kFlipGeneral;  // labels staged by local key, every thread has a cell
    int *LAB = S.LAB;
    uint32_t *CB = S.CB;
    const TileIdx<TX, TY, TZ> ti = TileIdx<TX, TY, TZ>::of(tile, d);
    const int L = d.L;
    const int lx = tid % TX, ly = (tid / TX) % TY, lz = tid / (TX * TY);
    const int x = ti.bx * TX + lx, y = ti.by * TY + ly, z = ti.bz * TZ + lz;
    const bool valid = ALIGNED || (x < L && y < L && z < L);
    const int cell = cell_index(x, y, z, L);
    const int64_t N = d.N;
    float *s = (float *)d.spins;
    int lab[16];
    const uint32_t hm = valid ? stage_cell_labels<NC, ALIGNED>(d.label, cell, tid, lab, LAB) : 0u;
    if constexpr (ALIGNED) {
        if (tid < NC / 8) reinterpret_cast<uint4 *>(CB)[tid] = aligned_coin_words<TX, TY, TZ>(ti, tid, st.t, d.key);
    } else {
        CB[tid] = valid ? cell_coins(cell, st.t, d.key) : 0u;
    }
    settle_tile_roots<TX, TY, TZ, ALIGNED>(d, st, ti, tid, cell, hm, LAB, S.HL, S.wtot);
    double M[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) M[k] = 0.0;
    if (valid) {
        float r[NV];
        sweep_axis<NV>(d, st.t, r);
        uint32_t flipmask;
        if constexpr (ALIGNED) flipmask = cell_flip_mask_keyed<TX, TY, TZ, MODE>(lab, LAB, CB, d.lgL, ti, cell, tid);
        else flipmask = cell_flip_mask<NC>(lab, LAB, CB, ti, cell, tid, st.t, d.key);
        float v[NV][16];
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const float4 *S4 = reinterpret_cast<const float4 *>(s + (int64_t)k * N) + 4 * (int64_t)cell;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float4 a = S4[q];
                v[k][4 * q] = a.x;
                v[k][4 * q + 1] = a.y;
                v[k][4 * q + 2] = a.z;
                v[k][4 * q + 3] = a.w;
            }
        }
        if (flipmask) {
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                if (!((flipmask >> q) & 1u)) continue;
                float a[NV];
#pragma unroll
                for (int k = 0; k < NV; ++k) a[k] = v[k][q];
                const float cc = -2.0f * project<NV>(a, r);
#pragma unroll
                for (int k = 0; k < NV; ++k) v[k][q] = __fmaf_rn(cc, r[k], v[k][q]);
            }
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                float4 *S4 = reinterpret_cast<float4 *>(s + (int64_t)k * N) + 4 * (int64_t)cell;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    S4[q] = make_float4(v[k][4 * q], v[k][4 * q + 1], v[k][4 * q + 2], v[k][4 * q + 3]);
            }
        }
#pragma unroll
        for (int k = 0; k < NV; ++k)
#pragma unroll
            for (int q = 0; q < 16; ++q) M[k] += (double)v[k][q];
    }
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double b = block_sum<double>(M[k], S.red);
        if (tid == 0) d.dpart[d.mpart_off * (1 + k) + tile] = b;
    }
}

template <int NV, int TX, int TY, int TZ>
__global__ __launch_bounds__(TX *TY *TZ) void k_settle_flip_on(Chain c)
{
    __shared__ OnFlipLds<TX, TY, TZ> S;
    const int rep = c.tile_rep[blockIdx.x];
    const RepState st = *c.state[rep];
    if (st.remaining <= 0) return;
    const RepDesc &d = c.desc[rep];
    if constexpr (TX % 8 == 0) {
        if (d.lgL >= 0) {
            on_settle_flip_pass<NV, TX, TY, TZ, kFlipPow2>(d, st, blockIdx.x - d.tile_base, threadIdx.x, S);
            return;
        }
        if (d.divisible) {
            on_settle_flip_pass<NV, TX, TY, TZ, kFlipDivisible>(d, st, blockIdx.x - d.tile_base, threadIdx.x, S);
            return;
        }
    }
    on_settle_flip_pass<NV, TX, TY, TZ, kFlipGeneral>(d, st, blockIdx.x - d.tile_base, threadIdx.x, S);
}

// Records and state (see k_finalize_ising).
template <int NV>
__global__ __launch_bounds__(kFinalizeThreads) void k_finalize_on(Chain c)
{
    __shared__ double red[16 * (1 + NV)];
    const int rep = blockIdx.x;
    const RepState st = *c.state[rep];
    if (st.remaining <= 0) return;
    const RepDesc &d = c.desc[rep];
    const int ntiles = d.ntx * d.nty * d.ntz;
    // the energy and the NV magnetisation sums, each in the order of one
    // block_sum of its own: their loads go out together and one barrier
    // serves all of them
    double v[1 + NV];
#pragma unroll
    for (int q = 0; q <= NV; ++q) v[q] = 0.0;
    for (int k = threadIdx.x; k < ntiles; k += blockDim.x) {
        v[0] += d.dpart[k];
#pragma unroll
        for (int q = 0; q < NV; ++q) v[1 + q] += d.dpart[d.mpart_off * (1 + q) + k];
    }
    block_sum_n<double, 1 + NV>(v, red);
    const double E = v[0];
    double M[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < NV; ++q) M[q] = v[1 + q];
    if (threadIdx.x == 0) {
        if (st.e_pending >= 0) d.ring[st.e_pending].E = -d.J * E;
        const int slot = st.ring_used;
        if (slot < d.ring_cap) {
            DevRecord rec;
            rec.sweep = st.t;
            rec.bond_sum = 0;
            rec.M_int = 0;
            rec.reserved = 0;
            rec.E = 0.0;
            rec.M[0] = M[0];
            rec.M[1] = M[1];
            rec.M[2] = M[2];
            const double m = sqrt(M[0] * M[0] + M[1] * M[1] + M[2] * M[2]) / (double)d.N;
            rec.m2 = m * m;
            rec.m4 = rec.m2 * rec.m2;
            d.ring[slot] = rec;
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
template <int NV>
__global__ __launch_bounds__(kBlock) void k_energy_on(Chain c)
{
    __shared__ double red[16];
    const int rep = c.cblk_rep[blockIdx.x];
    if (c.state[rep]->e_pending < 0) return;
    const RepDesc &d = c.desc[rep];
    const int blk = blockIdx.x - d.cblk_base;
    const int64_t cl = (int64_t)blk * kBlock + threadIdx.x;
    const float *__restrict__ s = (const float *)d.spins;
    const int64_t N = d.N;
    double esum = 0.0;
    if (cl < d.ncell) {
        const CellNbrs nb = cell_neighbours((int)cl, d.L);
#pragma unroll
        for (int j = 0; j < 48; ++j) {
            const SiteRef A = bond_end_a(j), B = bond_end_b(j);
            const int64_t ia = 16 * (int64_t)nb.c[A.cell] + A.site, ib = 16 * (int64_t)nb.c[B.cell] + B.site;
            double dd = 0.0;
#pragma unroll
            for (int k = 0; k < NV; ++k) dd += (double)s[k * N + ia] * (double)s[k * N + ib];
            esum += dd;
        }
    }
    const double b = block_sum<double>(esum, red);
    if (threadIdx.x == 0) d.dpart[d.tail_off + blk] = b;
}

__global__ __launch_bounds__(kBlock) void k_energy_tail_finalize_on(Chain c)
{
    __shared__ double red[16];
    const int rep = blockIdx.x;
    const RepState st = *c.state[rep];
    if (st.e_pending < 0) return;
    const RepDesc &d = c.desc[rep];
    const int ncb = blocks_for(d.ncell);
    double E = 0.0;
    for (int k = threadIdx.x; k < ncb; k += blockDim.x) E += d.dpart[d.tail_off + k];
    E = block_sum<double>(E, red);
    if (threadIdx.x == 0) {
        d.ring[st.e_pending].E = -d.J * E;
        c.state[rep]->e_pending = -1;
    }
}

template <int NV>
struct OnLocal {
    template <int TX, int TY, int TZ>
    static hipError_t run(const Chain &c, hipStream_t st, const LaunchHook &hook)
    {
        PYRO_LAUNCH(kKLocal, (k_local_on<NV, TX, TY, TZ>), c.ntile_blocks, TX * TY * TZ, c);
        return hipSuccess;
    }
};

template <int NV>
struct OnFlip {
    template <int TX, int TY, int TZ>
    static hipError_t run(const Chain &c, hipStream_t st, const LaunchHook &hook)
    {
        PYRO_LAUNCH(kKFlip, (k_settle_flip_on<NV, TX, TY, TZ>), c.ntile_blocks, TX * TY * TZ, c);
        return hipSuccess;
    }
};

template <int NV>
static hipError_t sweep_on(const Chain &c, hipStream_t st, const LaunchHook &hook)
{
    hipError_t e = with_tile_shape<OnLocal<NV>>(c.shape, c, st, hook);
    if (e == hipSuccess) e = launch_unite(c, st, hook);
    if (e == hipSuccess) e = with_tile_shape<OnFlip<NV>>(c.shape, c, st, hook);
    if (e != hipSuccess) return e;
    PYRO_LAUNCH(kKFinalize, k_finalize_on<NV>, c.nreps, kFinalizeThreads, c);
    return hipSuccess;
}

hipError_t launch_on_sweep(const Chain &c, hipStream_t st, const LaunchHook &hook)
{
    return c.model == 2 ? sweep_on<2>(c, st, hook) : sweep_on<3>(c, st, hook);
}

template <int NV>
static hipError_t energy_tail_on(const Chain &c, hipStream_t st, const LaunchHook &hook)
{
    PYRO_LAUNCH(kKEnergy, k_energy_on<NV>, c.ncell_blocks, kBlock, c);
    PYRO_LAUNCH(kKFinalize, k_energy_tail_finalize_on, c.nreps, kBlock, c);
    return hipSuccess;
}

hipError_t launch_on_energy_tail(const Chain &c, hipStream_t st, const LaunchHook &hook)
{
    return c.model == 2 ? energy_tail_on<2>(c, st, hook) : energy_tail_on<3>(c, st, hook);
}

}  // namespace pyro
