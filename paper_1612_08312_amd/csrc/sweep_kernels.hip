// Swendsen-Wang sweep kernels for gfx950: bond activation, union-find
// cluster labeling, cluster flips and moment reductions, for the Ising model
// and the Wolff-embedded O(n) models on the pyrochlore lattice.
//
// Method (Sec. 1, Sec. 2 of the paper): every bond whose (projected) spins
// are parallel is activated with probability 1 - exp(-2 beta J s_i s_j);
// clusters are the connected components of the active bonds; each cluster
// is flipped (reflected through the plane normal to the sweep's random axis
// for n > 1) with probability 1/2.  Moments follow Eq. (1) and Eq. (2).
//
// Random draws (Philox4x32-10, counter = (unit, sweep, stream, attempt)):
//   Ising bond b: uniform r32 = byte (b mod 16) of BOND(b/16) << 24 | low 24
//     bits of word (b mod 4) of BOND_LO(b/4); active iff r32 < thr where
//     thr = floor((1 - exp(-2J/T)) 2^32).  The low call is made only when
//     the top byte ties with thr >> 24, which decides the same comparison.
//   O(n) bond b: r32 = word (b mod 4) of BOND(b/4), u = (r32 + 0.5) 2^-32,
//     active iff (double)x > -log1p(-u), x = (x0 * sigma_a) * sigma_b in
//     FP32, x0 = (float)(2J/T), sigma = s . r.
//   Flip coin of the cluster with smallest site r: bit (r mod 32) of word
//     ((r/32) mod 4) of FLIP(r/128).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "device_util.hpp"
#include "kernels.hpp"
#include "lattice.hpp"
#include "philox.hpp"

namespace pyro {

const char *kernel_name(int id)
{
    static const char *names[kNumKernels] = {"init",    "bonds",    "union",    "flip_table", "flip",
                                             "energy",  "finalize", "axis",     "project"};
    return (id >= 0 && id < kNumKernels) ? names[id] : "?";
}

// ---------------------------------------------------------------- init ---
__global__ __launch_bounds__(kBlock) void k_init_ising(int8_t *__restrict__ s, int64_t N, int start,
                                                       PhiloxKey key)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int8_t v = 1;
    if (start) {
        const uint4 w = philox4x32_10((uint32_t)(i >> 7), 0u, kStreamInit, 0u, key);
        v = ((word_of(w, (uint32_t)(i >> 5) & 3u) >> (i & 31)) & 1u) ? -1 : 1;
    }
    s[i] = v;
}

// Uniform unit n-vector by rejection from the cube (n = 2, 3); attempt a
// uses counter (c0, c1, stream, a); after 64 rejections the x unit vector.
__device__ void unit_vector(uint32_t c0, uint32_t c1, uint32_t stream, int n, PhiloxKey key,
                            float out[3])
{
    for (uint32_t a = 0; a < 64u; ++a) {
        const uint4 w = philox4x32_10(c0, c1, stream, a, key);
        const float v0 = (float)(int32_t)w.x * 0x1p-31f;
        const float v1 = (float)(int32_t)w.y * 0x1p-31f;
        const float v2 = (float)(int32_t)w.z * 0x1p-31f;
        float r2 = __fmul_rn(v0, v0);
        r2 = __fmaf_rn(v1, v1, r2);
        if (n == 3) r2 = __fmaf_rn(v2, v2, r2);
        if (r2 > 1e-12f && r2 <= 1.0f) {
            const float nr = sqrtf(r2);
            out[0] = v0 / nr;
            out[1] = v1 / nr;
            out[2] = n == 3 ? v2 / nr : 0.0f;
            return;
        }
    }
    out[0] = 1.0f;
    out[1] = 0.0f;
    out[2] = 0.0f;
}

__global__ __launch_bounds__(kBlock) void k_init_on(float *__restrict__ s, int64_t N, int n, int start,
                                                    PhiloxKey key)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    float v[3] = {1.0f, 0.0f, 0.0f};
    if (start) unit_vector((uint32_t)i, 0u, kStreamInit, n, key, v);
    for (int k = 0; k < n; ++k) s[(int64_t)k * N + i] = v[k];
}

__global__ __launch_bounds__(kBlock) void k_identity_labels(int32_t *__restrict__ label, int64_t N)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) label[i] = (int32_t)i;
}

// ------------------------------------------------------------- bonds ---
// Ising activation: one thread per cell, 48 bonds -> 48 mask bits.  Also
// resets the 16 labels of the cell to the identity forest.
__global__ __launch_bounds__(kBlock) void k_bonds_ising(const int8_t *__restrict__ s,
                                                        uint64_t *__restrict__ mask,
                                                        int32_t *__restrict__ label, int L, int ncell,
                                                        IsingParams p, PhiloxKey key, uint32_t t)
{
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= ncell) return;
    const CellNbrs nb = cell_neighbours(cell, L);
    int8_t own[16];
    {
        const int4 v = reinterpret_cast<const int4 *>(s)[cell];
        const int w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 16; ++k) own[k] = (int8_t)(w[k >> 2] >> (8 * (k & 3)));
    }
    int8_t dv[16];
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            const SiteRef r = down_vertex(f, mu);
            dv[4 * f + mu] = r.cell == kSelf ? own[r.site] : s[16 * nb.c[r.cell] + r.site];
        }
    uint4 rnd[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) rnd[q] = philox4x32_10(3u * (uint32_t)cell + q, t, kStreamBond, 0u, key);
    uint64_t m = 0;
#pragma unroll
    for (int j = 0; j < 48; ++j) {
        const int tet = j / 6, e = j % 6;
        const int8_t sa = tet < 4 ? own[4 * tet + pair_a(e)] : dv[4 * (tet - 4) + pair_a(e)];
        const int8_t sb = tet < 4 ? own[4 * tet + pair_b(e)] : dv[4 * (tet - 4) + pair_b(e)];
        if (sa == sb) {
            const uint32_t hi8 = (word_of(rnd[j >> 4], (j & 15) >> 2) >> (8 * (j & 3))) & 0xFFu;
            bool act = hi8 < p.thr_hi;
            if (hi8 == p.thr_hi) {
                const uint4 lo = philox4x32_10(12u * (uint32_t)cell + (j >> 2), t, kStreamBondLo, 0u, key);
                act = (word_of(lo, j & 3) & 0xFFFFFFu) < p.thr_lo;
            }
            m |= (uint64_t)act << j;
        }
    }
    mask[cell] = m;
    int4 *lab = reinterpret_cast<int4 *>(label + 16 * cell);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int base = 16 * cell + 4 * q;
        lab[q] = make_int4(base, base + 1, base + 2, base + 3);
    }
}

// O(n) activation on the projections sigma (one thread per cell).
__global__ __launch_bounds__(kBlock) void k_bonds_on(const float *__restrict__ sigma,
                                                     uint64_t *__restrict__ mask,
                                                     int32_t *__restrict__ label, int L, int ncell,
                                                     float x0, PhiloxKey key, uint32_t t)
{
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= ncell) return;
    const CellNbrs nb = cell_neighbours(cell, L);
    float own[16];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float4 v = reinterpret_cast<const float4 *>(sigma)[4 * cell + q];
        own[4 * q] = v.x;
        own[4 * q + 1] = v.y;
        own[4 * q + 2] = v.z;
        own[4 * q + 3] = v.w;
    }
    float dv[16];
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            const SiteRef r = down_vertex(f, mu);
            dv[4 * f + mu] = r.cell == kSelf ? own[r.site] : sigma[16 * nb.c[r.cell] + r.site];
        }
    uint64_t m = 0;
#pragma unroll
    for (int q = 0; q < 12; ++q) {
        const uint4 rnd = philox4x32_10(12u * (uint32_t)cell + q, t, kStreamBond, 0u, key);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int j = 4 * q + k;
            const int tet = j / 6, e = j % 6;
            const float sa = tet < 4 ? own[4 * tet + pair_a(e)] : dv[4 * (tet - 4) + pair_a(e)];
            const float sb = tet < 4 ? own[4 * tet + pair_b(e)] : dv[4 * (tet - 4) + pair_b(e)];
            const float x = __fmul_rn(__fmul_rn(x0, sa), sb);
            if (x > 0.0f) {
                const double u = ((double)word_of(rnd, k) + 0.5) * 0x1p-32;
                if ((double)x > -log1p(-u)) m |= (uint64_t)1 << j;
            }
        }
    }
    mask[cell] = m;
    int4 *lab = reinterpret_cast<int4 *>(label + 16 * cell);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int base = 16 * cell + 4 * q;
        lab[q] = make_int4(base, base + 1, base + 2, base + 3);
    }
}

// ------------------------------------------------------------- union ---
__global__ __launch_bounds__(kBlock) void k_union(const uint64_t *__restrict__ mask, int32_t *label, int L,
                                                  int ncell)
{
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= ncell) return;
    const uint64_t m = mask[cell];
    if (m == 0) return;
    const CellNbrs nb = cell_neighbours(cell, L);
#pragma unroll
    for (int j = 0; j < 48; ++j) {
        if (!((m >> j) & 1u)) continue;
        const SiteRef A = bond_end_a(j), B = bond_end_b(j);
        const int a = 16 * nb.c[A.cell] + A.site;
        const int b = 16 * nb.c[B.cell] + B.site;
        uf_unite(label, a, b);
    }
}

// --------------------------------------------------------------- flip ---
// 128 flip coins per Philox call: thread g writes words 4g..4g+3.
__global__ __launch_bounds__(kBlock) void k_flip_table(uint32_t *__restrict__ fb, int64_t ncalls,
                                                       PhiloxKey key, uint32_t t)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ncalls) return;
    reinterpret_cast<uint4 *>(fb)[g] = philox4x32_10((uint32_t)g, t, kStreamFlip, 0u, key);
}

__global__ __launch_bounds__(kBlock) void k_flip_ising(int8_t *__restrict__ s, int32_t *label,
                                                       const uint32_t *__restrict__ fb, int64_t N)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int r = uf_find(label, (int)i);
    const uint32_t bit = (fb[r >> 5] >> (r & 31)) & 1u;
    if (bit) s[i] = (int8_t)-s[i];
    label[i] = r;
}

__global__ __launch_bounds__(kBlock) void k_flip_on(float *__restrict__ s, const float *__restrict__ sigma,
                                                    int32_t *label, const uint32_t *__restrict__ fb,
                                                    const float *__restrict__ axis, int64_t N, int n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int r = uf_find(label, (int)i);
    const uint32_t bit = (fb[r >> 5] >> (r & 31)) & 1u;
    if (bit) {
        const float c = -2.0f * sigma[i];
        for (int k = 0; k < n; ++k) {
            float *p = s + (int64_t)k * N + i;
            *p = __fmaf_rn(c, axis[k], *p);
        }
    }
    label[i] = r;
}

// ------------------------------------------------------------ moments ---
// Ising: per cell M = sum of 16 spins and the bond sum over its 48 bonds.
__global__ __launch_bounds__(kBlock) void k_energy_ising(const int8_t *__restrict__ s, int L, int ncell,
                                                         int64_t *__restrict__ ipart, int nblk)
{
    __shared__ int64_t red[16];
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    int64_t M = 0, B = 0;
    if (cell < ncell) {
        const CellNbrs nb = cell_neighbours(cell, L);
        int8_t own[16];
        const int4 v = reinterpret_cast<const int4 *>(s)[cell];
        const int w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            own[k] = (int8_t)(w[k >> 2] >> (8 * (k & 3)));
            M += own[k];
        }
        int8_t dv[16];
#pragma unroll
        for (int f = 0; f < 4; ++f)
#pragma unroll
            for (int mu = 0; mu < 4; ++mu) {
                const SiteRef r = down_vertex(f, mu);
                dv[4 * f + mu] = r.cell == kSelf ? own[r.site] : s[16 * nb.c[r.cell] + r.site];
            }
        int bs = 0;
#pragma unroll
        for (int j = 0; j < 48; ++j) {
            const int tet = j / 6, e = j % 6;
            const int8_t sa = tet < 4 ? own[4 * tet + pair_a(e)] : dv[4 * (tet - 4) + pair_a(e)];
            const int8_t sb = tet < 4 ? own[4 * tet + pair_b(e)] : dv[4 * (tet - 4) + pair_b(e)];
            bs += sa * sb;
        }
        B = bs;
    }
    const int64_t Ms = block_sum<int64_t>(M, red);
    const int64_t Bs = block_sum<int64_t>(B, red);
    if (threadIdx.x == 0) {
        ipart[blockIdx.x] = Ms;
        ipart[nblk + blockIdx.x] = Bs;
    }
}

__global__ __launch_bounds__(kBlock) void k_finalize_ising(const int64_t *__restrict__ ipart, int nblk,
                                                           DevRecord *__restrict__ rec, int64_t sweep,
                                                           int64_t N, double J)
{
    __shared__ int64_t red[16];
    int64_t M = 0, B = 0;
    for (int k = threadIdx.x; k < nblk; k += blockDim.x) {
        M += ipart[k];
        B += ipart[nblk + k];
    }
    M = block_sum<int64_t>(M, red);
    B = block_sum<int64_t>(B, red);
    if (threadIdx.x == 0) {
        DevRecord r;
        r.sweep = sweep;
        r.bond_sum = B;
        r.M_int = M;
        r.reserved = 0;
        r.E = -J * (double)B;
        r.M[0] = (double)M;
        r.M[1] = 0.0;
        r.M[2] = 0.0;
        const double m = (double)M / (double)N;
        r.m2 = m * m;
        r.m4 = r.m2 * r.m2;
        *rec = r;
    }
}

// O(n): per cell the FP64 magnetisation of its 16 sites and the FP64 sum of
// s_a . s_b over its 48 bonds.
__global__ __launch_bounds__(kBlock) void k_energy_on(const float *__restrict__ s, int L, int ncell, int n,
                                                      int64_t N, double *__restrict__ dpart, int nblk)
{
    __shared__ double red[16];
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    double M[3] = {0.0, 0.0, 0.0}, S = 0.0;
    if (cell < ncell) {
        const CellNbrs nb = cell_neighbours(cell, L);
        for (int k = 0; k < n; ++k) {
            const float *sk = s + (int64_t)k * N;
            float own[16], dv[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                own[q] = sk[16 * cell + q];
                M[k] += (double)own[q];
            }
#pragma unroll
            for (int f = 0; f < 4; ++f)
#pragma unroll
                for (int mu = 0; mu < 4; ++mu) {
                    const SiteRef r = down_vertex(f, mu);
                    dv[4 * f + mu] = r.cell == kSelf ? own[r.site] : sk[16 * nb.c[r.cell] + r.site];
                }
#pragma unroll
            for (int j = 0; j < 48; ++j) {
                const int tet = j / 6, e = j % 6;
                const float sa = tet < 4 ? own[4 * tet + pair_a(e)] : dv[4 * (tet - 4) + pair_a(e)];
                const float sb = tet < 4 ? own[4 * tet + pair_b(e)] : dv[4 * (tet - 4) + pair_b(e)];
                S += (double)sa * (double)sb;
            }
        }
    }
    for (int k = 0; k < 3; ++k) {
        const double v = block_sum<double>(M[k], red);
        if (threadIdx.x == 0) dpart[(int64_t)k * nblk + blockIdx.x] = v;
    }
    const double v = block_sum<double>(S, red);
    if (threadIdx.x == 0) dpart[(int64_t)3 * nblk + blockIdx.x] = v;
}

__global__ __launch_bounds__(kBlock) void k_finalize_on(const double *__restrict__ dpart, int nblk,
                                                        DevRecord *__restrict__ rec, int64_t sweep,
                                                        int64_t N, double J)
{
    __shared__ double red[16];
    double acc[4];
    for (int q = 0; q < 4; ++q) {
        double v = 0.0;
        for (int k = threadIdx.x; k < nblk; k += blockDim.x) v += dpart[(int64_t)q * nblk + k];
        acc[q] = block_sum<double>(v, red);
    }
    if (threadIdx.x == 0) {
        DevRecord r;
        r.sweep = sweep;
        r.bond_sum = 0;
        r.M_int = 0;
        r.reserved = 0;
        r.E = -J * acc[3];
        r.M[0] = acc[0];
        r.M[1] = acc[1];
        r.M[2] = acc[2];
        const double m = sqrt(acc[0] * acc[0] + acc[1] * acc[1] + acc[2] * acc[2]) / (double)N;
        r.m2 = m * m;
        r.m4 = r.m2 * r.m2;
        *rec = r;
    }
}

// --------------------------------------------------------------- O(n) ---
__global__ void k_axis(float *__restrict__ axis, int n, PhiloxKey key, uint32_t t)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    float r[3];
    unit_vector(0u, t, kStreamAxis, n, key, r);
    axis[0] = r[0];
    axis[1] = r[1];
    axis[2] = r[2];
    axis[3] = 0.0f;
}

__global__ __launch_bounds__(kBlock) void k_project(const float *__restrict__ s, float *__restrict__ sigma,
                                                    const float *__restrict__ axis, int64_t N, int n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    float sig = __fmul_rn(s[i], axis[0]);
    sig = __fmaf_rn(s[N + i], axis[1], sig);
    if (n == 3) sig = __fmaf_rn(s[2 * N + i], axis[2], sig);
    sigma[i] = sig;
}

// ----------------------------------------------------------- launchers ---
#define PYRO_LAUNCH(id, kernel, grid, ...)                      \
    do {                                                        \
        if (hook.before) hook.before(hook.ctx, id);             \
        kernel<<<(grid), kBlock, 0, st>>>(__VA_ARGS__);         \
        if (hook.after) hook.after(hook.ctx, id);               \
        hipError_t e_ = hipGetLastError();                      \
        if (e_ != hipSuccess) return e_;                        \
    } while (0)

hipError_t launch_init_ising(const SweepBuffers &b, int start, PhiloxKey key, hipStream_t st)
{
    k_init_ising<<<blocks_for(b.N), kBlock, 0, st>>>((int8_t *)b.spins, b.N, start, key);
    return hipGetLastError();
}

hipError_t launch_init_on(const SweepBuffers &b, int n, int start, PhiloxKey key, hipStream_t st)
{
    k_init_on<<<blocks_for(b.N), kBlock, 0, st>>>((float *)b.spins, b.N, n, start, key);
    return hipGetLastError();
}

hipError_t launch_identity_labels(const SweepBuffers &b, hipStream_t st)
{
    k_identity_labels<<<blocks_for(b.N), kBlock, 0, st>>>(b.label, b.N);
    return hipGetLastError();
}

hipError_t launch_sweep_ising(const SweepBuffers &b, IsingParams p, double J, PhiloxKey key, uint32_t t,
                              int slot, hipStream_t st, const LaunchHook &hook)
{
    const int ncell = (int)b.ncell;
    const int gc = blocks_for(ncell);
    const int64_t ncalls = (b.N + 127) / 128;
    PYRO_LAUNCH(kKBonds, k_bonds_ising, gc, (const int8_t *)b.spins, b.mask, b.label, b.L, ncell, p, key, t);
    PYRO_LAUNCH(kKUnion, k_union, gc, b.mask, b.label, b.L, ncell);
    PYRO_LAUNCH(kKFlipTable, k_flip_table, blocks_for(ncalls), b.flipbits, ncalls, key, t);
    PYRO_LAUNCH(kKFlip, k_flip_ising, blocks_for(b.N), (int8_t *)b.spins, b.label, b.flipbits, b.N);
    PYRO_LAUNCH(kKEnergy, k_energy_ising, gc, (const int8_t *)b.spins, b.L, ncell, b.ipart, gc);
    PYRO_LAUNCH(kKFinalize, k_finalize_ising, 1, b.ipart, gc, b.ring + slot, (int64_t)t, b.N, J);
    return hipSuccess;
}

hipError_t launch_sweep_on(const SweepBuffers &b, int n, float x0, double J, PhiloxKey key, uint32_t t,
                           int slot, hipStream_t st, const LaunchHook &hook)
{
    const int ncell = (int)b.ncell;
    const int gc = blocks_for(ncell);
    const int64_t ncalls = (b.N + 127) / 128;
    PYRO_LAUNCH(kKAxis, k_axis, 1, b.axis, n, key, t);
    PYRO_LAUNCH(kKProject, k_project, blocks_for(b.N), (const float *)b.spins, b.sigma, b.axis, b.N, n);
    PYRO_LAUNCH(kKBonds, k_bonds_on, gc, b.sigma, b.mask, b.label, b.L, ncell, x0, key, t);
    PYRO_LAUNCH(kKUnion, k_union, gc, b.mask, b.label, b.L, ncell);
    PYRO_LAUNCH(kKFlipTable, k_flip_table, blocks_for(ncalls), b.flipbits, ncalls, key, t);
    PYRO_LAUNCH(kKFlip, k_flip_on, blocks_for(b.N), (float *)b.spins, b.sigma, b.label, b.flipbits, b.axis,
                b.N, n);
    PYRO_LAUNCH(kKEnergy, k_energy_on, gc, (const float *)b.spins, b.L, ncell, n, b.N, b.dpart, gc);
    PYRO_LAUNCH(kKFinalize, k_finalize_on, 1, b.dpart, gc, b.ring + slot, (int64_t)t, b.N, J);
    return hipSuccess;
}

}  // namespace pyro
