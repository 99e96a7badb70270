// Swendsen-Wang sweep on any graph given as a bond list (nearest-neighbour
// table): the paper's remark that the algorithm carries over to other
// lattices once a nearest-neighbour table is supplied (Sec. 2, Sec. 4).
//
// No lattice tiles: windows of 4096 sites, and one thread per bond or per
// site.  Per sweep:
//   O(n) only  k_graph_prepare    sigma_i = s_i . r (each workgroup draws the
//                                 sweep's embedding axis r itself)
//              k_graph_local      sites cut into windows of 4096, one
//                                 workgroup each: activation of the bonds with
//                                 both ends in the window and their union in
//                                 LDS; every site stores its local root
//              k_graph_cross      activation of the bonds between windows and
//                                 union of their ends in the global forest
//                                 (index linking: the larger root is hooked
//                                 under the smaller by compare-and-swap, so
//                                 every tree root is its cluster's smallest
//                                 site)
//              k_graph_flip       root of each site (pointer chase, written
//                                 back), flip coin of the root, flip or
//                                 reflection, magnetisation partials
//              k_graph_energy     bond sums of the new state, partials
//              k_graph_finalize   fixed-order sums into the sweep's record
// Random numbers, thresholds and FP32 operation order are those of the
// pyrochlore sweep with bond b = position in the list and site i = index:
//   Ising: r32(b) = byte (b mod 16) of Philox(b/16, t, BOND) << 24 | low 24
//          bits of word (b mod 4) of Philox(b/4, t, BOND_LO); active iff the
//          spins are equal and nonzero and r32 < thr;
//   O(n):  r32(b) = word (b mod 4) of Philox(b/4, t, BOND);
//   coin:  bit (r mod 32) of word ((r/32) mod 4) of Philox(r/128, t, FLIP).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <deque>
#include <new>
#include <string>
#include <vector>

#include "../../include/pyro_sw.h"
#include "device_util.hpp"
#include "kernels.hpp"
#include "lattice.hpp"
#include "on_bond.hpp"
#include "philox.hpp"
#include "unit_vector.hpp"

namespace pyro {
namespace {

constexpr int kGraphRing = 1024;  // device records between drains

struct GraphDesc {
    int64_t N, NB;
    int64_t n_cross;  // bonds between windows (the last n_cross of the bond arrays)
    int n;  // 1 Ising, 2 XY, 3 Heisenberg
    const int32_t *ba, *bb;  // bond ends: bonds inside one site window first, grouped by window,
                             // then the bonds between windows
    const uint32_t *bond_id; // position of each bond in the caller's table (keys its draws)
    const int64_t *wstart;   // [nwin + 1] first bond of each window; wstart[nwin] = first bond between windows
    const int32_t *wsite;    // [N] window w holds the sites wsite[w kWindow ..], ascending within the
                             // window; NULL: window w holds the indices w kWindow ..
    const uint16_t *la, *lb; // bonds inside a window: positions of their ends in the window
    void *spins;  // int8 [N] or float [n][N]
    int32_t *label;
    float *sigma;  // O(n) projections [N]
    int64_t *ipart;  // Ising partials: [kPartBlocks bond blocks][kPartBlocks site blocks]
    double *dpart;   // O(n) partials: [kPartBlocks bond blocks][3][kPartBlocks site blocks]
    DevRecord *ring;
    unsigned long long *eacc;  // Ising: bond sum of the state entering the sweep, summed by the union
                               // passes; the finalize moves it into the record and clears it
    uint32_t thr_hi, thr_lo;  // Ising threshold split at bit 24
    float x0;
    double J;
    PhiloxKey key;
};

__device__ __forceinline__ int32_t lab_get(const int32_t *lab, int32_t x)
{
    return __hip_atomic_load(const_cast<int32_t *>(lab) + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x: parents are never larger than their children, so the chase
// ends.  Read only: in the flip pass every thread writes only its own site's
// entry, so the final labels are all roots.  (Halving the path during the
// union pass was measured slower: its extra stores cost more than the
// shorter chases save.)
__device__ __forceinline__ int32_t graph_root(const int32_t *lab, int32_t x)
{
    for (;;) {
        const int32_t p = lab_get(lab, x);
        if (p == x) return x;
        x = p;
    }
}

__device__ void graph_unite(int32_t *lab, int32_t a, int32_t b)
{
    for (;;) {
        a = graph_root(lab, a);
        b = graph_root(lab, b);
        if (a == b) return;
        if (a < b) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        int32_t expected = a;
        if (__hip_atomic_compare_exchange_strong(lab + a, &expected, b, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            return;
        a = expected;  // hooked meanwhile: continue from its new parent
    }
}

__device__ __forceinline__ uint32_t coin_of(int32_t r, uint32_t t, PhiloxKey key)
{
    const uint4 w = philox4x32_10((uint32_t)r >> 7, t, kStreamFlip, 0u, key);
    return (word_of(w, ((uint32_t)r >> 5) & 3u) >> (r & 31)) & 1u;
}

// Embedding axis of sweep t into LDS, drawn by the workgroup's first thread
// (a kernel of its own for it cost a launch per sweep).  Every thread of
// the workgroup must call it.
__device__ __forceinline__ void graph_axis(const GraphDesc &g, uint32_t t, float *ax)
{
    if (threadIdx.x == 0) unit_vector(0u, t, kStreamAxis, g.n, g.key, ax);
    __syncthreads();
}

__global__ __launch_bounds__(kBlock) void k_graph_prepare(GraphDesc g, uint32_t t)
{
    __shared__ float ax[3];
    graph_axis(g, t, ax);
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.N) return;
    const float *s = (const float *)g.spins;
    const float r[3] = {ax[0], ax[1], ax[2]};
    const float v[3] = {s[i], s[g.N + i], g.n == 3 ? s[2 * g.N + i] : 0.0f};
    g.sigma[i] = g.n == 2 ? project<2>(v, r) : project<3>(v, r);
}

// Activation of bond b (its position in the caller's table) between sites
// i and j in sweep t.
__device__ __forceinline__ bool ising_bond_active(const GraphDesc &g, uint32_t b, int8_t si, int8_t sj, uint32_t t)
{
    if (si != sj || si == 0) return false;
    const uint4 w = philox4x32_10(b >> 4, t, kStreamBond, 0u, g.key);
    const uint32_t k = b & 15u;
    const uint32_t hi = (word_of(w, k >> 2) >> (8 * (k & 3u))) & 0xFFu;
    if (hi != g.thr_hi) return hi < g.thr_hi;
    const uint4 v = philox4x32_10(b >> 2, t, kStreamBondLo, 0u, g.key);
    return (word_of(v, b & 3u) & 0xFFFFFFu) < g.thr_lo;
}

// Activation of bond b between sites i and j; for Ising, *e gains s_i s_j of
// the state entering the sweep (the energy of the previous record).
__device__ __forceinline__ bool graph_bond_active(const GraphDesc &g, uint32_t b, int32_t i, int32_t j, uint32_t t,
                                                  int64_t *e)
{
    if (g.n == 1) {
        const int8_t *s = (const int8_t *)g.spins;
        const int8_t si = s[i], sj = s[j];
        *e += (int64_t)si * (int64_t)sj;
        return ising_bond_active(g, b, si, sj, t);
    }
    const float x = __fmul_rn(__fmul_rn(g.x0, g.sigma[i]), g.sigma[j]);
    const uint4 w = philox4x32_10(b >> 2, t, kStreamBond, 0u, g.key);
    return on_bond_active(x, word_of(w, b & 3u));
}

// Ising: add a block's bond sum to the sweep's accumulator (integer, so the
// order of the additions does not matter).
__device__ __forceinline__ void add_bond_sum(const GraphDesc &g, int64_t e, int64_t *red)
{
    if (g.n != 1) return;
    const int64_t bs = block_sum<int64_t>(e, red);
    if (threadIdx.x == 0 && bs != 0)
        __hip_atomic_fetch_add(g.eacc, (unsigned long long)bs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sites are cut into windows of kWindow sites (the last may hold fewer):
// either consecutive indices, or, where that cuts fewer bonds, balls grown
// breadth first over the bond table (set-up, graph_windows).  Bonds with
// both ends in one window are grouped (at set-up) by window.
constexpr int kWindow = 4096;
constexpr int kLocalThreads = 512;  // threads of the window pass

__device__ __forceinline__ int lds_root(const int *P, int x)
{
    for (;;) {
        const int p = __hip_atomic_load(P + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (p == x) return x;
        x = p;
    }
}

// One workgroup per window: union of the active bonds with both ends in the
// window in LDS (index linking with atomic min, so each local root is the
// smallest site of its local component), then every site of the window
// stores the global index of its local root.
__global__ __launch_bounds__(kLocalThreads) void k_graph_local(GraphDesc g, uint32_t t)
{
    __shared__ int P[kWindow];
    __shared__ float SG[kWindow];  // the window's spins (Ising, as float) or projections (O(n))
    __shared__ int64_t red[16];
    const int64_t base = (int64_t)blockIdx.x * kWindow;
    const int nloc = (int)std::min<int64_t>(kWindow, g.N - base);
    const int32_t *ws = g.wsite ? g.wsite + base : nullptr;  // uniform
    for (int k = threadIdx.x; k < nloc; k += kLocalThreads) {
        const int64_t i = ws ? (int64_t)ws[k] : base + k;
        P[k] = k;
        SG[k] = g.n == 1 ? (float)((const int8_t *)g.spins)[i] : g.sigma[i];
    }
    __syncthreads();
    const int64_t b1 = g.wstart[blockIdx.x + 1];
    int64_t e = 0;
    for (int64_t q = g.wstart[blockIdx.x] + threadIdx.x; q < b1; q += kLocalThreads) {
        int a = g.la[q], b = g.lb[q];
        const float vi = SG[a], vj = SG[b];
        const uint32_t bid = g.bond_id[q];
        bool active;
        if (g.n == 1) {
            const int8_t si = (int8_t)vi, sj = (int8_t)vj;
            e += (int64_t)si * (int64_t)sj;
            active = ising_bond_active(g, bid, si, sj, t);
        } else {
            const float x = __fmul_rn(__fmul_rn(g.x0, vi), vj);
            const uint4 w = philox4x32_10(bid >> 2, t, kStreamBond, 0u, g.key);
            active = on_bond_active(x, word_of(w, bid & 3u));
        }
        if (!active) continue;
        for (;;) {
            a = lds_root(P, a);
            b = lds_root(P, b);
            if (a == b) break;
            if (a < b) {
                const int x = a;
                a = b;
                b = x;
            }
            const int old = __hip_atomic_fetch_min(P + a, b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (old == a) break;
            a = old;
        }
    }
    __syncthreads();
    // Positions ascend with site index inside a window, so the smallest
    // position of a component is its smallest site.
    for (int k = threadIdx.x; k < nloc; k += kLocalThreads) {
        const int r = lds_root(P, k);
        if (ws)
            g.label[ws[k]] = ws[r];
        else
            g.label[base + k] = (int32_t)(base + r);
    }
    add_bond_sum(g, e, red);
}

// Bonds whose ends lie in different windows: union in the global forest of
// local roots (after every window has stored its labels).
__global__ __launch_bounds__(kBlock) void k_graph_cross(GraphDesc g, uint32_t t)
{
    __shared__ int64_t red[16];
    const int64_t first = g.wstart[(g.N + kWindow - 1) / kWindow];
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    int64_t e = 0;
    for (int64_t q = first + (int64_t)blockIdx.x * kBlock + threadIdx.x; q < g.NB; q += stride) {
        const int32_t i = g.ba[q], j = g.bb[q];
        if (graph_bond_active(g, g.bond_id[q], i, j, t, &e)) graph_unite(g.label, i, j);
    }
    add_bond_sum(g, e, red);
}

// The flip and energy passes run a fixed grid of at most kPartBlocks blocks
// that stride over their sites or bonds, so the record is a fixed-order sum
// of at most 2 kPartBlocks partials: ipart / dpart hold the bond partials at
// [0, kPartBlocks) and the site partials (O(n): per component) after them.
constexpr int kPartBlocks = 2048;

__host__ __device__ inline int part_grid(int64_t n) { return (int)std::min<int64_t>(blocks_for(n), kPartBlocks); }

__global__ __launch_bounds__(kBlock) void k_graph_flip(GraphDesc g, uint32_t t)
{
    __shared__ int64_t ired[16];
    __shared__ double dred[16];
    __shared__ float ax[3];
    if (g.n > 1) graph_axis(g, t, ax);  // uniform branch
    int64_t m = 0;
    double mv[3] = {0.0, 0.0, 0.0};
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < g.N; i += stride) {
        const int32_t r = graph_root(g.label, (int32_t)i);
        g.label[i] = r;
        const uint32_t c = coin_of(r, t, g.key);
        if (g.n == 1) {
            int8_t *s = (int8_t *)g.spins;
            int8_t v = s[i];
            if (c) {
                v = (int8_t)-v;
                s[i] = v;
            }
            m += v;
        } else {
            float *s = (float *)g.spins;
            const float cf = __fmul_rn(-2.0f, g.sigma[i]);
            for (int k = 0; k < g.n; ++k) {
                float v = s[(int64_t)k * g.N + i];
                if (c) {
                    v = __fmaf_rn(cf, ax[k], v);
                    s[(int64_t)k * g.N + i] = v;
                }
                mv[k] += (double)v;
            }
        }
    }
    if (g.n == 1) {
        const int64_t bs = block_sum<int64_t>(m, ired);
        if (threadIdx.x == 0) g.ipart[kPartBlocks + blockIdx.x] = bs;
    } else {
        for (int k = 0; k < 3; ++k) {
            const double bs = block_sum<double>(mv[k], dred);
            if (threadIdx.x == 0) g.dpart[kPartBlocks + k * kPartBlocks + blockIdx.x] = bs;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_graph_energy(GraphDesc g)
{
    __shared__ int64_t ired[16];
    __shared__ double dred[16];
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const int64_t b0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g.n == 1) {
        const int8_t *s = (const int8_t *)g.spins;
        int64_t e = 0;
        for (int64_t b = b0; b < g.NB; b += stride) e += (int64_t)s[g.ba[b]] * (int64_t)s[g.bb[b]];
        const int64_t bs = block_sum<int64_t>(e, ired);
        if (threadIdx.x == 0) g.ipart[blockIdx.x] = bs;
    } else {
        const float *s = (const float *)g.spins;
        double e = 0.0;
        for (int64_t b = b0; b < g.NB; b += stride) {
            const int32_t i = g.ba[b], j = g.bb[b];
            for (int k = 0; k < g.n; ++k) e += (double)s[(int64_t)k * g.N + i] * (double)s[(int64_t)k * g.N + j];
        }
        const double bs = block_sum<double>(e, dred);
        if (threadIdx.x == 0) g.dpart[blockIdx.x] = bs;
    }
}

__global__ __launch_bounds__(kBlock) void k_graph_finalize(GraphDesc g, uint32_t t, int slot)
{
    __shared__ int64_t ired[16];
    __shared__ double dred[16];
    const int nbp = g.NB > 0 ? part_grid(g.NB) : 0, nsp = part_grid(g.N);
    DevRecord r{};
    r.sweep = t;
    if (g.n == 1) {
        // The bond sum of this record's state is counted by the next sweep's
        // union passes (or by the tail pass at a drain); the host moves it
        // in.  `reserved` carries the bond sum of the state entering this
        // sweep, which belongs to the previous record.
        int64_t M = 0;
        for (int k = threadIdx.x; k < nsp; k += kBlock) M += g.ipart[kPartBlocks + k];
        M = block_sum<int64_t>(M, ired);
        if (threadIdx.x == 0) {
            r.reserved = (int64_t)*g.eacc;
            *g.eacc = 0ull;
            r.M_int = M;
            r.M[0] = (double)M;
            const double mm = (double)M / (double)g.N;
            r.m2 = mm * mm;
            r.m4 = r.m2 * r.m2;
            g.ring[slot] = r;
        }
    } else {
        double S = 0.0, M[3] = {0.0, 0.0, 0.0};
        for (int k = threadIdx.x; k < nbp; k += kBlock) S += g.dpart[k];
        for (int c = 0; c < 3; ++c)
            for (int k = threadIdx.x; k < nsp; k += kBlock) M[c] += g.dpart[kPartBlocks + c * kPartBlocks + k];
        S = block_sum<double>(S, dred);
        for (int c = 0; c < 3; ++c) M[c] = block_sum<double>(M[c], dred);
        if (threadIdx.x == 0) {
            r.E = -g.J * S;
            r.M[0] = M[0];
            r.M[1] = M[1];
            r.M[2] = M[2];
            const double mm = sqrt(M[0] * M[0] + M[1] * M[1] + M[2] * M[2]) / (double)g.N;
            r.m2 = mm * mm;
            r.m4 = r.m2 * r.m2;
            g.ring[slot] = r;
        }
    }
}

// Ising: bond sum of the current state into ring[kGraphRing].bond_sum (the
// energy of the last record, read at a drain).
__global__ __launch_bounds__(kBlock) void k_graph_bond_total(GraphDesc g)
{
    __shared__ int64_t ired[16];
    const int nbp = g.NB > 0 ? part_grid(g.NB) : 0;
    int64_t E = 0;
    for (int k = threadIdx.x; k < nbp; k += kBlock) E += g.ipart[k];
    E = block_sum<int64_t>(E, ired);
    if (threadIdx.x == 0) g.ring[kGraphRing].bond_sum = E;
}

hipError_t launch_graph_bond_total(const GraphDesc &g, hipStream_t st)
{
    if (g.NB > 0) k_graph_energy<<<part_grid(g.NB), kBlock, 0, st>>>(g);
    k_graph_bond_total<<<1, kBlock, 0, st>>>(g);
    return hipGetLastError();
}

hipError_t launch_graph_sweep(const GraphDesc &g, uint32_t t, int slot, hipStream_t st)
{
    const int nsb = blocks_for(g.N), nbb = blocks_for(g.NB);
    if (g.n > 1) {
        k_graph_prepare<<<nsb, kBlock, 0, st>>>(g, t);
    }
    k_graph_local<<<blocks_for(g.N, kWindow), kLocalThreads, 0, st>>>(g, t);
    // the cross pass writes no partials (its bond sum goes to an atomic), so
    // its grid may exceed kPartBlocks: more bonds in flight hide the chases
    if (g.n_cross > 0)
        k_graph_cross<<<(int)std::min<int64_t>(blocks_for(g.n_cross), 8 * kPartBlocks), kBlock, 0, st>>>(g, t);
    k_graph_flip<<<part_grid(g.N), kBlock, 0, st>>>(g, t);
    if (nbb > 0 && g.n > 1) k_graph_energy<<<part_grid(g.NB), kBlock, 0, st>>>(g);
    k_graph_finalize<<<1, kBlock, 0, st>>>(g, t, slot);
    return hipGetLastError();
}

int gfail(int status, const std::string &msg) { return record_error(status, msg.c_str()); }

}  // namespace
}  // namespace pyro

using namespace pyro;

struct pyro_sw_graph {
    int model = 0;
    int64_t N = 0, NB = 0;
    double T = 0, J = 0;
    uint64_t seed = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false, broken = false;
    char *mem = nullptr;  // one device allocation for everything
    GraphDesc d{};
    uint32_t t = 0;       // global index of the next sweep
    int ring_used = 0;
    std::deque<pyro_sw_record> host_q;
};

namespace {

int gdevice(pyro_sw_graph *g, hipError_t e, const char *what)
{
    g->broken = true;
    (void)hipGetLastError();
    return gfail(PYRO_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define GHIP(call)                                       \
    do {                                                 \
        hipError_t e__ = (call);                         \
        if (e__ != hipSuccess) return gdevice(g, e__, #call); \
    } while (0)

int gusable(const pyro_sw_graph *g)
{
    if (!g) return gfail(PYRO_EINVAL, "graph is NULL");
    if (g->broken) return gfail(PYRO_ESTATE, "graph had a device error");
    return PYRO_OK;
}

void graph_params(pyro_sw_graph *g, double T)
{
    g->T = T;
    const double twobj = 2.0 * g->J / T;
    const uint64_t thr = (uint64_t)floor(-expm1(-twobj) * 4294967296.0);
    g->d.thr_hi = (uint32_t)(thr >> 24);
    g->d.thr_lo = (uint32_t)(thr & 0xFFFFFFu);
    g->d.x0 = (float)twobj;
}

int graph_drain(pyro_sw_graph *g)
{
    if (g->ring_used == 0) return PYRO_OK;
    std::vector<pyro_sw_record> tmp((size_t)g->ring_used);
    GHIP(hipStreamSynchronize(g->stream));
    GHIP(hipMemcpy(tmp.data(), g->d.ring, sizeof(DevRecord) * tmp.size(), hipMemcpyDeviceToHost));
    if (g->model == PYRO_ISING) {
        // Record k's bond sum was counted by sweep k + 1 (its `reserved`);
        // the last one is counted now, from the current state.
        int64_t tail = 0;
        GHIP(launch_graph_bond_total(g->d, g->stream));
        GHIP(hipStreamSynchronize(g->stream));
        GHIP(hipMemcpy(&tail, &g->d.ring[kGraphRing].bond_sum, sizeof(int64_t), hipMemcpyDeviceToHost));
        for (size_t k = 0; k < tmp.size(); ++k) {
            const int64_t b = k + 1 < tmp.size() ? tmp[k + 1].reserved : tail;
            tmp[k].bond_sum = b;
            tmp[k].E = -g->J * (double)b;
        }
        for (auto &r : tmp) r.reserved = 0;
    }
    for (const auto &r : tmp) g->host_q.push_back(r);
    g->ring_used = 0;
    return PYRO_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Windows as balls grown breadth first over the bond table: window w takes
// sites in breadth-first order from the smallest site not yet taken until it
// holds kWindow sites (a component that runs out continues from the next
// smallest free site), so every window but the last is full.  On a lattice
// numbered row by row, consecutive indices make thin slabs whose faces cut
// many bonds (a third of the simple cubic's at L = 256); balls cut about a
// third as many.  The balls are kept only when they cut fewer bonds than
// consecutive windows.  Then wsite lists each window's sites in ascending
// order, win gives each site's window and pos its position in it; otherwise
// all three are left empty.  Windows change the work split only: labels are
// canonical and every draw is keyed by bond, site and sweep.
void graph_windows(int64_t N, int64_t NB, const int32_t *ba, const int32_t *bb, std::vector<int32_t> &wsite,
                   std::vector<int32_t> &win, std::vector<uint16_t> &pos)
{
    if (N <= kWindow || NB == 0) return;
    std::vector<int32_t> order;
    {
        std::vector<int64_t> off((size_t)N + 1, 0);
        for (int64_t k = 0; k < NB; ++k) {
            ++off[(size_t)ba[k] + 1];
            ++off[(size_t)bb[k] + 1];
        }
        for (int64_t i = 0; i < N; ++i) off[(size_t)i + 1] += off[(size_t)i];
        std::vector<int32_t> adj((size_t)(2 * NB));
        {
            std::vector<int64_t> cur(off.begin(), off.end() - 1);
            for (int64_t k = 0; k < NB; ++k) {
                adj[(size_t)cur[(size_t)ba[k]]++] = bb[k];
                adj[(size_t)cur[(size_t)bb[k]]++] = ba[k];
            }
        }
        win.assign((size_t)N, -1);
        order.reserve((size_t)N);
        std::vector<int32_t> queue;
        queue.reserve(kWindow);
        int32_t w = 0;
        int fill = 0;
        int64_t next = 0;
        auto take = [&](int32_t x) {  // true when the window is full
            win[(size_t)x] = w;
            order.push_back(x);
            if (++fill < kWindow) return false;
            ++w;
            fill = 0;
            return true;
        };
        while ((int64_t)order.size() < N) {
            while (win[(size_t)next] >= 0) ++next;
            queue.clear();
            queue.push_back((int32_t)next);
            bool full = take((int32_t)next);
            for (size_t h = 0; !full && h < queue.size(); ++h) {
                const int32_t x = queue[h];
                for (int64_t j = off[(size_t)x]; j < off[(size_t)x + 1] && !full; ++j) {
                    const int32_t y = adj[(size_t)j];
                    if (win[(size_t)y] < 0) {
                        queue.push_back(y);
                        full = take(y);
                    }
                }
            }
        }
    }
    int64_t cut_balls = 0, cut_runs = 0;
    for (int64_t k = 0; k < NB; ++k) {
        cut_balls += win[(size_t)ba[k]] != win[(size_t)bb[k]];
        cut_runs += ba[k] / kWindow != bb[k] / kWindow;
    }
    if (cut_balls >= cut_runs) {
        win.clear();
        return;
    }
    for (int64_t w0 = 0; w0 < N; w0 += kWindow)
        std::sort(order.begin() + w0, order.begin() + std::min<int64_t>(N, w0 + kWindow));
    pos.resize((size_t)N);
    for (int64_t q = 0; q < N; ++q) pos[(size_t)order[(size_t)q]] = (uint16_t)(q % kWindow);
    wsite.swap(order);
}

}  // namespace

extern "C" {

int pyro_sw_graph_init(pyro_sw_graph **out, int64_t n_sites, int64_t n_bonds, const int32_t *bond_a,
                       const int32_t *bond_b, int model, double T, double J, uint64_t seed, int start, void *stream)
{
    if (!out) return gfail(PYRO_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_sites < 1 || n_sites > (int64_t)INT32_MAX) return gfail(PYRO_EINVAL, "n_sites must be in [1, 2^31 - 1]");
    if (n_bonds < 0 || n_bonds > (int64_t)UINT32_MAX) return gfail(PYRO_EINVAL, "n_bonds must be in [0, 2^32 - 1]");
    if (n_bonds > 0 && (!bond_a || !bond_b)) return gfail(PYRO_EINVAL, "bond lists are NULL");
    if (model < PYRO_ISING || model > PYRO_HEISENBERG) return gfail(PYRO_EINVAL, "model must be 1, 2 or 3");
    if (!(T > 0.0)) return gfail(PYRO_EINVAL, "T must be > 0 (inf allowed)");
    if (!(J > 0.0) || isinf(J)) return gfail(PYRO_EINVAL, "J must be finite and > 0");
    if (start != PYRO_START_COLD && start != PYRO_START_RANDOM)
        return gfail(PYRO_EINVAL, "start must be PYRO_START_COLD or PYRO_START_RANDOM");
    for (int64_t k = 0; k < n_bonds; ++k)
        if (bond_a[k] < 0 || bond_a[k] >= n_sites || bond_b[k] < 0 || bond_b[k] >= n_sites || bond_a[k] == bond_b[k])
            return gfail(PYRO_EINVAL, "bond " + std::to_string(k) + " has an end out of range or joins a site to itself");
    pyro_sw_graph *g = new (std::nothrow) pyro_sw_graph();
    if (!g) return gfail(PYRO_ENOMEM, "graph handle");
    g->model = model;
    g->N = n_sites;
    g->NB = n_bonds;
    g->J = J;
    g->seed = seed;
    const size_t spin_bytes = model == PYRO_ISING ? (size_t)n_sites : sizeof(float) * model * (size_t)n_sites;
    // Bonds inside one window first, grouped by window (stable counting
    // sort), then the bonds between windows in table order; bond_id keeps
    // each one's position in the caller's table, and la / lb the positions of
    // an inside bond's ends in its window.
    const int64_t nwin = (n_sites + kWindow - 1) / kWindow;
    std::vector<int32_t> wsite, win;
    std::vector<uint16_t> pos;
    try {
        graph_windows(n_sites, n_bonds, bond_a, bond_b, wsite, win, pos);
    } catch (const std::bad_alloc &) {  // no host memory for the balls: consecutive windows
        wsite.clear();
        win.clear();
        pos.clear();
    }
    const bool balls = !wsite.empty();
    auto wof = [&](int32_t i) -> int64_t { return balls ? (int64_t)win[(size_t)i] : (int64_t)(i / kWindow); };
    auto pof = [&](int32_t i) -> uint16_t { return balls ? pos[(size_t)i] : (uint16_t)(i % kWindow); };
    std::vector<int64_t> wstart((size_t)nwin + 1, 0);
    std::vector<int32_t> ga((size_t)n_bonds), gb((size_t)n_bonds);
    std::vector<uint32_t> gid((size_t)n_bonds);
    auto inside = [&](int64_t k) { return wof(bond_a[k]) == wof(bond_b[k]); };
    for (int64_t k = 0; k < n_bonds; ++k)
        if (inside(k)) ++wstart[(size_t)wof(bond_a[k]) + 1];
    for (int64_t w = 0; w < nwin; ++w) wstart[(size_t)w + 1] += wstart[(size_t)w];
    const int64_t n_inside = wstart[(size_t)nwin];
    std::vector<uint16_t> hla((size_t)n_inside), hlb((size_t)n_inside);
    {
        std::vector<int64_t> cur(wstart.begin(), wstart.end() - 1);
        int64_t cross = n_inside;
        for (int64_t k = 0; k < n_bonds; ++k) {
            const bool in = inside(k);
            const int64_t q = in ? cur[(size_t)wof(bond_a[k])]++ : cross++;
            ga[(size_t)q] = bond_a[k];
            gb[(size_t)q] = bond_b[k];
            gid[(size_t)q] = (uint32_t)k;
            if (in) {
                hla[(size_t)q] = pof(bond_a[k]);
                hlb[(size_t)q] = pof(bond_b[k]);
            }
        }
    }
    win.clear();
    win.shrink_to_fit();
    pos.clear();
    pos.shrink_to_fit();
    constexpr int kParts = 14;
    size_t off[kParts], total = 0;
    const size_t sizes[kParts] = {sizeof(int32_t) * (size_t)n_bonds, sizeof(int32_t) * (size_t)n_bonds, spin_bytes,
                                  sizeof(int32_t) * (size_t)n_sites, model == PYRO_ISING ? 0 : sizeof(float) * (size_t)n_sites,
                                  sizeof(int64_t) * 2 * kPartBlocks, sizeof(double) * 4 * kPartBlocks,
                                  sizeof(DevRecord) * (kGraphRing + 1), sizeof(uint32_t) * (size_t)n_bonds,
                                  sizeof(int64_t) * (size_t)(nwin + 1), sizeof(unsigned long long),
                                  sizeof(int32_t) * wsite.size(), sizeof(uint16_t) * (size_t)n_inside,
                                  sizeof(uint16_t) * (size_t)n_inside};
    for (int k = 0; k < kParts; ++k) {
        off[k] = total;
        total += align256(sizes[k]);
    }
    if (stream) {
        g->stream = (hipStream_t)stream;
    } else {
        const hipError_t e = hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            delete g;
            return gfail(PYRO_EDEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
        }
        g->own_stream = true;
    }
    if (hipMalloc((void **)&g->mem, total) != hipSuccess) {
        (void)hipGetLastError();
        if (g->own_stream) hipStreamDestroy(g->stream);
        delete g;
        return gfail(PYRO_ENOMEM, "graph device memory");
    }
    GraphDesc &d = g->d;
    d.N = n_sites;
    d.NB = n_bonds;
    d.n_cross = n_bonds - n_inside;
    d.n = model;
    d.ba = (const int32_t *)(g->mem + off[0]);
    d.bb = (const int32_t *)(g->mem + off[1]);
    d.spins = g->mem + off[2];
    d.label = (int32_t *)(g->mem + off[3]);
    d.sigma = model == PYRO_ISING ? nullptr : (float *)(g->mem + off[4]);
    d.ipart = (int64_t *)(g->mem + off[5]);
    d.dpart = (double *)(g->mem + off[6]);
    d.ring = (DevRecord *)(g->mem + off[7]);
    d.bond_id = (const uint32_t *)(g->mem + off[8]);
    d.wstart = (const int64_t *)(g->mem + off[9]);
    d.eacc = (unsigned long long *)(g->mem + off[10]);
    d.wsite = balls ? (const int32_t *)(g->mem + off[11]) : nullptr;
    d.la = (const uint16_t *)(g->mem + off[12]);
    d.lb = (const uint16_t *)(g->mem + off[13]);
    d.J = J;
    d.key = philox_key(seed);
    graph_params(g, T);
    hipError_t e = hipMemcpy((void *)d.wstart, wstart.data(), sizeof(int64_t) * wstart.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(d.eacc, 0, sizeof(unsigned long long));
    if (e == hipSuccess && balls)
        e = hipMemcpy((void *)d.wsite, wsite.data(), sizeof(int32_t) * wsite.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && n_inside > 0)
        e = hipMemcpy((void *)d.la, hla.data(), sizeof(uint16_t) * (size_t)n_inside, hipMemcpyHostToDevice);
    if (e == hipSuccess && n_inside > 0)
        e = hipMemcpy((void *)d.lb, hlb.data(), sizeof(uint16_t) * (size_t)n_inside, hipMemcpyHostToDevice);
    if (n_bonds > 0) {
        if (e == hipSuccess)
            e = hipMemcpy((void *)d.ba, ga.data(), sizeof(int32_t) * (size_t)n_bonds, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy((void *)d.bb, gb.data(), sizeof(int32_t) * (size_t)n_bonds, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy((void *)d.bond_id, gid.data(), sizeof(uint32_t) * (size_t)n_bonds, hipMemcpyHostToDevice);
    }
    RepDesc rd{};
    rd.N = n_sites;
    rd.spins = d.spins;
    rd.label = d.label;
    rd.key = d.key;
    if (e == hipSuccess) e = launch_init(rd, model, start, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) {  // nothing is handed out: release what was taken
        (void)hipGetLastError();
        (void)hipStreamSynchronize(g->stream);
        hipFree(g->mem);
        if (g->own_stream) hipStreamDestroy(g->stream);
        delete g;
        return gfail(PYRO_EDEVICE, std::string("graph set-up: ") + hipGetErrorString(e));
    }
    *out = g;
    return PYRO_OK;
}

int pyro_sw_graph_sweep(pyro_sw_graph *g, int64_t n_sweeps)
{
    int rc = gusable(g);
    if (rc) return rc;
    if (n_sweeps < 0) return gfail(PYRO_EINVAL, "n_sweeps must be >= 0");
    if ((int64_t)g->t + n_sweeps > (int64_t)UINT32_MAX) return gfail(PYRO_EINVAL, "sweep index would pass 2^32 - 1");
    for (int64_t k = 0; k < n_sweeps; ++k) {
        if (g->ring_used == kGraphRing && (rc = graph_drain(g))) return rc;
        GHIP(launch_graph_sweep(g->d, g->t, g->ring_used, g->stream));
        ++g->ring_used;
        ++g->t;
    }
    return PYRO_OK;
}

int pyro_sw_graph_moments(pyro_sw_graph *g, pyro_sw_record *out, int64_t cap, int64_t *n_out)
{
    int rc = gusable(g);
    if (rc) return rc;
    if (!n_out || cap < 0 || (cap > 0 && !out)) return gfail(PYRO_EINVAL, "bad output arguments");
    if ((rc = graph_drain(g))) return rc;
    GHIP(hipStreamSynchronize(g->stream));
    int64_t n = 0;
    if (cap == 0) {
        *n_out = (int64_t)g->host_q.size();
        return PYRO_OK;
    }
    while (n < cap && !g->host_q.empty()) {
        out[n++] = g->host_q.front();
        g->host_q.pop_front();
    }
    *n_out = n;
    return PYRO_OK;
}

int pyro_sw_graph_get_spins(pyro_sw_graph *g, void *host, size_t bytes)
{
    int rc = gusable(g);
    if (rc) return rc;
    const size_t need = g->model == PYRO_ISING ? (size_t)g->N : sizeof(float) * g->model * (size_t)g->N;
    if (!host || bytes != need) return gfail(PYRO_EINVAL, "host buffer size must equal the spin array size");
    GHIP(hipStreamSynchronize(g->stream));
    GHIP(hipMemcpy(host, g->d.spins, need, hipMemcpyDeviceToHost));
    return PYRO_OK;
}

int pyro_sw_graph_set_spins(pyro_sw_graph *g, const void *host, size_t bytes, int64_t next_sweep)
{
    int rc = gusable(g);
    if (rc) return rc;
    const size_t need = g->model == PYRO_ISING ? (size_t)g->N : sizeof(float) * g->model * (size_t)g->N;
    if (!host || bytes != need) return gfail(PYRO_EINVAL, "host buffer size must equal the spin array size");
    if (next_sweep < 0 || next_sweep > (int64_t)UINT32_MAX) return gfail(PYRO_EINVAL, "bad sweep index");
    if (g->model == PYRO_ISING) {
        const int8_t *s = (const int8_t *)host;
        for (int64_t i = 0; i < g->N; ++i)
            if (s[i] != 1 && s[i] != -1 && s[i] != 0) return gfail(PYRO_EINVAL, "Ising spins must be +1, -1 or 0 (vacant)");
    }
    GHIP(hipStreamSynchronize(g->stream));
    GHIP(hipMemcpy(g->d.spins, host, need, hipMemcpyHostToDevice));
    g->t = (uint32_t)next_sweep;
    g->ring_used = 0;
    g->host_q.clear();
    return PYRO_OK;
}

int pyro_sw_graph_get_labels(pyro_sw_graph *g, int32_t *host, size_t n)
{
    int rc = gusable(g);
    if (rc) return rc;
    if (!host || n != (size_t)g->N) return gfail(PYRO_EINVAL, "n must equal the number of sites");
    GHIP(hipStreamSynchronize(g->stream));
    GHIP(hipMemcpy(host, g->d.label, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    return PYRO_OK;
}

int pyro_sw_graph_set_temperature(pyro_sw_graph *g, double T)
{
    int rc = gusable(g);
    if (rc) return rc;
    if (!(T > 0.0)) return gfail(PYRO_EINVAL, "T must be > 0 (inf allowed)");
    GHIP(hipStreamSynchronize(g->stream));
    graph_params(g, T);
    return PYRO_OK;
}

int pyro_sw_graph_destroy(pyro_sw_graph *g)
{
    if (!g) return PYRO_OK;
    int rc = PYRO_OK;
    if (g->stream && hipStreamSynchronize(g->stream) != hipSuccess) rc = gfail(PYRO_EDEVICE, "synchronize failed");
    hipFree(g->mem);
    if (g->own_stream) hipStreamDestroy(g->stream);
    delete g;
    return rc;
}

int pyro_sw_bonds(int L, int32_t *bond_a, int32_t *bond_b, int64_t n)
{
    if (L < 1 || L > 406) return gfail(PYRO_EINVAL, "L must be in [1, 406]");
    if (!bond_a || !bond_b || n != 48 * (int64_t)L * L * L) return gfail(PYRO_EINVAL, "n must equal 48 L^3");
    const int64_t nc = (int64_t)L * L * L;
    for (int64_t c = 0; c < nc; ++c) {
        const CellNbrs nb = cell_neighbours((int)c, L);
        for (int j = 0; j < 48; ++j) {
            const SiteRef a = bond_end_a(j), b = bond_end_b(j);
            bond_a[48 * c + j] = 16 * nb.c[a.cell] + a.site;
            bond_b[48 * c + j] = 16 * nb.c[b.cell] + b.site;
        }
    }
    return PYRO_OK;
}

int pyro_sw_sc_bonds(int L, int32_t *bond_a, int32_t *bond_b, int64_t n)
{
    // L^3 sites below 2^31 and 3 L^3 bonds in an int64 count: L <= 1290.
    if (L < 1 || L > 1290) return gfail(PYRO_EINVAL, "L must be in [1, 1290]");
    const int64_t ns = (int64_t)L * L * L;
    if (!bond_a || !bond_b || n != 3 * ns) return gfail(PYRO_EINVAL, "n must equal 3 L^3");
    for (int64_t i = 0; i < ns; ++i) {
        const int64_t x = i % L, y = (i / L) % L, z = i / ((int64_t)L * L);
        const int64_t xp = x + 1 == L ? 0 : x + 1, yp = y + 1 == L ? 0 : y + 1, zp = z + 1 == L ? 0 : z + 1;
        bond_a[3 * i] = bond_a[3 * i + 1] = bond_a[3 * i + 2] = (int32_t)i;
        bond_b[3 * i] = (int32_t)((z * L + y) * L + xp);
        bond_b[3 * i + 1] = (int32_t)((z * L + yp) * L + x);
        bond_b[3 * i + 2] = (int32_t)((zp * L + y) * L + x);
    }
    return PYRO_OK;
}

}  // extern "C"
