// C-ABI layer of the pyrochlore Swendsen-Wang library (declared in
// include/pyro_sw.h): argument checks, device memory, replica descriptors,
// groups of lattices swept together from one captured graph, the tile-shape
// autotuner, the per-sweep record rings, kernel timing and error state.
//
// No arithmetic of the method lives here except the two per-run constants of
// Sec. 2 that the kernels read: the Ising activation threshold
// floor((1 - exp(-2J/T)) 2^32) and the O(n) coupling x0 = (float)(2J/T).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/pyro_sw.h"
#include "kernels.hpp"
#include "lattice.hpp"
#include "resident.hpp"

using namespace pyro;

static_assert(sizeof(pyro_sw_record) == sizeof(DevRecord), "record layout");
static_assert(sizeof(pyro_sw_record) == 80, "record size");

namespace {
thread_local std::string g_last_error;
}  // namespace

int pyro::record_error(int status, const char *msg)
{
    g_last_error = msg;
    return status;
}

namespace {

int fail(int status, const std::string &msg) { return record_error(status, msg.c_str()); }

// Philox throughput probe: each thread draws the blocks i = gid, gid +
// stride, ... below `calls` and XOR-folds their words; each block writes its
// fold to out[blockIdx.x] (the host folds those).
__global__ __launch_bounds__(256) void k_philox_rate(uint64_t calls, PhiloxKey key, uint32_t *out)
{
    __shared__ uint32_t wf[4];
    uint32_t acc = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < calls; i += stride) {
        const uint4 r = philox4x32_10((uint32_t)i, 0x5EEDu, kStreamBond, 0u, key);
        acc ^= r.x ^ r.y ^ r.z ^ r.w;
    }
    for (int off = 32; off > 0; off >>= 1) acc ^= __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) wf[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = wf[0] ^ wf[1] ^ wf[2] ^ wf[3];
}

// Device atomic throughput probe.  Mode 0: every op loads a pseudo-random
// word of a[0 .. words) and compare-and-swaps it from the loaded value v to
// v + 1, as a forest hook does; each block adds its successful swaps to
// out[0], so that sum(a) = out[0] checks that no swap was lost.  Mode 1:
// every op adds 1 to a[0] (one address, as a work counter).
__global__ __launch_bounds__(256) void k_atomic_rate(int mode, uint32_t *a, uint64_t words, uint64_t ops,
                                                     unsigned long long *out)
{
    __shared__ unsigned long long ws[4];
    unsigned long long ok = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ops; i += stride) {
        if (mode == 0) {
            uint64_t h = (i + 1) * 0x9E3779B97F4A7C15ull;
            h ^= h >> 29;
            const uint64_t w = h % words;
            const uint32_t v = __hip_atomic_load(a + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ok += atomicCAS(a + w, v, v + 1u) == v;
        } else {
            atomicAdd(a, 1u);
            ++ok;
        }
    }
    for (int off = 32; off > 0; off >>= 1) ok += __shfl_xor(ok, off, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = ok;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(out, ws[0] + ws[1] + ws[2] + ws[3]);
}

__global__ __launch_bounds__(256) void k_sum_words(const uint32_t *a, uint64_t words, unsigned long long *out)
{
    __shared__ unsigned long long ws[4];
    unsigned long long v = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (uint64_t)gridDim.x * blockDim.x)
        v += a[i];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(out, ws[0] + ws[1] + ws[2] + ws[3]);
}

// Default tile shape for lattices of edge up to L (measured on MI355X):
// small lattices need smaller tiles to give every CU work.
int default_tile_shape(int L) { return L >= 96 ? kTile888 : (L >= 48 ? kTile884 : kTile844); }

constexpr int kRing = 16384;  // device records per lattice before a forced drain
constexpr int kMaxSlices = 8;  // concurrent slices of a group
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int64_t tiles_for(int L, int shape)
{
    const TileDims t = tile_dims(shape);
    return (int64_t)((L + t.x - 1) / t.x) * ((L + t.y - 1) / t.y) * ((L + t.z - 1) / t.z);
}

int64_t max_tiles(int L)
{
    int64_t m = 0;
    for (int s = 0; s < kNumTileShapes; ++s) m = std::max(m, tiles_for(L, s));
    return m;
}

struct Layout {
    size_t spin_bytes;
    size_t label, ipart, dpart, ring, pairs, state, solo_desc, solo_stp, solo_map, total;
    int64_t map_len;
};

Layout layout_for(int L, int model)
{
    const int64_t ncell = (int64_t)L * L * L;
    const int64_t N = 16 * ncell;
    Layout ly{};
    ly.spin_bytes = align_up(model == PYRO_ISING ? (size_t)N : sizeof(float) * (size_t)model * N);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += align_up(bytes);
        return at;
    };
    ly.label = take(sizeof(int32_t) * (size_t)N);
    ly.ipart = take(sizeof(int64_t) * (size_t)ipart_count(L));
    ly.dpart = take(model == PYRO_ISING ? 0 : sizeof(double) * (size_t)dpart_count(L));
    ly.ring = take(sizeof(pyro_sw_record) * (size_t)kRing);
    ly.pairs = take(sizeof(int) * (size_t)pair_list_ints(L));
    ly.state = take(sizeof(RepState));
    ly.solo_desc = take(sizeof(RepDesc));
    ly.solo_stp = take(sizeof(RepState *));
    ly.map_len = std::max<int64_t>(max_tiles(L), blocks_for(ncell));
    ly.solo_map = take(sizeof(int) * (size_t)ly.map_len);
    ly.total = off;
    return ly;
}

int check_args(int L, int model, double T, double J, int start)
{
    if (L < 1 || L > 406) return fail(PYRO_EINVAL, "L must be in [1, 406]");
    if (model < PYRO_ISING || model > PYRO_HEISENBERG) return fail(PYRO_EINVAL, "model must be 1, 2 or 3");
    if (!(T > 0.0)) return fail(PYRO_EINVAL, "T must be > 0 (inf allowed)");
    if (!(J > 0.0) || isinf(J)) return fail(PYRO_EINVAL, "J must be finite and > 0");
    if (start != PYRO_START_COLD && start != PYRO_START_RANDOM)
        return fail(PYRO_EINVAL, "start must be PYRO_START_COLD or PYRO_START_RANDOM");
    return PYRO_OK;
}

struct TimedLaunch {
    int id;
    hipEvent_t e0, e1;
};

// Kernel timing with HIP events (handles and groups each own one).
struct Timer {
    int mask = 0;
    hipStream_t stream = nullptr;
    std::vector<TimedLaunch> inflight;
    std::vector<hipEvent_t> pool;
    double ms[kNumKernels] = {};
    int64_t launches[kNumKernels] = {};

    hipEvent_t take()
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    static void before(void *ctx, int id)
    {
        Timer *t = (Timer *)ctx;
        if (!((t->mask >> id) & 1)) return;
        TimedLaunch tl{id, t->take(), t->take()};
        if (tl.e0 && tl.e1) {
            hipEventRecord(tl.e0, t->stream);
            t->inflight.push_back(tl);
        }
    }
    static void after(void *ctx, int id)
    {
        Timer *t = (Timer *)ctx;
        if (!((t->mask >> id) & 1)) return;
        if (!t->inflight.empty() && t->inflight.back().id == id) hipEventRecord(t->inflight.back().e1, t->stream);
    }
    LaunchHook hook() { return LaunchHook{before, after, this}; }
    hipError_t collect()
    {
        if (inflight.empty()) return hipSuccess;
        hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return e;
        for (auto &tl : inflight) {
            float v = 0.f;
            e = hipEventElapsedTime(&v, tl.e0, tl.e1);
            if (e != hipSuccess) return e;
            ms[tl.id] += v;
            launches[tl.id] += 1;
            pool.push_back(tl.e0);
            pool.push_back(tl.e1);
        }
        inflight.clear();
        return hipSuccess;
    }
    void reset(int m)
    {
        mask = m;
        for (int k = 0; k < kNumKernels; ++k) {
            ms[k] = 0.0;
            launches[k] = 0;
        }
    }
    void release()
    {
        for (auto &tl : inflight) {
            hipEventDestroy(tl.e0);
            hipEventDestroy(tl.e1);
        }
        inflight.clear();
        for (auto e : pool) hipEventDestroy(e);
        pool.clear();
    }
};

// Chain tables in device memory for a list of replicas of one model.
struct ChainTables {
    int model = 0, shape = kTile888;
    std::vector<pyro_sw *> reps;
    RepDesc *d_desc = nullptr;
    RepState **d_stp = nullptr;
    int *d_tile_rep = nullptr, *d_cblk_rep = nullptr;
    Chain chain{};
    int *d_ctl = nullptr;    // control words of a persistent launch (groups in persistent mode)
    int persist_grid = 0;    // workgroups of that launch
    bool owned = true;       // tables in `block` (groups) or in a workspace (solo)
    void *block = nullptr;   // stream-ordered allocation holding a group's tables
    hipStream_t stream = nullptr;
};

// Process-wide autotuning results: (model, multiset of L) -> tile shape.
struct TuneChoice {
    int shape;
    int ising_mode;  // Ising chains only
    bool resident;
};
std::mutex g_tune_mu;
std::map<std::string, TuneChoice> g_tune_cache;

}  // namespace

struct pyro_sw {
    int L = 0, model = 0;
    int64_t ncell = 0, N = 0;
    double T = 0, J = 0;
    uint64_t seed = 0;
    int start = 0;
    uint32_t thr_hi = 0, thr_lo = 0;
    float x0 = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false, own_mem = false;
    void *spins = nullptr;
    char *work = nullptr;
    Layout ly{};
    RepState *d_state = nullptr;
    // host mirror of the device state (the kernels advance it deterministically)
    RepState hs{};
    std::deque<pyro_sw_record> host_q;
    bool broken = false;
    int busy = 0;  // nonzero while a group sweeps this lattice
    // solo sweeps
    ChainTables solo;
    int solo_shape = kTile888;  // set from L at init (default_tile_shape)
    hipGraphExec_t solo_exec = nullptr;
    uint64_t param_version = 1, solo_version = 0;
    Timer timer;
    // Ising site dilution: per-cell masks of the bonds with two occupied ends
    // (library-owned, allocated on the first set_spins with a vacant site)
    uint64_t *d_present = nullptr;
    bool diluted = false;
};

// A slice of a group's members with its own chains, captured sweep and
// internal stream: the slices of a group run concurrently, so the
// latency-bound passes of one slice overlap the arithmetic of another.
struct SubGroup {
    ChainTables chains[3];  // Ising, XY, Heisenberg members of this slice
    hipGraphExec_t exec = nullptr;   // one sweep of the per-sweep chains
    hipGraphExec_t pexec = nullptr;  // persistent launch of the Ising chain (all sweeps of a call)
    hipStream_t stream = nullptr;  // internal, default priority
    hipEvent_t join = nullptr;
};

struct pyro_sw_group {
    std::vector<pyro_sw *> members;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    ChainTables chains[3];  // all members per model: tile shape and tuning key
    std::vector<SubGroup> subs;
    hipEvent_t fork = nullptr;
    std::vector<uint64_t> seen_versions;
    bool tables_dirty = true;
    RepState **d_members = nullptr;  // state pointer of every member (stream-ordered allocation)
    bool broken = false;
    Timer timer;
    // Ising modes (pyro_sw_group_set_mode): persistent fused launch for the
    // tiled Ising members; LDS-resident launch for small Ising members
    int ising_mode = PYRO_MODE_GRAPH;
    int64_t persist_cap = kRing;  // sweeps per persistent launch (item counts stay below 2^31)
    bool resident = false;
    ChainTables res;  // LDS-resident members (one launch, own stream)
    int res_maxL = 0;
    hipGraphExec_t rexec = nullptr;
    hipStream_t res_stream = nullptr;
    hipEvent_t res_join = nullptr;
    unsigned long long *d_counts = nullptr;  // unite-pass compare-and-swap counters (measurement)
    bool counting = false;
};

namespace {

int device_fail(bool *broken, hipError_t e, const char *what)
{
    if (broken) *broken = true;
    (void)hipGetLastError();
    return fail(PYRO_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_OR_FAIL(flag, call)                                          \
    do {                                                                 \
        hipError_t e__ = (call);                                         \
        if (e__ != hipSuccess) return device_fail(flag, e__, #call);     \
    } while (0)

// The two per-run constants of Sec. 2: Ising threshold floor((1 -
// exp(-2J/T)) 2^32), split at bit 24, and the O(n) coupling (float)(2J/T).
void run_constants(double T, double J, uint32_t *thr_hi, uint32_t *thr_lo, float *x0)
{
    const double twobj = 2.0 * J / T;
    const double p = -expm1(-twobj);
    const uint64_t thr = (uint64_t)floor(p * 4294967296.0);
    *thr_hi = (uint32_t)(thr >> 24);
    *thr_lo = (uint32_t)(thr & 0xFFFFFFu);
    *x0 = (float)twobj;
}

void set_params(pyro_sw *h, double T)
{
    h->T = T;
    run_constants(T, h->J, &h->thr_hi, &h->thr_lo, &h->x0);
    h->param_version++;
}

// Bond masks of a site-diluted Ising lattice: bit j of cell c is set when
// both ends of bond 48 c + j hold a nonzero spin (a vacant site, spin 0,
// carries no bond).
void present_masks(const int8_t *s, int L, std::vector<uint64_t> &pm)
{
    const int64_t nc = (int64_t)L * L * L;
    pm.assign((size_t)nc, 0);
    for (int64_t c = 0; c < nc; ++c) {
        const CellNbrs nb = cell_neighbours((int)c, L);
        uint64_t m = 0;
        for (int j = 0; j < 48; ++j) {
            const SiteRef a = bond_end_a(j), b = bond_end_b(j);
            if (s[16 * (int64_t)nb.c[a.cell] + a.site] != 0 && s[16 * (int64_t)nb.c[b.cell] + b.site] != 0)
                m |= 1ull << j;
        }
        pm[(size_t)c] = m;
    }
}

// Descriptor of a lattice (edge L, model, run constants, spins and a
// workspace laid out by layout_for) for a chain with tile shape `shape`.
RepDesc lattice_desc(int L, int model, double J, uint64_t seed, uint32_t thr_hi, uint32_t thr_lo, float x0,
                     void *spins, char *work, const Layout &ly, const uint64_t *present, int shape, int tile_base,
                     int cblk_base)
{
    RepDesc d{};
    const TileDims t = tile_dims(shape);
    d.L = L;
    d.ntx = (L + t.x - 1) / t.x;
    d.nty = (L + t.y - 1) / t.y;
    d.ntz = (L + t.z - 1) / t.z;
    d.lgL = -1;
    d.divisible = L % t.x == 0 && L % t.y == 0 && L % t.z == 0 && L >= 2 * std::max(t.x, std::max(t.y, t.z));
    if ((L & (L - 1)) == 0 && L % t.x == 0 && L % t.y == 0 && L % t.z == 0)
        for (int v = L, k = 0; v > 0; v >>= 1, ++k)
            if (v == 1) d.lgL = k;
    d.ncell = (int64_t)L * L * L;
    d.N = 16 * d.ncell;
    d.spins = spins;
    d.label = (int32_t *)(work + ly.label);
    d.ipart = (int64_t *)(work + ly.ipart);
    d.dpart = model == PYRO_ISING ? nullptr : (double *)(work + ly.dpart);
    d.ring = (DevRecord *)(work + ly.ring);
    d.pairs = (int *)(work + ly.pairs);
    d.list_stride = tile_list_stride(shape);
    d.present = present;
    d.thr_hi = thr_hi;
    d.thr_lo = thr_lo;
    d.x0 = x0;
    d.J = J;
    d.key = philox_key(seed);
    d.ring_cap = kRing;
    d.mpart_off = (int)max_tiles(L);
    d.tail_off = (int)(model == PYRO_ISING ? 2 * max_tiles(L) : 4 * max_tiles(L));
    d.tile_base = tile_base;
    d.cblk_base = cblk_base;
    return d;
}

// Descriptor of a replica for a chain with tile shape `shape`.
RepDesc make_desc(const pyro_sw *h, int shape, int tile_base, int cblk_base)
{
    return lattice_desc(h->L, h->model, h->J, h->seed, h->thr_hi, h->thr_lo, h->x0, h->spins, h->work, h->ly,
                        h->diluted ? h->d_present : nullptr, shape, tile_base, cblk_base);
}

// Group tables live in one stream-ordered allocation on the group's stream,
// so building or dropping a group never waits for other streams (plain
// hipFree synchronises the whole device).
void free_tables(ChainTables &ct)
{
    if (ct.owned && ct.block) hipFreeAsync(ct.block, ct.stream);
    ct.block = nullptr;
    ct.d_desc = nullptr;
    ct.d_stp = nullptr;
    ct.d_tile_rep = ct.d_cblk_rep = nullptr;
    ct.d_ctl = nullptr;
}

// Workgroups of a persistent launch with tile shape `shape`: all that can
// be resident on the current device.
int persist_grid_for(int shape)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        ising_persistent_blocks_per_cu(shape, &per_cu) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return std::max(1, cus * std::max(per_cu, 1));
}

// Build (or rebuild) the device tables of a group chain on stream st (with
// the control words of a persistent launch when `persistent`); the copies
// are complete when this returns.
hipError_t build_group_chain(ChainTables &ct, int shape, hipStream_t st, bool persistent = false)
{
    free_tables(ct);
    ct.owned = true;
    ct.stream = st;
    ct.shape = shape;
    const int n = (int)ct.reps.size();
    ct.chain = Chain{};
    ct.chain.nreps = n;
    ct.chain.model = ct.model;
    ct.chain.shape = shape;
    if (n == 0) return hipSuccess;
    std::vector<RepDesc> desc(n);
    std::vector<RepState *> stp(n);
    std::vector<int> tmap, cmap;
    int tb = 0, cb = 0;
    for (int r = 0; r < n; ++r) {
        pyro_sw *h = ct.reps[r];
        desc[r] = make_desc(h, shape, tb, cb);
        stp[r] = h->d_state;
        const int nt = (int)tiles_for(h->L, shape), nc = blocks_for(h->ncell);
        tmap.insert(tmap.end(), nt, r);
        cmap.insert(cmap.end(), nc, r);
        tb += nt;
        cb += nc;
    }
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t b_desc = up(sizeof(RepDesc) * n), b_stp = up(sizeof(RepState *) * n);
    const size_t b_t = up(sizeof(int) * tmap.size()), b_c = up(sizeof(int) * cmap.size());
    const size_t b_ctl = persistent ? up(sizeof(int) * kPersistStride * (n + 1)) : 0;
    hipError_t e = hipMallocAsync(&ct.block, b_desc + b_stp + b_t + b_c + b_ctl, st);
    if (e != hipSuccess) return e;
    char *p = (char *)ct.block;
    ct.d_desc = (RepDesc *)p;
    ct.d_stp = (RepState **)(p + b_desc);
    ct.d_tile_rep = (int *)(p + b_desc + b_stp);
    ct.d_cblk_rep = (int *)(p + b_desc + b_stp + b_t);
    ct.d_ctl = persistent ? (int *)(p + b_desc + b_stp + b_t + b_c) : nullptr;
    ct.persist_grid = persistent ? persist_grid_for(shape) : 0;
    if (persistent && ct.persist_grid == 0) return hipErrorInvalidValue;
    if ((e = hipMemcpyAsync(ct.d_desc, desc.data(), sizeof(RepDesc) * n, hipMemcpyHostToDevice, st)) != hipSuccess)
        return e;
    if ((e = hipMemcpyAsync(ct.d_stp, stp.data(), sizeof(RepState *) * n, hipMemcpyHostToDevice, st)) != hipSuccess)
        return e;
    if ((e = hipMemcpyAsync(ct.d_tile_rep, tmap.data(), sizeof(int) * tmap.size(), hipMemcpyHostToDevice, st)) !=
        hipSuccess)
        return e;
    if ((e = hipMemcpyAsync(ct.d_cblk_rep, cmap.data(), sizeof(int) * cmap.size(), hipMemcpyHostToDevice, st)) !=
        hipSuccess)
        return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;  // host vectors go out of scope
    ct.chain.desc = ct.d_desc;
    ct.chain.state = ct.d_stp;
    ct.chain.tile_rep = ct.d_tile_rep;
    ct.chain.cblk_rep = ct.d_cblk_rep;
    ct.chain.ntile_blocks = tb;
    ct.chain.ncell_blocks = cb;
    return hipSuccess;
}

// Solo chain: tables inside the handle's workspace (block maps all zero).
hipError_t build_solo_chain(pyro_sw *h)
{
    ChainTables &ct = h->solo;
    ct.owned = false;
    ct.model = h->model;
    ct.shape = h->solo_shape;
    ct.reps.assign(1, h);
    const RepDesc d = make_desc(h, h->solo_shape, 0, 0);
    ct.d_desc = (RepDesc *)(h->work + h->ly.solo_desc);
    ct.d_stp = (RepState **)(h->work + h->ly.solo_stp);
    int *zeros = (int *)(h->work + h->ly.solo_map);
    ct.d_tile_rep = ct.d_cblk_rep = zeros;
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return e;
    if ((e = hipMemcpy(ct.d_desc, &d, sizeof(RepDesc), hipMemcpyHostToDevice)) != hipSuccess) return e;
    RepState *p = h->d_state;
    if ((e = hipMemcpy(ct.d_stp, &p, sizeof(p), hipMemcpyHostToDevice)) != hipSuccess) return e;
    Chain &c = ct.chain;
    c = Chain{};
    c.desc = ct.d_desc;
    c.state = ct.d_stp;
    c.tile_rep = c.cblk_rep = zeros;
    c.nreps = 1;
    c.shape = h->solo_shape;
    c.model = h->model;
    c.ntile_blocks = (int)tiles_for(h->L, h->solo_shape);
    c.ncell_blocks = blocks_for(h->ncell);
    if (h->solo_exec) {
        hipGraphExecDestroy(h->solo_exec);
        h->solo_exec = nullptr;
    }
    h->solo_version = h->param_version;
    return hipSuccess;
}

// Capture the launches `launch(stream)` makes on a private stream (nothing
// runs); the executable graph is later launched on the caller's stream.
template <typename F>
hipError_t capture_graph(F launch, hipGraphExec_t *exec)
{
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    hipGraph_t graph = nullptr;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    hipError_t le = hipSuccess;
    if (e == hipSuccess) {
        le = launch(cs);
        e = hipStreamEndCapture(cs, &graph);
    }
    if (e == hipSuccess && le != hipSuccess) e = le;
    if (e == hipSuccess) e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
    if (graph) hipGraphDestroy(graph);
    hipStreamDestroy(cs);
    return e;
}

// Capture one sweep of the given chains.
hipError_t capture_sweep(const Chain *chains, int nchains, hipGraphExec_t *exec)
{
    const LaunchHook none{nullptr, nullptr, nullptr};
    return capture_graph(
        [&](hipStream_t cs) {
            hipError_t le = hipSuccess;
            for (int k = 0; k < nchains && le == hipSuccess; ++k) le = launch_chain_sweep(chains[k], cs, none);
            return le;
        },
        exec);
}

// Arming writes replica states in stream order.  The states travel as
// kernel arguments, which are copied when the launch is enqueued, so no host
// buffer has to outlive the call (an asynchronous copy from pageable host
// memory gives no such guarantee).
constexpr int kArmBatch = 96;  // 96 x 16 B of kernel arguments per launch
struct ArmBatch {
    RepState v[kArmBatch];
};
static_assert(sizeof(RepState) == 16, "RepState layout");

__global__ void k_arm(RepState *const *stp, ArmBatch b, int first, int n)
{
    const int i = threadIdx.x;
    if (i < n) *stp[first + i] = b.v[i];
}

__global__ void k_arm_one(RepState *dst, RepState v)
{
    if (threadIdx.x == 0) *dst = v;
}

int usable(const pyro_sw *h)
{
    if (!h) return fail(PYRO_EINVAL, "handle is NULL");
    if (h->broken) return fail(PYRO_ESTATE, "handle failed earlier");
    if (h->busy) return fail(PYRO_ESTATE, "handle is sweeping inside a group");
    return PYRO_OK;
}

LaunchHook hook_of(Timer &tm, hipStream_t st)
{
    tm.stream = st;
    return tm.mask ? tm.hook() : LaunchHook{nullptr, nullptr, nullptr};
}

// Energy of the pending record (tail), then copy the ring to the host queue.
int drain(pyro_sw *h)
{
    if (h->hs.e_pending >= 0) {
        if (h->solo_version != h->param_version) HIP_OR_FAIL(&h->broken, build_solo_chain(h));
        HIP_OR_FAIL(&h->broken, launch_chain_energy_tail(h->solo.chain, h->stream, hook_of(h->timer, h->stream)));
        h->hs.e_pending = -1;
    }
    HIP_OR_FAIL(&h->broken, hipStreamSynchronize(h->stream));
    if (h->hs.ring_used > 0) {
        // The kernels advance the device state exactly as the host mirror
        // assumes; a persistent launch that gave up a wait leaves it behind.
        RepState ds{};
        HIP_OR_FAIL(&h->broken, hipMemcpy(&ds, h->d_state, sizeof(RepState), hipMemcpyDeviceToHost));
        if (ds.t != h->hs.t || ds.ring_used != h->hs.ring_used) {
            h->broken = true;
            return fail(PYRO_EDEVICE, "device sweep state disagrees with the host (a persistent launch gave up)");
        }
        std::vector<pyro_sw_record> tmp((size_t)h->hs.ring_used);
        HIP_OR_FAIL(&h->broken, hipMemcpy(tmp.data(), h->work + h->ly.ring, sizeof(pyro_sw_record) * tmp.size(),
                                          hipMemcpyDeviceToHost));
        for (auto &r : tmp) h->host_q.push_back(r);
        h->hs.ring_used = 0;
    }
    return PYRO_OK;
}

int create(pyro_sw **out, int L, int model, double T, double J, uint64_t seed, int start, void *stream,
           void *dev_spins, size_t spin_bytes, void *dev_work, size_t work_bytes, bool ext)
{
    if (!out) return fail(PYRO_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_args(L, model, T, J, start);
    if (rc) return rc;
    const Layout ly = layout_for(L, model);
    if (ext) {
        if (!dev_spins || !dev_work) return fail(PYRO_EINVAL, "device buffers must not be NULL");
        if (((uintptr_t)dev_spins % kAlign) || ((uintptr_t)dev_work % kAlign))
            return fail(PYRO_EINVAL, "device buffers must be 256-byte aligned");
        if (spin_bytes < ly.spin_bytes || work_bytes < ly.total)
            return fail(PYRO_EINVAL, "device buffers too small (see pyro_sw_workspace_size)");
    }
    pyro_sw *h = new (std::nothrow) pyro_sw();
    if (!h) return fail(PYRO_ENOMEM, "host allocation failed");
    h->L = L;
    h->solo_shape = default_tile_shape(L);
    h->model = model;
    h->ncell = (int64_t)L * L * L;
    h->N = 16 * h->ncell;
    h->J = J;
    h->seed = seed;
    h->start = start;
    h->ly = ly;
    set_params(h, T);
    if (stream) {
        h->stream = (hipStream_t)stream;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete h;
            return fail(PYRO_EDEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
        }
        h->own_stream = true;
    }
    if (ext) {
        h->spins = dev_spins;
        h->work = (char *)dev_work;
    } else {
        hipError_t e1 = hipMalloc(&h->spins, ly.spin_bytes);
        hipError_t e2 = e1 == hipSuccess ? hipMalloc((void **)&h->work, ly.total) : e1;
        if (e1 != hipSuccess || e2 != hipSuccess) {
            if (e1 == hipSuccess) hipFree(h->spins);
            if (h->own_stream) hipStreamDestroy(h->stream);
            delete h;
            (void)hipGetLastError();
            return fail(PYRO_ENOMEM, "hipMalloc failed");
        }
        h->own_mem = true;
    }
    h->d_state = (RepState *)(h->work + ly.state);
    h->hs = RepState{0u, 0, 0, -1};
    std::vector<int> zeros((size_t)ly.map_len, 0);
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess)
        e = hipMemcpy(h->work + ly.solo_map, zeros.data(), sizeof(int) * zeros.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(h->d_state, &h->hs, sizeof(RepState), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = build_solo_chain(h);
    if (e == hipSuccess) e = launch_init(make_desc(h, h->solo_shape, 0, 0), model, start, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        int r = fail(PYRO_EDEVICE, std::string("initial state: ") + hipGetErrorString(e));
        pyro_sw_destroy(h);
        return r;
    }
    *out = h;
    return PYRO_OK;
}

// Before a call that runs up to `n` more sweeps of h: room in the ring.
int make_room(pyro_sw *h, int64_t n)
{
    if (h->hs.ring_used + n > kRing) return drain(h);
    return PYRO_OK;
}

std::string tune_key(const ChainTables &ct)
{
    std::vector<int> Ls;
    for (auto *r : ct.reps) Ls.push_back(r->L);
    std::sort(Ls.begin(), Ls.end());
    std::string k = "m" + std::to_string(ct.model) + ":";
    for (int L : Ls) k += std::to_string(L) + ",";
    return k;
}

}  // namespace

// (Re)deal a group's members to nslices slices, largest first to the
// lightest slice; every slice beyond the first gets its own stream.
static void drop_graphs(pyro_sw_group *g)
{
    for (auto &sg : g->subs) {
        if (sg.exec) hipGraphExecDestroy(sg.exec);
        if (sg.pexec) hipGraphExecDestroy(sg.pexec);
        sg.exec = sg.pexec = nullptr;
    }
    if (g->rexec) hipGraphExecDestroy(g->rexec);
    g->rexec = nullptr;
}

static void drop_slices(pyro_sw_group *g)
{
    drop_graphs(g);
    for (auto &sg : g->subs) {
        if (sg.stream) hipStreamSynchronize(sg.stream);
        for (auto &ct : sg.chains) free_tables(ct);
        if (sg.join) hipEventDestroy(sg.join);
        if (sg.stream) hipStreamDestroy(sg.stream);
    }
    g->subs.clear();
}

// Small pure Ising lattices sweep LDS-resident when the group asks for it.
static bool resident_member(const pyro_sw_group *g, const pyro_sw *h)
{
    return g->resident && h->model == PYRO_ISING && h->L <= kResidentMaxL && !h->diluted;
}

// Deal the members to the slices, largest first to the lightest slice (the
// LDS-resident ones to their own launch).
static void deal_members(pyro_sw_group *g)
{
    const int n = (int)g->members.size(), nslices = (int)g->subs.size();
    for (auto &sg : g->subs)
        for (auto &ct : sg.chains) ct.reps.clear();
    g->res.reps.clear();
    g->res.model = PYRO_ISING;
    g->res_maxL = 0;
    std::vector<double> load(nslices, 0.0);
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return g->members[a]->N > g->members[b]->N; });
    for (int i : order) {
        pyro_sw *h = g->members[i];
        if (resident_member(g, h)) {
            g->res.reps.push_back(h);
            g->res_maxL = std::max(g->res_maxL, h->L);
            continue;
        }
        const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[k] += (double)h->N;
        g->subs[k].chains[h->model - 1].reps.push_back(h);
    }
}

static int make_slices(pyro_sw_group *g, int nslices)
{
    drop_slices(g);
    g->subs.resize(nslices);
    bool ok = g->fork || hipEventCreateWithFlags(&g->fork, hipEventDisableTiming) == hipSuccess;
    for (auto &sg : g->subs) {
        for (int m = 0; m < 3; ++m) sg.chains[m].model = m + 1;
        if (nslices > 1) {
            ok = ok && hipStreamCreateWithFlags(&sg.stream, hipStreamNonBlocking) == hipSuccess;
            ok = ok && hipEventCreateWithFlags(&sg.join, hipEventDisableTiming) == hipSuccess;
        }
    }
    deal_members(g);
    g->tables_dirty = true;
    if (!ok) {
        (void)hipGetLastError();
        return fail(PYRO_EDEVICE, "group stream or event creation failed");
    }
    return PYRO_OK;
}

extern "C" {

int pyro_sw_workspace_size(int L, int model, size_t *spin_bytes, size_t *work_bytes)
{
    if (L < 1 || L > 406) return fail(PYRO_EINVAL, "L must be in [1, 406]");
    if (model < PYRO_ISING || model > PYRO_HEISENBERG) return fail(PYRO_EINVAL, "model must be 1, 2 or 3");
    const Layout ly = layout_for(L, model);
    if (spin_bytes) *spin_bytes = ly.spin_bytes;
    if (work_bytes) *work_bytes = ly.total;
    return PYRO_OK;
}

int pyro_sw_init(pyro_sw **out, int L, int model, double T, double J, uint64_t seed, int start, void *stream)
{
    return create(out, L, model, T, J, seed, start, stream, nullptr, 0, nullptr, 0, false);
}

int pyro_sw_init_ext(pyro_sw **out, int L, int model, double T, double J, uint64_t seed, int start,
                     void *stream, void *dev_spins, size_t spin_bytes, void *dev_work, size_t work_bytes)
{
    return create(out, L, model, T, J, seed, start, stream, dev_spins, spin_bytes, dev_work, work_bytes, true);
}

int pyro_sw_sweep(pyro_sw *h, int64_t n_sweeps)
{
    int rc = usable(h);
    if (rc) return rc;
    if (n_sweeps < 0) return fail(PYRO_EINVAL, "n_sweeps must be >= 0");
    if ((int64_t)h->hs.t + n_sweeps > (int64_t)UINT32_MAX)
        return fail(PYRO_EINVAL, "sweep index would exceed 2^32 - 1");
    Timer &tm = h->timer;
    while (n_sweeps > 0) {
        const int64_t chunk = std::min<int64_t>(n_sweeps, kRing);
        rc = make_room(h, chunk);
        if (rc) return rc;
        if (h->solo_version != h->param_version) HIP_OR_FAIL(&h->broken, build_solo_chain(h));
        RepState armed = h->hs;
        armed.remaining = (int32_t)chunk;
        k_arm_one<<<1, 64, 0, h->stream>>>(h->d_state, armed);
        HIP_OR_FAIL(&h->broken, hipGetLastError());
        if (tm.mask) {
            const LaunchHook hook = hook_of(tm, h->stream);
            for (int64_t k = 0; k < chunk; ++k) {
                HIP_OR_FAIL(&h->broken, launch_chain_sweep(h->solo.chain, h->stream, hook));
                if (tm.inflight.size() > 8192) HIP_OR_FAIL(&h->broken, tm.collect());
            }
        } else {
            if (!h->solo_exec) HIP_OR_FAIL(&h->broken, capture_sweep(&h->solo.chain, 1, &h->solo_exec));
            for (int64_t k = 0; k < chunk; ++k) HIP_OR_FAIL(&h->broken, hipGraphLaunch(h->solo_exec, h->stream));
        }
        // mirror what the kernels did to the device state
        h->hs.t += (uint32_t)chunk;
        h->hs.ring_used += (int32_t)chunk;
        h->hs.e_pending = h->hs.ring_used - 1;
        h->hs.remaining = 0;
        n_sweeps -= chunk;
    }
    return PYRO_OK;
}

int pyro_sw_moments(pyro_sw *h, pyro_sw_record *out, int64_t cap, int64_t *n_out)
{
    int rc = usable(h);
    if (rc) return rc;
    if (cap < 0 || (cap > 0 && !out) || !n_out) return fail(PYRO_EINVAL, "bad output arguments");
    rc = drain(h);
    if (rc) return rc;
    if (cap == 0) {
        *n_out = (int64_t)h->host_q.size();
        return PYRO_OK;
    }
    int64_t n = 0;
    while (n < cap && !h->host_q.empty()) {
        out[n++] = h->host_q.front();
        h->host_q.pop_front();
    }
    *n_out = n;
    return PYRO_OK;
}

int pyro_sw_get_spins(pyro_sw *h, void *host, size_t bytes)
{
    int rc = usable(h);
    if (rc) return rc;
    const size_t need = h->model == PYRO_ISING ? (size_t)h->N : sizeof(float) * h->model * (size_t)h->N;
    if (!host || bytes != need) return fail(PYRO_EINVAL, "host buffer size must equal the spin array size");
    HIP_OR_FAIL(&h->broken, hipStreamSynchronize(h->stream));
    HIP_OR_FAIL(&h->broken, hipMemcpy(host, h->spins, need, hipMemcpyDeviceToHost));
    return PYRO_OK;
}

int pyro_sw_set_spins(pyro_sw *h, const void *host, size_t bytes, int64_t next_sweep)
{
    int rc = usable(h);
    if (rc) return rc;
    const size_t need = h->model == PYRO_ISING ? (size_t)h->N : sizeof(float) * h->model * (size_t)h->N;
    if (!host || bytes != need) return fail(PYRO_EINVAL, "host buffer size must equal the spin array size");
    if (next_sweep < 0 || next_sweep > (int64_t)UINT32_MAX) return fail(PYRO_EINVAL, "bad sweep index");
    bool vacant = false;
    if (h->model == PYRO_ISING) {
        const int8_t *s = (const int8_t *)host;
        for (int64_t i = 0; i < h->N; ++i) {
            if (s[i] != 1 && s[i] != -1 && s[i] != 0) return fail(PYRO_EINVAL, "Ising spins must be +1, -1 or 0 (vacant)");
            vacant |= s[i] == 0;
        }
    }
    HIP_OR_FAIL(&h->broken, hipStreamSynchronize(h->stream));
    if (vacant) {
        std::vector<uint64_t> pm;
        present_masks((const int8_t *)host, h->L, pm);
        if (!h->d_present && hipMalloc((void **)&h->d_present, sizeof(uint64_t) * (size_t)h->ncell) != hipSuccess) {
            (void)hipGetLastError();
            h->d_present = nullptr;
            return fail(PYRO_ENOMEM, "bond masks of a diluted lattice");
        }
        HIP_OR_FAIL(&h->broken, hipMemcpy(h->d_present, pm.data(), sizeof(uint64_t) * pm.size(), hipMemcpyHostToDevice));
    }
    h->diluted = vacant;
    h->param_version++;  // descriptors (and captured sweeps) pick up the masks
    HIP_OR_FAIL(&h->broken, hipMemcpy(h->spins, host, need, hipMemcpyHostToDevice));
    h->hs = RepState{(uint32_t)next_sweep, 0, 0, -1};
    h->host_q.clear();
    return PYRO_OK;
}

int pyro_sw_get_labels(pyro_sw *h, int32_t *host, size_t n)
{
    int rc = usable(h);
    if (rc) return rc;
    if (!host || n != (size_t)h->N) return fail(PYRO_EINVAL, "n must equal N");
    const RepDesc d = make_desc(h, h->solo_shape, 0, 0);
    int32_t *tmp = nullptr;
    if (hipMalloc((void **)&tmp, sizeof(int32_t) * n) != hipSuccess) {
        (void)hipGetLastError();
        return fail(PYRO_ENOMEM, "label buffer");
    }
    hipError_t e = launch_canonical_labels(d, tmp, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) e = hipMemcpy(host, tmp, sizeof(int32_t) * n, hipMemcpyDeviceToHost);
    hipFree(tmp);
    if (e != hipSuccess) return device_fail(&h->broken, e, "get_labels");
    return PYRO_OK;
}

int pyro_sw_set_temperature(pyro_sw *h, double T)
{
    int rc = usable(h);
    if (rc) return rc;
    if (!(T > 0.0)) return fail(PYRO_EINVAL, "T must be > 0 (inf allowed)");
    set_params(h, T);
    return PYRO_OK;
}

int pyro_sw_set_tile_shape(pyro_sw *h, int shape)
{
    int rc = usable(h);
    if (rc) return rc;
    if (shape < 0 || shape >= kNumTileShapes) return fail(PYRO_EINVAL, "unknown tile shape");
    h->solo_shape = shape;
    h->param_version++;
    return PYRO_OK;
}

int pyro_sw_info(const pyro_sw *h, int64_t *n_sites, int64_t *next_sweep)
{
    if (!h) return fail(PYRO_EINVAL, "handle is NULL");
    if (n_sites) *n_sites = h->N;
    if (next_sweep) *next_sweep = h->hs.t;
    return PYRO_OK;
}

int pyro_sw_set_timing(pyro_sw *h, int kernel_mask)
{
    int rc = usable(h);
    if (rc) return rc;
    h->timer.stream = h->stream;
    HIP_OR_FAIL(&h->broken, h->timer.collect());
    h->timer.reset(kernel_mask);
    return PYRO_OK;
}

static int report_times(Timer &tm, bool *broken, const char **names, int64_t *launches, double *ms, int cap,
                        int *n_out)
{
    if (!n_out || cap < 0) return fail(PYRO_EINVAL, "bad output arguments");
    HIP_OR_FAIL(broken, tm.collect());
    int n = 0;
    for (int k = 0; k < kNumKernels && n < cap; ++k) {
        if (names) names[n] = kernel_name(k);
        if (launches) launches[n] = tm.launches[k];
        if (ms) ms[n] = tm.ms[k];
        ++n;
    }
    *n_out = n;
    return PYRO_OK;
}

int pyro_sw_kernel_times(pyro_sw *h, const char **names, int64_t *launches, double *ms, int cap, int *n_out)
{
    int rc = usable(h);
    if (rc) return rc;
    return report_times(h->timer, &h->broken, names, launches, ms, cap, n_out);
}

int pyro_sw_philox_rate(int64_t calls, int repeats, uint64_t seed, double *calls_per_second, uint32_t *fold)
{
    if (calls < 1 || calls > ((int64_t)1 << 32)) return fail(PYRO_EINVAL, "calls must be in [1, 2^32]");
    if (repeats < 1) return fail(PYRO_EINVAL, "repeats must be >= 1");
    if (!calls_per_second || !fold) return fail(PYRO_EINVAL, "outputs must not be NULL");
    constexpr int kBlocks = 2048;  // 8 workgroups of 256 threads per CU
    uint32_t *d_out = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::vector<uint32_t> folds(kBlocks);
    float best = -1.0f;
    hipError_t e = hipMalloc(&d_out, sizeof(uint32_t) * kBlocks);
    if (e == hipSuccess) e = hipStreamCreate(&st);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    for (int r = 0; r < repeats && e == hipSuccess; ++r) {
        e = hipEventRecord(e0, st);
        if (e == hipSuccess) {
            k_philox_rate<<<kBlocks, 256, 0, st>>>((uint64_t)calls, philox_key(seed), d_out);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && (best < 0.0f || ms < best)) best = ms;
    }
    if (e == hipSuccess) e = hipMemcpy(folds.data(), d_out, sizeof(uint32_t) * kBlocks, hipMemcpyDeviceToHost);
    if (e1) (void)hipEventDestroy(e1);
    if (e0) (void)hipEventDestroy(e0);
    if (st) (void)hipStreamDestroy(st);
    if (d_out) (void)hipFree(d_out);
    if (e != hipSuccess) return fail(PYRO_EDEVICE, std::string("philox rate: ") + hipGetErrorString(e));
    uint32_t f = 0;
    for (uint32_t v : folds) f ^= v;
    *fold = f;
    *calls_per_second = (double)calls / (std::max(best, 1e-6f) * 1e-3);
    return PYRO_OK;
}

// ------------------------------------------------ no-allocation sweeps ---
// Workspace of pyro_sw_sweep_static: one fixed array per device, held until
// the process ends.  Host code never passes `scratch` itself to a kernel (in
// host code the name is a stand-in, not a device address): each device's
// address is looked up once with hipGetSymbolAddress and used from then on.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on that device).
int static_scratch(char **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(PYRO_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(PYRO_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(PYRO_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = (char *)p;
    }
    *out = g_scratch_ptr[dev];
    return PYRO_OK;
}

// Descriptor, state and zero block map of a solo chain written into the
// scratch by one kernel whose arguments carry them (no host buffer, no
// memset node).
__global__ void k_static_setup(RepDesc *desc_dst, RepDesc d, RepState **stp_dst, RepState *state, RepState s,
                               int *map, int map_len)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        *desc_dst = d;
        *stp_dst = state;
        *state = s;
    }
    for (int k = i; k < map_len; k += gridDim.x * blockDim.x) map[k] = 0;
}
}  // namespace

int pyro_sw_sweep_static(void *dev_spins, int L, int model, double T, double J, uint64_t seed, int64_t first_sweep,
                         int64_t n_sweeps, pyro_sw_record *dev_records, void *stream)
{
    int rc = check_args(L, model, T, J, PYRO_START_COLD);
    if (rc) return rc;
    if (!dev_spins || (n_sweeps > 0 && !dev_records)) return fail(PYRO_EINVAL, "device buffers must not be NULL");
    if (((uintptr_t)dev_spins % 16) || ((uintptr_t)dev_records % 8))
        return fail(PYRO_EINVAL, "spins must be 16-byte and records 8-byte aligned");
    if (n_sweeps < 0 || n_sweeps > INT32_MAX) return fail(PYRO_EINVAL, "n_sweeps must be in [0, 2^31 - 1]");
    if (first_sweep < 0 || first_sweep + n_sweeps > (int64_t)UINT32_MAX)
        return fail(PYRO_EINVAL, "sweep indices must stay below 2^32");
    const Layout ly = layout_for(L, model);
    if (ly.total > kStaticScratchBytes)
        return fail(PYRO_EINVAL, "lattice too large for the static workspace (64 MiB: L <= 80)");
    if (n_sweeps == 0) return PYRO_OK;
    char *work = nullptr;
    rc = static_scratch(&work);
    if (rc) return rc;
    uint32_t thr_hi = 0, thr_lo = 0;
    float x0 = 0.0f;
    run_constants(T, J, &thr_hi, &thr_lo, &x0);
    const int shape = default_tile_shape(L);
    RepDesc d = lattice_desc(L, model, J, seed, thr_hi, thr_lo, x0, dev_spins, work, ly, nullptr, shape, 0, 0);
    d.ring = (DevRecord *)dev_records;  // records go straight to the caller's buffer
    d.ring_cap = (int)n_sweeps;
    const int64_t ncell = (int64_t)L * L * L;
    RepDesc *d_desc = (RepDesc *)(work + ly.solo_desc);
    RepState **d_stp = (RepState **)(work + ly.solo_stp);
    RepState *d_state = (RepState *)(work + ly.state);
    int *map = (int *)(work + ly.solo_map);
    const RepState s0{(uint32_t)first_sweep, (int32_t)n_sweeps, 0, -1};
    hipStream_t st = (hipStream_t)stream;
    k_static_setup<<<std::max(1, std::min(blocks_for(ly.map_len), 1024)), kBlock, 0, st>>>(
        d_desc, d, d_stp, d_state, s0, map, (int)ly.map_len);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(PYRO_EDEVICE, std::string("static setup: ") + hipGetErrorString(e));
    Chain c{};
    c.desc = d_desc;
    c.state = d_stp;
    c.tile_rep = c.cblk_rep = map;
    c.nreps = 1;
    c.shape = shape;
    c.model = model;
    c.ntile_blocks = (int)tiles_for(L, shape);
    c.ncell_blocks = blocks_for(ncell);
    const LaunchHook none{nullptr, nullptr, nullptr};
    for (int64_t k = 0; k < n_sweeps && e == hipSuccess; ++k) e = launch_chain_sweep(c, st, none);
    if (e == hipSuccess) e = launch_chain_energy_tail(c, st, none);
    if (e != hipSuccess) return fail(PYRO_EDEVICE, std::string("static sweep: ") + hipGetErrorString(e));
    return PYRO_OK;
}

int pyro_sw_atomic_rate(int mode, int64_t words, int64_t ops, int repeats, double *ops_per_second,
                        int64_t *succeeded, int64_t *word_sum)
{
    if (mode != 0 && mode != 1) return fail(PYRO_EINVAL, "mode must be 0 (random CAS) or 1 (one-address add)");
    if (words < 1 || words > ((int64_t)1 << 32)) return fail(PYRO_EINVAL, "words must be in [1, 2^32]");
    if (ops < 1 || ops > ((int64_t)1 << 40)) return fail(PYRO_EINVAL, "ops must be in [1, 2^40]");
    if (repeats < 1) return fail(PYRO_EINVAL, "repeats must be >= 1");
    if (!ops_per_second || !succeeded || !word_sum) return fail(PYRO_EINVAL, "outputs must not be NULL");
    constexpr int kBlocks = 4096;  // 16 workgroups of 256 threads per CU
    uint32_t *a = nullptr;
    unsigned long long *d_out = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float best = -1.0f;
    unsigned long long out[2] = {0, 0};
    hipError_t e = hipMalloc(&a, sizeof(uint32_t) * (size_t)words);
    if (e == hipSuccess) e = hipMalloc(&d_out, 2 * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipStreamCreate(&st);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    for (int r = 0; r < repeats && e == hipSuccess; ++r) {
        e = hipMemsetAsync(a, 0, sizeof(uint32_t) * (size_t)words, st);
        if (e == hipSuccess) e = hipMemsetAsync(d_out, 0, 2 * sizeof(unsigned long long), st);
        if (e == hipSuccess) e = hipEventRecord(e0, st);
        if (e == hipSuccess) {
            k_atomic_rate<<<kBlocks, 256, 0, st>>>(mode, a, (uint64_t)words, (uint64_t)ops, d_out);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) {
            k_sum_words<<<1024, 256, 0, st>>>(a, (uint64_t)words, d_out + 1);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && (best < 0.0f || ms < best)) best = ms;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipMemcpy(out, d_out, sizeof(out), hipMemcpyDeviceToHost);
    if (e1) (void)hipEventDestroy(e1);
    if (e0) (void)hipEventDestroy(e0);
    if (st) (void)hipStreamDestroy(st);
    if (d_out) (void)hipFree(d_out);
    if (a) (void)hipFree(a);
    if (e != hipSuccess) return fail(PYRO_EDEVICE, std::string("atomic rate: ") + hipGetErrorString(e));
    *succeeded = (int64_t)out[0];
    *word_sum = (int64_t)out[1];
    *ops_per_second = (double)ops / (std::max(best, 1e-6f) * 1e-3);
    return PYRO_OK;
}

int pyro_sw_destroy(pyro_sw *h)
{
    if (!h) return PYRO_OK;
    int rc = PYRO_OK;
    if (h->stream && hipStreamSynchronize(h->stream) != hipSuccess) rc = fail(PYRO_EDEVICE, "synchronize failed");
    h->timer.release();
    if (h->solo_exec) hipGraphExecDestroy(h->solo_exec);
    if (h->own_mem) {
        hipFree(h->spins);
        hipFree(h->work);
    }
    if (h->d_present) hipFree(h->d_present);
    if (h->own_stream) hipStreamDestroy(h->stream);
    delete h;
    return rc;
}

// ------------------------------------------------------------------ groups --

int pyro_sw_group_create(pyro_sw_group **out, pyro_sw *const *members, int n, void *stream)
{
    if (!out) return fail(PYRO_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || !members) return fail(PYRO_EINVAL, "a group needs at least one member");
    for (int i = 0; i < n; ++i) {
        int rc = usable(members[i]);
        if (rc) return rc;
        for (int j = 0; j < i; ++j)
            if (members[j] == members[i]) return fail(PYRO_EINVAL, "a lattice appears twice in the group");
    }
    pyro_sw_group *g = new (std::nothrow) pyro_sw_group();
    if (!g) return fail(PYRO_ENOMEM, "host allocation failed");
    g->members.assign(members, members + n);
    for (int m = 0; m < 3; ++m) g->chains[m].model = m + 1;
    for (auto *h : g->members) g->chains[h->model - 1].reps.push_back(h);
    if (stream) {
        g->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking) != hipSuccess) {
            delete g;
            return fail(PYRO_EDEVICE, "hipStreamCreate failed");
        }
        g->own_stream = true;
    }
    std::vector<RepState *> ptrs(n);
    for (int i = 0; i < n; ++i) ptrs[i] = g->members[i]->d_state;
    if (hipMallocAsync((void **)&g->d_members, sizeof(RepState *) * n, g->stream) != hipSuccess ||
        hipMemcpyAsync(g->d_members, ptrs.data(), sizeof(RepState *) * n, hipMemcpyHostToDevice, g->stream) !=
            hipSuccess ||
        hipStreamSynchronize(g->stream) != hipSuccess) {
        (void)hipGetLastError();
        pyro_sw_group_destroy(g);
        return fail(PYRO_ENOMEM, "group state buffers");
    }
    // tile shapes: autotuned results when known for this mix of lattices
    for (auto &ct : g->chains) {
        if (ct.reps.empty()) continue;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(tune_key(ct));
        int lmax = 1;
        for (const pyro_sw *h : ct.reps) lmax = std::max(lmax, h->L);
        ct.shape = it != g_tune_cache.end() ? it->second.shape : default_tile_shape(lmax);
        if (it != g_tune_cache.end() && ct.model == PYRO_ISING) {
            g->ising_mode = it->second.ising_mode;
            g->resident = it->second.resident;
        }
    }
    if (int rc = make_slices(g, std::min(n, kMaxSlices))) {
        pyro_sw_group_destroy(g);
        return rc;
    }
    *out = g;
    return PYRO_OK;
}

static int group_prepare(pyro_sw_group *g)
{
    bool changed = g->tables_dirty || g->seen_versions.size() != g->members.size();
    if (!changed)
        for (size_t i = 0; i < g->members.size(); ++i)
            if (g->seen_versions[i] != g->members[i]->param_version) changed = true;
    if (!changed) return PYRO_OK;
    HIP_OR_FAIL(&g->broken, hipStreamSynchronize(g->stream));
    drop_graphs(g);
    deal_members(g);  // a member's dilution decides whether it may stay LDS-resident
    const bool persistent = g->ising_mode == PYRO_MODE_PERSISTENT;
    g->persist_cap = kRing;
    for (auto &sg : g->subs) {
        for (int m = 0; m < 3; ++m) {
            HIP_OR_FAIL(&g->broken, build_group_chain(sg.chains[m], g->chains[m].shape, g->stream, m == 0 && persistent));
            sg.chains[m].chain.counts = g->counting ? g->d_counts : nullptr;
        }
        if (persistent)
            for (const pyro_sw *h : sg.chains[0].reps)
                g->persist_cap = std::min<int64_t>(g->persist_cap, (INT32_MAX / 4) / tiles_for(h->L, g->chains[0].shape));
    }
    HIP_OR_FAIL(&g->broken, build_group_chain(g->res, kTile888, g->stream));
    if (!g->res.reps.empty() && !g->res_stream) {
        if (hipStreamCreateWithFlags(&g->res_stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&g->res_join, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            return fail(PYRO_EDEVICE, "group stream or event creation failed");
        }
    }
    g->seen_versions.clear();
    for (auto *h : g->members) g->seen_versions.push_back(h->param_version);
    g->tables_dirty = false;
    return PYRO_OK;
}

// Does slice sg sweep its Ising chain in one persistent launch per call?
static bool slice_persistent(const pyro_sw_group *g, const SubGroup &sg)
{
    return g->ising_mode == PYRO_MODE_PERSISTENT && sg.chains[0].chain.nreps > 0;
}

// Chains of slice sg swept by one graph per sweep.
static int per_sweep_chains(const pyro_sw_group *g, const SubGroup &sg, Chain *cs)
{
    int nc = 0;
    for (int m = 0; m < 3; ++m) {
        const ChainTables &ct = sg.chains[m];
        if (ct.chain.nreps == 0 || (m == 0 && slice_persistent(g, sg))) continue;
        cs[nc++] = ct.chain;
    }
    return nc;
}

// Run `reps` armed sweeps: graph replays (per-sweep graphs `reps` times, the
// persistent and LDS-resident launches once, since they run every armed
// sweep themselves), or timed direct launches.
static int group_run(pyro_sw_group *g, int64_t reps)
{
    Timer &tm = g->timer;
    const LaunchHook none{nullptr, nullptr, nullptr};
    if (tm.mask) {  // every kernel in order on the group's stream
        const LaunchHook hook = hook_of(tm, g->stream);
        if (g->res.chain.nreps > 0)
            HIP_OR_FAIL(&g->broken, launch_resident_ising(g->res.chain, g->res_maxL, g->stream, hook));
        for (auto &sg : g->subs)
            if (slice_persistent(g, sg))
                HIP_OR_FAIL(&g->broken, launch_ising_persistent(sg.chains[0].chain, sg.chains[0].d_ctl,
                                                                sg.chains[0].persist_grid, g->stream, hook));
        for (int64_t k = 0; k < reps; ++k) {
            for (auto &sg : g->subs) {
                Chain cs[3];
                const int nc = per_sweep_chains(g, sg, cs);
                for (int q = 0; q < nc; ++q) HIP_OR_FAIL(&g->broken, launch_chain_sweep(cs[q], g->stream, hook));
            }
            if (tm.inflight.size() > 8192) HIP_OR_FAIL(&g->broken, tm.collect());
        }
        return PYRO_OK;
    }
    for (auto &sg : g->subs) {
        Chain cs[3];
        const int nc = per_sweep_chains(g, sg, cs);
        if (!sg.exec && nc > 0) HIP_OR_FAIL(&g->broken, capture_sweep(cs, nc, &sg.exec));
        if (!sg.pexec && slice_persistent(g, sg)) {
            const ChainTables &ct = sg.chains[0];
            HIP_OR_FAIL(&g->broken, capture_graph(
                                        [&](hipStream_t cs2) {
                                            return launch_ising_persistent(ct.chain, ct.d_ctl, ct.persist_grid, cs2,
                                                                           none);
                                        },
                                        &sg.pexec));
        }
    }
    if (!g->rexec && g->res.chain.nreps > 0)
        HIP_OR_FAIL(&g->broken, capture_graph(
                                    [&](hipStream_t cs2) { return launch_resident_ising(g->res.chain, g->res_maxL, cs2, none); },
                                    &g->rexec));
    auto run_slice = [&](SubGroup &sg, hipStream_t st) -> int {
        if (sg.pexec) HIP_OR_FAIL(&g->broken, hipGraphLaunch(sg.pexec, st));
        if (sg.exec)
            for (int64_t k = 0; k < reps; ++k) HIP_OR_FAIL(&g->broken, hipGraphLaunch(sg.exec, st));
        return PYRO_OK;
    };
    if (g->subs.size() == 1 && !g->rexec) return run_slice(g->subs[0], g->stream);
    // fork the slices (and the LDS-resident launch) off the group's stream
    // and join them back
    HIP_OR_FAIL(&g->broken, hipEventRecord(g->fork, g->stream));
    if (g->rexec) {
        HIP_OR_FAIL(&g->broken, hipStreamWaitEvent(g->res_stream, g->fork, 0));
        HIP_OR_FAIL(&g->broken, hipGraphLaunch(g->rexec, g->res_stream));
        HIP_OR_FAIL(&g->broken, hipEventRecord(g->res_join, g->res_stream));
    }
    if (g->subs.size() == 1) {
        if (int rc = run_slice(g->subs[0], g->stream)) return rc;
    } else {
        // The slices' sweeps are enqueued round robin in blocks of
        // kEnqueueBlock: enqueued slice by slice, a long call filled the
        // first slice's queue and blocked the host there while the other
        // slices had no work yet (one call of 10^4 sweeps of five L = 128
        // lattices ran at 1.55 ms per step instead of 1.42).
        constexpr int64_t kEnqueueBlock = 64;
        for (auto &sg : g->subs) {
            HIP_OR_FAIL(&g->broken, hipStreamWaitEvent(sg.stream, g->fork, 0));
            if (sg.pexec) HIP_OR_FAIL(&g->broken, hipGraphLaunch(sg.pexec, sg.stream));
        }
        for (int64_t k0 = 0; k0 < reps; k0 += kEnqueueBlock)
            for (auto &sg : g->subs)
                for (int64_t k = k0; k < std::min(reps, k0 + kEnqueueBlock); ++k)
                    if (sg.exec) HIP_OR_FAIL(&g->broken, hipGraphLaunch(sg.exec, sg.stream));
        for (auto &sg : g->subs) {
            HIP_OR_FAIL(&g->broken, hipEventRecord(sg.join, sg.stream));
            HIP_OR_FAIL(&g->broken, hipStreamWaitEvent(g->stream, sg.join, 0));
        }
    }
    if (g->rexec) HIP_OR_FAIL(&g->broken, hipStreamWaitEvent(g->stream, g->res_join, 0));
    return PYRO_OK;
}

int pyro_sw_group_sweep(pyro_sw_group *g, int64_t n_sweeps, const int64_t *per_member)
{
    if (!g) return fail(PYRO_EINVAL, "group is NULL");
    if (g->broken) return fail(PYRO_ESTATE, "group failed earlier");
    if (n_sweeps < 0) return fail(PYRO_EINVAL, "n_sweeps must be >= 0");
    const int n = (int)g->members.size();
    std::vector<int64_t> want(n);
    for (int i = 0; i < n; ++i) {
        want[i] = per_member ? per_member[i] : n_sweeps;
        if (want[i] < 0) return fail(PYRO_EINVAL, "per-member sweep counts must be >= 0");
        int rc = usable(g->members[i]);
        if (rc) return rc;
        if ((int64_t)g->members[i]->hs.t + want[i] > (int64_t)UINT32_MAX)
            return fail(PYRO_EINVAL, "sweep index would exceed 2^32 - 1");
    }
    int rc = group_prepare(g);
    if (rc) return rc;
    for (;;) {
        int64_t chunk = 0;
        for (int i = 0; i < n; ++i) chunk = std::max(chunk, std::min<int64_t>(want[i], g->persist_cap));
        if (chunk == 0) break;
        for (int i = 0; i < n; ++i) {
            pyro_sw *h = g->members[i];
            rc = make_room(h, std::min<int64_t>(want[i], chunk));
            if (rc) return rc;
            if (h->stream != g->stream) HIP_OR_FAIL(&g->broken, hipStreamSynchronize(h->stream));
        }
        for (int first = 0; first < n; first += kArmBatch) {
            ArmBatch b{};
            const int cnt = std::min(kArmBatch, n - first);
            for (int i = 0; i < cnt; ++i) {
                b.v[i] = g->members[first + i]->hs;
                b.v[i].remaining = (int32_t)std::min<int64_t>(want[first + i], chunk);
            }
            k_arm<<<1, kArmBatch, 0, g->stream>>>(g->d_members, b, first, cnt);
            HIP_OR_FAIL(&g->broken, hipGetLastError());
        }
        for (auto *h : g->members) h->busy++;
        rc = group_run(g, chunk);
        for (auto *h : g->members) h->busy--;
        if (rc) return rc;
        for (int i = 0; i < n; ++i) {
            pyro_sw *h = g->members[i];
            const int64_t k = std::min<int64_t>(want[i], chunk);
            if (k > 0) {
                h->hs.t += (uint32_t)k;
                h->hs.ring_used += (int32_t)k;
                h->hs.e_pending = h->hs.ring_used - 1;
            }
            h->hs.remaining = 0;
            want[i] -= k;
        }
    }
    // members' later calls on their own streams must see this work
    bool other = false;
    for (auto *h : g->members) other |= h->stream != g->stream;
    if (other) HIP_OR_FAIL(&g->broken, hipStreamSynchronize(g->stream));
    return PYRO_OK;
}

int pyro_sw_group_set_slices(pyro_sw_group *g, int nslices)
{
    if (!g) return fail(PYRO_EINVAL, "group is NULL");
    if (g->broken) return fail(PYRO_ESTATE, "group failed earlier");
    if (nslices < 1 || nslices > kMaxSlices) return fail(PYRO_EINVAL, "nslices must be in [1, 8]");
    HIP_OR_FAIL(&g->broken, hipStreamSynchronize(g->stream));
    return make_slices(g, std::min(nslices, (int)g->members.size()));
}

int pyro_sw_group_set_tile_shape(pyro_sw_group *g, int model, int shape)
{
    if (!g) return fail(PYRO_EINVAL, "group is NULL");
    if (model < 1 || model > 3 || shape < 0 || shape >= kNumTileShapes)
        return fail(PYRO_EINVAL, "bad model or shape");
    g->chains[model - 1].shape = shape;
    g->tables_dirty = true;
    return PYRO_OK;
}

int pyro_sw_group_set_mode(pyro_sw_group *g, int ising_mode, int resident)
{
    if (!g) return fail(PYRO_EINVAL, "group is NULL");
    if (g->broken) return fail(PYRO_ESTATE, "group failed earlier");
    if (ising_mode != PYRO_MODE_GRAPH && ising_mode != PYRO_MODE_PERSISTENT)
        return fail(PYRO_EINVAL, "ising_mode must be PYRO_MODE_GRAPH or PYRO_MODE_PERSISTENT");
    if (ising_mode == PYRO_MODE_PERSISTENT && persist_grid_for(g->chains[0].shape) == 0)
        return fail(PYRO_EDEVICE, "no persistent launch fits the device");
    g->ising_mode = ising_mode;
    g->resident = resident != 0;
    g->tables_dirty = true;
    return PYRO_OK;
}

int pyro_sw_group_set_counting(pyro_sw_group *g, int on)
{
    if (!g) return fail(PYRO_EINVAL, "group is NULL");
    if (g->broken) return fail(PYRO_ESTATE, "group failed earlier");
    HIP_OR_FAIL(&g->broken, hipStreamSynchronize(g->stream));
    if (on && !g->d_counts) {
        if (hipMalloc((void **)&g->d_counts, 2 * sizeof(unsigned long long)) != hipSuccess) {
            (void)hipGetLastError();
            g->d_counts = nullptr;
            return fail(PYRO_ENOMEM, "counters");
        }
    }
    if (on) HIP_OR_FAIL(&g->broken, hipMemset(g->d_counts, 0, 2 * sizeof(unsigned long long)));
    g->counting = on != 0;
    g->tables_dirty = true;
    return PYRO_OK;
}

int pyro_sw_group_counts(pyro_sw_group *g, int64_t *cas_tried, int64_t *cas_hooked)
{
    if (!g) return fail(PYRO_EINVAL, "group is NULL");
    if (!cas_tried || !cas_hooked) return fail(PYRO_EINVAL, "outputs must not be NULL");
    unsigned long long v[2] = {0, 0};
    if (g->d_counts) {
        HIP_OR_FAIL(&g->broken, hipStreamSynchronize(g->stream));
        HIP_OR_FAIL(&g->broken, hipMemcpy(v, g->d_counts, sizeof(v), hipMemcpyDeviceToHost));
    }
    *cas_tried = (int64_t)v[0];
    *cas_hooked = (int64_t)v[1];
    return PYRO_OK;
}

int pyro_sw_group_get_mode(const pyro_sw_group *g, int *ising_mode, int *resident)
{
    if (!g) return fail(PYRO_EINVAL, "group is NULL");
    if (ising_mode) *ising_mode = g->ising_mode;
    if (resident) *resident = g->resident ? 1 : 0;
    return PYRO_OK;
}

int pyro_sw_group_autotune(pyro_sw_group *g, int trial_sweeps, int *shapes_out)
{
    if (!g) return fail(PYRO_EINVAL, "group is NULL");
    if (g->broken) return fail(PYRO_ESTATE, "group failed earlier");
    if (trial_sweeps < 1 || trial_sweeps > 1000) return fail(PYRO_EINVAL, "trial_sweeps must be in [1, 1000]");
    const int n = (int)g->members.size();
    // Save every member: spins and the mirrored sweep state (records so far
    // are first moved to the member's host queue).
    std::vector<void *> saved(n, nullptr);
    std::vector<RepState> saved_hs(n);
    std::vector<size_t> bytes(n);
    int rc = PYRO_OK;
    for (int i = 0; i < n && rc == PYRO_OK; ++i) {
        pyro_sw *h = g->members[i];
        rc = usable(h);
        if (rc == PYRO_OK) rc = drain(h);
        if (rc) break;
        bytes[i] = h->model == PYRO_ISING ? (size_t)h->N : sizeof(float) * h->model * (size_t)h->N;
        if (hipMalloc(&saved[i], bytes[i]) != hipSuccess) {
            (void)hipGetLastError();
            rc = fail(PYRO_ENOMEM, "autotune backup");
            break;
        }
        if (hipMemcpy(saved[i], h->spins, bytes[i], hipMemcpyDeviceToDevice) != hipSuccess)
            rc = device_fail(&g->broken, hipErrorUnknown, "autotune backup copy");
        saved_hs[i] = h->hs;
    }
    // Every timed trial starts from the saved state, so that every candidate
    // runs the same sweeps of the same lattices.  Sweep times depend on the
    // state (clusters grow over the first sweeps from a random start): timed
    // one after another from a drifting state, the candidates tried first
    // were favoured.
    auto restore = [&](int model) {
        if (hipStreamSynchronize(g->stream) != hipSuccess)
            return device_fail(&g->broken, hipErrorUnknown, "autotune synchronize");
        for (int i = 0; i < n; ++i) {
            pyro_sw *h = g->members[i];
            if (!saved[i] || h->model != model) continue;
            hipStreamSynchronize(h->stream);
            if (hipMemcpy(h->spins, saved[i], bytes[i], hipMemcpyDeviceToDevice) != hipSuccess)
                return device_fail(&g->broken, hipErrorUnknown, "autotune restore");
            h->hs = saved_hs[i];
            h->hs.ring_used = 0;
            h->hs.e_pending = -1;
        }
        return (int)PYRO_OK;
    };
    for (int m = 0; m < 3 && rc == PYRO_OK; ++m) {
        ChainTables &ct = g->chains[m];
        if (ct.reps.empty()) continue;
        // candidates: every tile shape per-sweep; for Ising also the
        // persistent launch with the shapes whose workgroups fit it well,
        // each with and without the LDS-resident small lattices
        std::vector<TuneChoice> cands;
        bool small = false;
        for (const pyro_sw *h : ct.reps) small |= h->model == PYRO_ISING && h->L <= kResidentMaxL && !h->diluted;
        for (int res = 0; res < ((m == 0 && small) ? 2 : 1); ++res) {
            for (int s = 0; s < kNumTileShapes; ++s) cands.push_back({s, PYRO_MODE_GRAPH, res != 0});
            if (m == 0)
                for (int s : {kTile888, kTile884, kTile844})
                    if (persist_grid_for(s) > 0) cands.push_back({s, PYRO_MODE_PERSISTENT, res != 0});
        }
        double best = 1e300;
        TuneChoice best_c{ct.shape, g->ising_mode, g->resident};
        std::vector<int64_t> per(n, 0);
        for (int i = 0; i < n; ++i)
            if (g->members[i]->model == m + 1) per[i] = trial_sweeps;
        for (const TuneChoice &cand : cands) {
            if (rc != PYRO_OK) break;
            ct.shape = cand.shape;
            if (m == 0) {
                g->ising_mode = cand.ising_mode;
                g->resident = cand.resident;
            }
            g->tables_dirty = true;
            rc = restore(m + 1);
            if (rc == PYRO_OK) rc = pyro_sw_group_sweep(g, 0, per.data());  // builds tables and graphs, warms caches
            if (rc) break;
            float ms = 1e30f;  // the faster of two timed trials
            for (int rep = 0; rep < 2 && rc == PYRO_OK; ++rep) {
                rc = restore(m + 1);
                if (rc) break;
                hipEvent_t e0 = nullptr, e1 = nullptr;
                hipEventCreate(&e0);
                hipEventCreate(&e1);
                hipEventRecord(e0, g->stream);
                rc = pyro_sw_group_sweep(g, 0, per.data());
                hipEventRecord(e1, g->stream);
                hipEventSynchronize(e1);
                float t = 0.f;
                hipEventElapsedTime(&t, e0, e1);
                hipEventDestroy(e0);
                hipEventDestroy(e1);
                ms = std::min(ms, t);
            }
            if (rc == PYRO_OK && ms < best) {
                best = ms;
                best_c = cand;
            }
        }
        ct.shape = best_c.shape;
        if (m == 0) {
            g->ising_mode = best_c.ising_mode;
            g->resident = best_c.resident;
        }
        g->tables_dirty = true;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[tune_key(ct)] = best_c;
    }
    // Restore every member exactly, dropping the trial records.
    hipStreamSynchronize(g->stream);
    for (int i = 0; i < n; ++i) {
        pyro_sw *h = g->members[i];
        if (!saved[i]) continue;
        hipStreamSynchronize(h->stream);
        if (hipMemcpy(h->spins, saved[i], bytes[i], hipMemcpyDeviceToDevice) != hipSuccess && rc == PYRO_OK)
            rc = device_fail(&g->broken, hipErrorUnknown, "autotune restore");
        hipFree(saved[i]);
        h->hs = saved_hs[i];
        h->hs.ring_used = 0;
        h->hs.e_pending = -1;
    }
    if (shapes_out)
        for (int m = 0; m < 3; ++m) shapes_out[m] = g->chains[m].shape;
    return rc;
}

int pyro_sw_group_set_timing(pyro_sw_group *g, int kernel_mask)
{
    if (!g) return fail(PYRO_EINVAL, "group is NULL");
    g->timer.stream = g->stream;
    HIP_OR_FAIL(&g->broken, g->timer.collect());
    g->timer.reset(kernel_mask);
    return PYRO_OK;
}

int pyro_sw_group_kernel_times(pyro_sw_group *g, const char **names, int64_t *launches, double *ms, int cap,
                               int *n_out)
{
    if (!g) return fail(PYRO_EINVAL, "group is NULL");
    return report_times(g->timer, &g->broken, names, launches, ms, cap, n_out);
}

int pyro_sw_group_destroy(pyro_sw_group *g)
{
    if (!g) return PYRO_OK;
    int rc = PYRO_OK;
    if (g->stream && hipStreamSynchronize(g->stream) != hipSuccess) rc = fail(PYRO_EDEVICE, "synchronize failed");
    g->timer.release();
    drop_slices(g);
    free_tables(g->res);
    if (g->d_counts) hipFree(g->d_counts);
    if (g->res_stream) {
        hipStreamSynchronize(g->res_stream);
        hipStreamDestroy(g->res_stream);
    }
    if (g->res_join) hipEventDestroy(g->res_join);
    if (g->fork) hipEventDestroy(g->fork);
    if (g->d_members) hipFreeAsync(g->d_members, g->stream);
    if (g->own_stream) hipStreamDestroy(g->stream);
    delete g;
    return rc;
}

const char *pyro_sw_strerror(int status)
{
    switch (status) {
    case PYRO_OK: return "ok";
    case PYRO_EINVAL: return "invalid argument";
    case PYRO_ENOMEM: return "out of memory";
    case PYRO_EDEVICE: return "HIP device error";
    case PYRO_ESTATE: return "handle in failed state";
    default: return "unknown status";
    }
}

const char *pyro_sw_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
