// C-ABI layer of the pyrochlore Swendsen-Wang library (declared in
// include/pyro_sw.h): argument checks, device memory, the per-sweep record
// ring, kernel timing and error state.  No arithmetic of the method lives
// here except the two per-run constants of Sec. 2 that every kernel reads:
// the Ising activation threshold floor((1 - exp(-2J/T)) 2^32) and the O(n)
// coupling x0 = (float)(2J/T).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <deque>
#include <new>
#include <string>
#include <vector>

#include "../../include/pyro_sw.h"
#include "kernels.hpp"

using namespace pyro;

static_assert(sizeof(pyro_sw_record) == sizeof(DevRecord), "record layout");
static_assert(sizeof(pyro_sw_record) == 80, "record size");

namespace {

thread_local std::string g_last_error;

int fail(int status, const std::string &msg)
{
    g_last_error = msg;
    return status;
}

constexpr int64_t kRing = 16384;  // device records before a forced drain
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t spin_bytes, label, mask, flip, sigma, axis, ipart, dpart, ring, total;
};

Layout layout_for(int L, int model)
{
    const int64_t ncell = (int64_t)L * L * L;
    const int64_t N = 16 * ncell;
    const int n = model;
    Layout ly{};
    ly.spin_bytes = align_up(model == PYRO_ISING ? (size_t)N : sizeof(float) * (size_t)n * N);
    size_t off = 0;
    ly.label = off;
    off += align_up(sizeof(int32_t) * (size_t)N);
    ly.mask = off;
    off += align_up(sizeof(uint64_t) * (size_t)ncell);
    ly.flip = off;
    off += align_up(16 * (size_t)((N + 127) / 128));
    ly.sigma = off;
    off += model == PYRO_ISING ? 0 : align_up(sizeof(float) * (size_t)N);
    ly.axis = off;
    off += kAlign;
    const int64_t nblk = blocks_for(ncell);
    ly.ipart = off;
    off += align_up(sizeof(int64_t) * 2 * (size_t)nblk);
    ly.dpart = off;
    off += model == PYRO_ISING ? 0 : align_up(sizeof(double) * 4 * (size_t)nblk);
    ly.ring = off;
    off += align_up(sizeof(pyro_sw_record) * (size_t)kRing);
    ly.total = off;
    return ly;
}

int check_args(int L, int model, double T, double J, int start)
{
    if (L < 1 || L > 447) return fail(PYRO_EINVAL, "L must be in [1, 447]");
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

}  // namespace

struct pyro_sw {
    int L = 0, model = 0;
    int64_t ncell = 0, N = 0;
    double T = 0, J = 0;
    uint64_t seed = 0;
    int start = 0;
    IsingParams ip{};
    float x0 = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool own_mem = false;
    void *spins = nullptr;
    char *work = nullptr;
    Layout ly{};
    SweepBuffers buf{};
    int64_t ring_used = 0;
    std::deque<pyro_sw_record> host_q;
    int64_t t = 0;
    bool broken = false;
    // timing
    int timing = 0;  // bit mask of timed kernel ids
    std::vector<TimedLaunch> inflight;
    std::vector<hipEvent_t> pool;
    double ms[kNumKernels] = {};
    int64_t launches[kNumKernels] = {};
};

namespace {

int device_fail(pyro_sw *h, hipError_t e, const char *what)
{
    if (h) h->broken = true;
    return fail(PYRO_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_OR_FAIL(h, call)                                 \
    do {                                                     \
        hipError_t e__ = (call);                             \
        if (e__ != hipSuccess) return device_fail(h, e__, #call); \
    } while (0)

void set_params(pyro_sw *h, double T)
{
    h->T = T;
    const double twobj = 2.0 * h->J / T;
    const double p = -expm1(-twobj);
    const uint64_t thr = (uint64_t)floor(p * 4294967296.0);
    h->ip.thr_hi = (uint32_t)(thr >> 24);
    h->ip.thr_lo = (uint32_t)(thr & 0xFFFFFFu);
    h->x0 = (float)twobj;
}

hipEvent_t take_event(pyro_sw *h)
{
    if (!h->pool.empty()) {
        hipEvent_t e = h->pool.back();
        h->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void hook_before(void *ctx, int id)
{
    pyro_sw *h = (pyro_sw *)ctx;
    if (!((h->timing >> id) & 1)) return;
    TimedLaunch tl{id, take_event(h), take_event(h)};
    if (tl.e0 && tl.e1) {
        hipEventRecord(tl.e0, h->stream);
        h->inflight.push_back(tl);
    }
}

void hook_after(void *ctx, int id)
{
    pyro_sw *h = (pyro_sw *)ctx;
    if (!h->inflight.empty() && h->inflight.back().id == id) hipEventRecord(h->inflight.back().e1, h->stream);
}

// Fold completed timed launches into the totals (synchronises).
int collect_timing(pyro_sw *h)
{
    if (h->inflight.empty()) return PYRO_OK;
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    for (auto &tl : h->inflight) {
        float ms = 0.f;
        HIP_OR_FAIL(h, hipEventElapsedTime(&ms, tl.e0, tl.e1));
        h->ms[tl.id] += ms;
        h->launches[tl.id] += 1;
        h->pool.push_back(tl.e0);
        h->pool.push_back(tl.e1);
    }
    h->inflight.clear();
    return PYRO_OK;
}

int drain(pyro_sw *h)
{
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    if (h->ring_used > 0) {
        std::vector<pyro_sw_record> tmp((size_t)h->ring_used);
        HIP_OR_FAIL(h, hipMemcpy(tmp.data(), h->buf.ring, sizeof(pyro_sw_record) * tmp.size(),
                                 hipMemcpyDeviceToHost));
        for (auto &r : tmp) h->host_q.push_back(r);
        h->ring_used = 0;
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
    Layout ly = layout_for(L, model);
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
            if (h->spins && e1 == hipSuccess) hipFree(h->spins);
            if (h->own_stream) hipStreamDestroy(h->stream);
            delete h;
            (void)hipGetLastError();
            return fail(PYRO_ENOMEM, "hipMalloc failed");
        }
        h->own_mem = true;
    }
    SweepBuffers &b = h->buf;
    b.L = L;
    b.ncell = h->ncell;
    b.N = h->N;
    b.spins = h->spins;
    b.label = (int32_t *)(h->work + ly.label);
    b.mask = (uint64_t *)(h->work + ly.mask);
    b.flipbits = (uint32_t *)(h->work + ly.flip);
    b.sigma = model == PYRO_ISING ? nullptr : (float *)(h->work + ly.sigma);
    b.axis = (float *)(h->work + ly.axis);
    b.ipart = (int64_t *)(h->work + ly.ipart);
    b.dpart = model == PYRO_ISING ? nullptr : (double *)(h->work + ly.dpart);
    b.ring = (DevRecord *)(h->work + ly.ring);
    const PhiloxKey key = philox_key(seed);
    hipError_t e = model == PYRO_ISING ? launch_init_ising(b, start, key, h->stream)
                                       : launch_init_on(b, model, start, key, h->stream);
    if (e == hipSuccess) e = launch_identity_labels(b, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        int r = fail(PYRO_EDEVICE, std::string("initial state: ") + hipGetErrorString(e));
        pyro_sw_destroy(h);
        return r;
    }
    *out = h;
    return PYRO_OK;
}

int usable(const pyro_sw *h)
{
    if (!h) return fail(PYRO_EINVAL, "handle is NULL");
    if (h->broken) return fail(PYRO_ESTATE, "handle failed earlier");
    return PYRO_OK;
}

}  // namespace

extern "C" {

int pyro_sw_workspace_size(int L, int model, size_t *spin_bytes, size_t *work_bytes)
{
    if (L < 1 || L > 447) return fail(PYRO_EINVAL, "L must be in [1, 447]");
    if (model < PYRO_ISING || model > PYRO_HEISENBERG) return fail(PYRO_EINVAL, "model must be 1, 2 or 3");
    Layout ly = layout_for(L, model);
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
    if (h->t + n_sweeps > (int64_t)UINT32_MAX) return fail(PYRO_EINVAL, "sweep index would exceed 2^32 - 1");
    const PhiloxKey key = philox_key(h->seed);
    LaunchHook hook{nullptr, nullptr, h};
    if (h->timing) {
        hook.before = hook_before;
        hook.after = hook_after;
    }
    for (int64_t k = 0; k < n_sweeps; ++k) {
        if (h->ring_used == kRing) {
            rc = drain(h);
            if (rc) return rc;
        }
        if (h->timing && h->inflight.size() > 8192) {
            rc = collect_timing(h);
            if (rc) return rc;
        }
        const uint32_t t = (uint32_t)h->t;
        hipError_t e = h->model == PYRO_ISING
                           ? launch_sweep_ising(h->buf, h->ip, h->J, key, t, (int)h->ring_used, h->stream, hook)
                           : launch_sweep_on(h->buf, h->model, h->x0, h->J, key, t, (int)h->ring_used,
                                             h->stream, hook);
        if (e != hipSuccess) return device_fail(h, e, "sweep launch");
        h->ring_used++;
        h->t++;
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
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    HIP_OR_FAIL(h, hipMemcpy(host, h->spins, need, hipMemcpyDeviceToHost));
    return PYRO_OK;
}

int pyro_sw_set_spins(pyro_sw *h, const void *host, size_t bytes, int64_t next_sweep)
{
    int rc = usable(h);
    if (rc) return rc;
    const size_t need = h->model == PYRO_ISING ? (size_t)h->N : sizeof(float) * h->model * (size_t)h->N;
    if (!host || bytes != need) return fail(PYRO_EINVAL, "host buffer size must equal the spin array size");
    if (next_sweep < 0 || next_sweep > (int64_t)UINT32_MAX) return fail(PYRO_EINVAL, "bad sweep index");
    if (h->model == PYRO_ISING) {
        const int8_t *s = (const int8_t *)host;
        for (int64_t i = 0; i < h->N; ++i)
            if (s[i] != 1 && s[i] != -1) return fail(PYRO_EINVAL, "Ising spins must be +1 or -1");
    }
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    HIP_OR_FAIL(h, hipMemcpy(h->spins, host, need, hipMemcpyHostToDevice));
    h->t = next_sweep;
    h->ring_used = 0;
    h->host_q.clear();
    return PYRO_OK;
}

int pyro_sw_get_labels(pyro_sw *h, int32_t *host, size_t n)
{
    int rc = usable(h);
    if (rc) return rc;
    if (!host || n != (size_t)h->N) return fail(PYRO_EINVAL, "n must equal N");
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    HIP_OR_FAIL(h, hipMemcpy(host, h->buf.label, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
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

int pyro_sw_info(const pyro_sw *h, int64_t *n_sites, int64_t *next_sweep)
{
    if (!h) return fail(PYRO_EINVAL, "handle is NULL");
    if (n_sites) *n_sites = h->N;
    if (next_sweep) *next_sweep = h->t;
    return PYRO_OK;
}

int pyro_sw_set_timing(pyro_sw *h, int kernel_mask)
{
    int rc = usable(h);
    if (rc) return rc;
    rc = collect_timing(h);
    if (rc) return rc;
    h->timing = kernel_mask;
    for (int k = 0; k < kNumKernels; ++k) {
        h->ms[k] = 0.0;
        h->launches[k] = 0;
    }
    return PYRO_OK;
}

int pyro_sw_kernel_times(pyro_sw *h, const char **names, int64_t *launches, double *ms, int cap, int *n_out)
{
    int rc = usable(h);
    if (rc) return rc;
    if (!n_out || cap < 0) return fail(PYRO_EINVAL, "bad output arguments");
    rc = collect_timing(h);
    if (rc) return rc;
    int n = 0;
    for (int k = 0; k < kNumKernels && n < cap; ++k) {
        if (names) names[n] = kernel_name(k);
        if (launches) launches[n] = h->launches[k];
        if (ms) ms[n] = h->ms[k];
        ++n;
    }
    *n_out = n;
    return PYRO_OK;
}

int pyro_sw_destroy(pyro_sw *h)
{
    if (!h) return PYRO_OK;
    int rc = PYRO_OK;
    if (h->stream && hipStreamSynchronize(h->stream) != hipSuccess) rc = fail(PYRO_EDEVICE, "synchronize failed");
    for (auto &tl : h->inflight) {
        hipEventDestroy(tl.e0);
        hipEventDestroy(tl.e1);
    }
    for (auto e : h->pool) hipEventDestroy(e);
    if (h->own_mem) {
        hipFree(h->spins);
        hipFree(h->work);
    }
    if (h->own_stream) hipStreamDestroy(h->stream);
    delete h;
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
