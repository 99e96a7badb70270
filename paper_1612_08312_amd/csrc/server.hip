// Job server with continuous batching over the handle and group API of
// this library (declarations and the scheduling contract in
// include/pyro_sw.h).
//
// One device allocation (the budget) is carved by a host-side first-fit
// arena into job regions; each admitted job is a handle created on that
// region (pyro_sw_init_ext) and on its lane's stream.  A lane is a group of
// running jobs of similar lattice size advanced one quantum at a time; its
// membership is rebuilt only while the lane is idle, so admission,
// retirement and group rebuilds never wait for another lane's work (group
// tables use stream-ordered allocation).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <memory>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/pyro_sw.h"
#include "arena.hpp"
#include "kernels.hpp"

using namespace pyro;

namespace {

constexpr int kLanes = 5;
constexpr int kLaneMaxL[kLanes] = {16, 40, 72, 136, 1 << 30};
constexpr int64_t kMaxQuantum = 16384;  // sweeps per member per quantum (one record ring)
constexpr size_t kAlign = 256;

size_t round_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int lane_of(int L)
{
    int k = 0;
    while (L > kLaneMaxL[k]) ++k;
    return k;
}

struct Job {
    int64_t id = 0;
    pyro_sw_job spec{};
    int state = PYRO_JOB_QUEUED;
    int lane = -1;
    int error = 0;
    double t_submit = -1, t_admit = -1, t_done = -1;
    size_t spin_bytes = 0, work_bytes = 0, footprint = 0;
    size_t off = Arena::kNone;
    pyro_sw *h = nullptr;
    int64_t remaining = 0, done = 0;
    std::vector<pyro_sw_record> recs;
    std::vector<char> spins;
};

struct Lane {
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    pyro_sw_group *g = nullptr;
    std::vector<Job *> members;
    bool dirty = false, busy = false;
    int64_t replays = 0;
    double ms_per_replay = -1.0;  // measured, exponentially averaged
};

int job_footprint(const pyro_sw_job &j, size_t *spin, size_t *work)
{
    size_t s = 0, w = 0;
    const int rc = pyro_sw_workspace_size(j.L, j.model, &s, &w);
    if (rc) return rc;
    *spin = round_up(s);
    *work = round_up(w);
    return PYRO_OK;
}

}  // namespace

struct pyro_sw_server {
    char *base = nullptr;
    Arena arena;
    int max_running = 1, running = 0;
    double quantum_ms = 10.0, starve_ms = 0.0;
    std::deque<Job *> queue;
    std::unordered_map<int64_t, std::unique_ptr<Job>> jobs;
    int64_t next_id = 1;
    Lane lanes[kLanes];
    std::chrono::steady_clock::time_point t0;
    bool broken = false;

    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

namespace {

int server_fail(pyro_sw_server *s, int status, const char *msg)
{
    if (status == PYRO_EDEVICE) s->broken = true;
    return record_error(status, msg);
}

// Copy out a finished job's results and give its memory back.
int finish_job(pyro_sw_server *s, Job *j)
{
    int rc = PYRO_OK;
    int64_t n = 0;
    rc = pyro_sw_moments(j->h, nullptr, 0, &n);
    if (rc == PYRO_OK) {
        j->recs.resize((size_t)n);
        rc = pyro_sw_moments(j->h, j->recs.data(), n, &n);
    }
    if (rc == PYRO_OK && j->spec.keep_spins) {
        size_t sb = 0, wb = 0;
        pyro_sw_workspace_size(j->spec.L, j->spec.model, &sb, &wb);
        const int64_t N = 16ll * j->spec.L * j->spec.L * j->spec.L;
        j->spins.resize(j->spec.model == PYRO_ISING ? (size_t)N : sizeof(float) * (size_t)j->spec.model * N);
        rc = pyro_sw_get_spins(j->h, j->spins.data(), j->spins.size());
    }
    pyro_sw_destroy(j->h);
    j->h = nullptr;
    s->arena.release(j->off);
    j->off = Arena::kNone;
    j->error = rc;
    j->state = PYRO_JOB_DONE;
    j->t_done = s->now();
    s->running--;
    return rc;
}

// A lane whose quantum ended: measure it and retire its finished jobs.
int retire(pyro_sw_server *s, Lane &ln)
{
    ln.busy = false;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ln.e0, ln.e1) == hipSuccess && ln.replays > 0) {
        const double per = ms / (double)ln.replays;
        ln.ms_per_replay = ln.ms_per_replay < 0 ? per : 0.5 * ln.ms_per_replay + 0.5 * per;
    }
    std::vector<Job *> keep;
    for (Job *j : ln.members) {
        if (j->remaining > 0) {
            keep.push_back(j);
            continue;
        }
        const int rc = finish_job(s, j);
        if (rc == PYRO_EDEVICE) return server_fail(s, rc, "finishing a job failed on the device");
        ln.dirty = true;
    }
    ln.members.swap(keep);
    if (ln.members.empty() && ln.g) {  // an empty lane holds no group
        pyro_sw_group_destroy(ln.g);
        ln.g = nullptr;
    }
    return PYRO_OK;
}

int poll_lanes(pyro_sw_server *s, bool *progress)
{
    for (Lane &ln : s->lanes) {
        if (!ln.busy) continue;
        const hipError_t q = hipEventQuery(ln.e1);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) return server_fail(s, PYRO_EDEVICE, "lane event failed");
        const int rc = retire(s, ln);
        if (rc) return rc;
        *progress = true;
    }
    return PYRO_OK;
}

int admit(pyro_sw_server *s, bool *progress)
{
    const double t = s->now();
    bool head = true;  // the job being looked at is the oldest still queued
    for (auto it = s->queue.begin(); it != s->queue.end();) {
        if (s->running >= s->max_running) break;
        Job *j = *it;
        Lane &ln = s->lanes[j->lane];
        if (ln.busy) {  // joins when its lane is between quanta
            ++it;
            head = false;
            continue;
        }
        const size_t off = s->arena.alloc(j->footprint);
        if (off == Arena::kNone) {
            if (head && (t - j->t_submit) * 1e3 >= s->starve_ms) break;  // keep the budget for it
            ++it;
            head = false;
            continue;
        }
        pyro_sw *h = nullptr;
        const int rc = pyro_sw_init_ext(&h, j->spec.L, j->spec.model, j->spec.T, j->spec.J, j->spec.seed,
                                        j->spec.start, ln.st, s->base + off, j->spin_bytes,
                                        s->base + off + j->spin_bytes, j->work_bytes);
        if (rc) {
            s->arena.release(off);
            if (rc == PYRO_EDEVICE) return server_fail(s, rc, "job initialisation failed on the device");
            j->error = rc;
            j->state = PYRO_JOB_DONE;
            j->t_admit = j->t_done = s->now();
            it = s->queue.erase(it);
            continue;
        }
        j->h = h;
        j->off = off;
        j->state = PYRO_JOB_RUNNING;
        j->t_admit = s->now();
        j->remaining = j->spec.sweeps;
        s->running++;
        ln.members.push_back(j);
        ln.dirty = true;
        *progress = true;
        it = s->queue.erase(it);
    }
    return PYRO_OK;
}

int launch_quanta(pyro_sw_server *s, bool *progress)
{
    for (Lane &ln : s->lanes) {
        if (ln.busy || ln.members.empty()) continue;
        if (ln.dirty || !ln.g) {
            if (ln.g) pyro_sw_group_destroy(ln.g);
            ln.g = nullptr;
            std::vector<pyro_sw *> hs;
            for (Job *j : ln.members) hs.push_back(j->h);
            int rc = pyro_sw_group_create(&ln.g, hs.data(), (int)hs.size(), ln.st);
            if (!rc) rc = pyro_sw_group_set_slices(ln.g, 1);  // the lanes already run concurrently
            if (rc) return server_fail(s, rc == PYRO_EDEVICE ? rc : PYRO_EDEVICE, "lane group creation failed");
            ln.dirty = false;
        }
        double sites = 0;
        int64_t most = 0;
        for (Job *j : ln.members) {
            sites += 16.0 * j->spec.L * j->spec.L * j->spec.L * (j->spec.model == PYRO_ISING ? 1 : 4);
            most = std::max(most, j->remaining);
        }
        const double per = ln.ms_per_replay > 0 ? ln.ms_per_replay : 0.03 + 2e-8 * sites;
        int64_t q = (int64_t)std::floor(s->quantum_ms / per);
        q = std::max<int64_t>(1, std::min<int64_t>({q, kMaxQuantum, most}));
        std::vector<int64_t> per_member;
        for (Job *j : ln.members) per_member.push_back(std::min(q, j->remaining));
        if (hipEventRecord(ln.e0, ln.st) != hipSuccess) return server_fail(s, PYRO_EDEVICE, "event record");
        const int rc = pyro_sw_group_sweep(ln.g, 0, per_member.data());
        if (rc) return server_fail(s, rc == PYRO_EINVAL ? PYRO_ESTATE : rc, "lane quantum failed");
        if (hipEventRecord(ln.e1, ln.st) != hipSuccess) return server_fail(s, PYRO_EDEVICE, "event record");
        for (size_t i = 0; i < ln.members.size(); ++i) {
            ln.members[i]->remaining -= per_member[i];
            ln.members[i]->done += per_member[i];
        }
        ln.replays = q;
        ln.busy = true;
        *progress = true;
    }
    return PYRO_OK;
}

int round_once(pyro_sw_server *s, bool *progress)
{
    int rc = poll_lanes(s, progress);
    if (!rc) rc = admit(s, progress);
    if (!rc) rc = launch_quanta(s, progress);
    return rc;
}

}  // namespace

extern "C" {

int pyro_sw_server_job_bytes(const pyro_sw_job *job, size_t *bytes)
{
    if (!job || !bytes) return record_error(PYRO_EINVAL, "job and bytes must not be NULL");
    size_t sb = 0, wb = 0;
    const int rc = job_footprint(*job, &sb, &wb);
    if (rc) return rc;
    *bytes = sb + wb;
    return PYRO_OK;
}

int pyro_sw_server_create(pyro_sw_server **out, size_t hbm_budget, int max_running, double quantum_ms,
                          double starve_ms)
{
    if (!out) return record_error(PYRO_EINVAL, "out is NULL");
    *out = nullptr;
    if (hbm_budget < ((size_t)1 << 20)) return record_error(PYRO_EINVAL, "hbm_budget must be >= 1 MiB");
    if (max_running < 1) return record_error(PYRO_EINVAL, "max_running must be >= 1");
    if (!(quantum_ms > 0.0) || std::isinf(quantum_ms)) return record_error(PYRO_EINVAL, "quantum_ms must be > 0");
    if (!(starve_ms >= 0.0)) return record_error(PYRO_EINVAL, "starve_ms must be >= 0");
    pyro_sw_server *s = new (std::nothrow) pyro_sw_server();
    if (!s) return record_error(PYRO_ENOMEM, "host allocation failed");
    s->t0 = std::chrono::steady_clock::now();
    s->max_running = max_running;
    s->quantum_ms = quantum_ms;
    s->starve_ms = starve_ms;
    const size_t budget = hbm_budget / kAlign * kAlign;
    if (hipMalloc((void **)&s->base, budget) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return record_error(PYRO_ENOMEM, "hipMalloc of the server budget failed");
    }
    s->arena = Arena(budget, kAlign);
    for (Lane &ln : s->lanes) {
        if (hipStreamCreateWithFlags(&ln.st, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreate(&ln.e0) != hipSuccess || hipEventCreate(&ln.e1) != hipSuccess) {
            pyro_sw_server_destroy(s);
            return record_error(PYRO_EDEVICE, "lane stream or event creation failed");
        }
    }
    *out = s;
    return PYRO_OK;
}

int pyro_sw_server_submit(pyro_sw_server *s, const pyro_sw_job *job, int64_t *id)
{
    if (!s || !job || !id) return record_error(PYRO_EINVAL, "server, job and id must not be NULL");
    if (s->broken) return record_error(PYRO_ESTATE, "server failed earlier");
    if (job->sweeps < 1 || job->sweeps > INT32_MAX) return record_error(PYRO_EINVAL, "sweeps must be in [1, 2^31-1]");
    if (job->model < PYRO_ISING || job->model > PYRO_HEISENBERG)
        return record_error(PYRO_EINVAL, "model must be 1, 2 or 3");
    if (job->L < 1 || job->L > 406) return record_error(PYRO_EINVAL, "L must be in [1, 406]");
    if (!(job->T > 0.0)) return record_error(PYRO_EINVAL, "T must be > 0 (inf allowed)");
    if (!(job->J > 0.0) || std::isinf(job->J)) return record_error(PYRO_EINVAL, "J must be finite and > 0");
    if (job->start != PYRO_START_COLD && job->start != PYRO_START_RANDOM)
        return record_error(PYRO_EINVAL, "start must be PYRO_START_COLD or PYRO_START_RANDOM");
    auto j = std::unique_ptr<Job>(new (std::nothrow) Job());
    if (!j) return record_error(PYRO_ENOMEM, "host allocation failed");
    int rc = job_footprint(*job, &j->spin_bytes, &j->work_bytes);
    if (rc) return rc;
    j->footprint = j->spin_bytes + j->work_bytes;
    if (j->footprint > s->arena.size()) return record_error(PYRO_ENOMEM, "job footprint exceeds the server budget");
    j->id = s->next_id++;
    j->spec = *job;
    j->lane = lane_of(job->L);
    j->t_submit = s->now();
    *id = j->id;
    s->queue.push_back(j.get());
    s->jobs[j->id] = std::move(j);
    return PYRO_OK;
}

int pyro_sw_server_step(pyro_sw_server *s, double wait_ms, int *n_queued, int *n_running)
{
    if (!s) return record_error(PYRO_EINVAL, "server is NULL");
    if (s->broken) return record_error(PYRO_ESTATE, "server failed earlier");
    if (!(wait_ms >= 0.0)) return record_error(PYRO_EINVAL, "wait_ms must be >= 0");
    bool progress = false;
    int rc = round_once(s, &progress);
    if (!rc && !progress && wait_ms > 0.0) {
        const double until = s->now() + wait_ms * 1e-3;
        bool any_busy = false;
        for (Lane &ln : s->lanes) any_busy |= ln.busy;
        while (any_busy && s->now() < until) {
            bool ended = false;
            for (Lane &ln : s->lanes) {
                if (!ln.busy) continue;
                const hipError_t q = hipEventQuery(ln.e1);
                if (q == hipSuccess) ended = true;
                else if (q != hipErrorNotReady) return server_fail(s, PYRO_EDEVICE, "lane event failed");
            }
            if (ended) break;
            std::this_thread::sleep_for(std::chrono::microseconds(50));
        }
        rc = round_once(s, &progress);
    }
    if (n_queued) *n_queued = (int)s->queue.size();
    if (n_running) *n_running = s->running;
    return rc;
}

int pyro_sw_server_status(pyro_sw_server *s, int64_t id, pyro_sw_job_status *out)
{
    if (!s || !out) return record_error(PYRO_EINVAL, "server and out must not be NULL");
    auto it = s->jobs.find(id);
    if (it == s->jobs.end()) return record_error(PYRO_EINVAL, "unknown job id");
    const Job &j = *it->second;
    pyro_sw_job_status st{};
    st.id = j.id;
    st.state = j.state;
    st.lane = j.state == PYRO_JOB_QUEUED ? -1 : j.lane;
    st.sweeps_done = j.done;
    st.footprint = (int64_t)j.footprint;
    st.error = j.error;
    st.t_submit = j.t_submit;
    st.t_admit = j.t_admit;
    st.t_done = j.t_done;
    *out = st;
    return PYRO_OK;
}

int pyro_sw_server_take(pyro_sw_server *s, int64_t id, pyro_sw_record *out, int64_t cap, int64_t *n_out,
                        void *spins_host, size_t spin_bytes)
{
    if (!s || !n_out) return record_error(PYRO_EINVAL, "server and n_out must not be NULL");
    if (cap < 0 || (cap > 0 && !out)) return record_error(PYRO_EINVAL, "bad output arguments");
    auto it = s->jobs.find(id);
    if (it == s->jobs.end()) return record_error(PYRO_EINVAL, "unknown job id");
    Job &j = *it->second;
    if (j.state != PYRO_JOB_DONE) return record_error(PYRO_ESTATE, "job has not finished");
    if (j.error) return record_error(j.error, "job failed");
    if (cap == 0) {
        *n_out = (int64_t)j.recs.size();
        return PYRO_OK;
    }
    if (spins_host) {
        if (j.spins.empty()) return record_error(PYRO_EINVAL, "job was submitted without keep_spins");
        if (spin_bytes != j.spins.size()) return record_error(PYRO_EINVAL, "spin_bytes does not match the job");
        std::copy(j.spins.begin(), j.spins.end(), (char *)spins_host);
    }
    const int64_t n = std::min<int64_t>(cap, (int64_t)j.recs.size());
    std::copy(j.recs.begin(), j.recs.begin() + n, out);
    *n_out = n;
    s->jobs.erase(it);
    return PYRO_OK;
}

int pyro_sw_server_clock(pyro_sw_server *s, double *seconds)
{
    if (!s || !seconds) return record_error(PYRO_EINVAL, "server and seconds must not be NULL");
    *seconds = s->now();
    return PYRO_OK;
}

int pyro_sw_server_destroy(pyro_sw_server *s)
{
    if (!s) return PYRO_OK;
    int rc = PYRO_OK;
    for (Lane &ln : s->lanes)
        if (ln.st && hipStreamSynchronize(ln.st) != hipSuccess) rc = record_error(PYRO_EDEVICE, "synchronize failed");
    for (Lane &ln : s->lanes) {
        if (ln.g) pyro_sw_group_destroy(ln.g);
        for (Job *j : ln.members)
            if (j->h) pyro_sw_destroy(j->h);
        if (ln.e0) hipEventDestroy(ln.e0);
        if (ln.e1) hipEventDestroy(ln.e1);
        if (ln.st) hipStreamDestroy(ln.st);
    }
    if (s->base) hipFree(s->base);
    delete s;
    return rc;
}

}  // extern "C"
