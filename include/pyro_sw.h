/*
 * pyro_sw.h -- C ABI of the MI355X (gfx950) Swendsen-Wang library for the
 * ferromagnetic O(n) model on the periodic pyrochlore lattice.
 *
 * Method: Soldatov, Nefedev, Komura, Okabe, "Large-scale calculation of
 * ferromagnetic spin systems on the pyrochlore lattice".
 *   - lattice: 16-site cubic unit cell, L x L x L cells, periodic, N = 16 L^3
 *     sites, coordination six (Sec. 2);
 *   - model: H = -J sum_<ij> s_i . s_j with unit n-vectors, n = 1 (Ising),
 *     2 (XY), 3 (Heisenberg) (Sec. 2, Eq. 1);
 *   - update: Swendsen-Wang multi-cluster flips, with Wolff's embedded-cluster
 *     idea for n = 2, 3 (Sec. 1, Sec. 2);
 *   - measurement: M, m = M/N, m^2 and m^4 per sweep for the moment ratio
 *     U = <m^4>/<m^2>^2 (Sec. 3.1, Eq. 2), and E = H.
 *
 * Conventions shared by every call:
 *   - Every call returns PYRO_OK (0) or a negative pyro_status; the text of
 *     the last error on the calling thread is pyro_sw_last_error().
 *   - A handle is not thread-safe: calls on one handle must be serialised.
 *     Distinct handles are independent.
 *   - pyro_sw_sweep only enqueues work on the handle's HIP stream;
 *     pyro_sw_moments, pyro_sw_get_* and pyro_sw_destroy synchronise it.
 *   - Host buffers always belong to the caller.  Device memory passed to
 *     pyro_sw_init_ext belongs to the caller and must outlive the handle.
 *   - After a HIP error a handle returns PYRO_ESTATE from every call except
 *     pyro_sw_destroy.
 *   - Results are a deterministic function of (L, model, T, J, seed, start,
 *     sweep index): cluster labels are the smallest site index of each
 *     cluster and every random draw is keyed by (seed, sweep, stream, unit),
 *     so the trajectory does not depend on launch order or tiling.
 *
 * Site numbering: cell (x, y, z) has index (z*L + y)*L + x; site (cell, f,
 * mu) has index 16*cell + 4*f + mu, at position 4*(x,y,z) + F_f + B_mu in
 * units of a/4, with FCC points F = (0,0,0), (0,2,2), (2,0,2), (2,2,0) and
 * tetrahedral basis B = (0,0,0), (0,1,1), (1,0,1), (1,1,0).
 */
#ifndef PYRO_SW_H
#define PYRO_SW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pyro_sw pyro_sw;

/* Model = number of spin components n (Sec. 2, Eq. 1). */
enum { PYRO_ISING = 1, PYRO_XY = 2, PYRO_HEISENBERG = 3 };

/* Initial state: all spins +1 (Ising) or (1, 0, 0) (O(n)); or drawn from the
 * INIT random stream (independent uniform signs / unit vectors). */
enum { PYRO_START_COLD = 0, PYRO_START_RANDOM = 1 };

typedef enum {
    PYRO_OK = 0,
    PYRO_EINVAL = -1, /* an argument is out of range */
    PYRO_ENOMEM = -2, /* device or host allocation failed */
    PYRO_EDEVICE = -3, /* a HIP call failed; the handle is now unusable */
    PYRO_ESTATE = -4   /* the handle failed earlier, or a call is out of order */
} pyro_status;

/* One record per sweep, describing the state after that sweep (Eq. 1, Eq. 2). */
typedef struct {
    int64_t sweep;    /* global 0-based index of the sweep */
    int64_t bond_sum; /* Ising: sum over the 3N bonds of s_i s_j, exact; O(n): 0 */
    int64_t M_int;    /* Ising: sum of s_i, exact; O(n): 0 */
    int64_t reserved;
    double E;         /* energy -J sum_<ij> s_i . s_j (O(n): FP64 sum of FP32 spins) */
    double M[3];      /* magnetisation vector sum_i s_i (Ising: M[0] = M_int) */
    double m2;        /* m*m with m = |M| / N */
    double m4;        /* m2*m2 */
} pyro_sw_record;

/*
 * Create a simulation of one lattice.
 *   L      number of cubic cells per edge, 1 <= L <= 406 (so that N < 2^30);
 *   model  PYRO_ISING, PYRO_XY or PYRO_HEISENBERG;
 *   T      temperature in units of J/k_B, T > 0; T = +inf is accepted (no bond
 *          is ever activated);
 *   J      coupling, 0 < J < inf (ferromagnet);
 *   seed   64-bit key of every random stream;
 *   start  PYRO_START_COLD or PYRO_START_RANDOM;
 *   stream a hipStream_t on which all work is enqueued, or NULL for a stream
 *          the handle creates and owns.
 * All device memory is allocated by the library and freed by destroy.
 * Errors: PYRO_EINVAL (arguments), PYRO_ENOMEM, PYRO_EDEVICE.
 */
int pyro_sw_init(pyro_sw **out, int L, int model, double T, double J, uint64_t seed,
                 int start, void *stream);

/*
 * Device memory needed by pyro_sw_init_ext for (L, model): spin_bytes for the
 * spin array (Ising: int8 [N]; O(n): float [n][N], component-major) and
 * work_bytes for everything else.  Both are multiples of 256.
 */
int pyro_sw_workspace_size(int L, int model, size_t *spin_bytes, size_t *work_bytes);

/*
 * As pyro_sw_init, but the spin array and the workspace are caller-owned
 * device memory (for example tensors allocated by PyTorch), 256-byte aligned,
 * of at least the sizes pyro_sw_workspace_size returns.  The library writes
 * the initial state into dev_spins.  Errors as pyro_sw_init, plus
 * PYRO_EINVAL for NULL, misaligned or too small buffers.
 */
int pyro_sw_init_ext(pyro_sw **out, int L, int model, double T, double J, uint64_t seed,
                     int start, void *stream, void *dev_spins, size_t spin_bytes,
                     void *dev_work, size_t work_bytes);

/*
 * Enqueue n_sweeps >= 0 Swendsen-Wang sweeps (bond activation, cluster
 * labeling, cluster flips, moments).  Asynchronous on the handle's stream
 * (one captured graph replayed per sweep); records are kept on the device and
 * drained to the host automatically when the device ring of 16384 records
 * fills (which synchronises).  Errors: PYRO_EINVAL (n_sweeps < 0),
 * PYRO_EDEVICE, PYRO_ESTATE.
 */
int pyro_sw_sweep(pyro_sw *h, int64_t n_sweeps);

/*
 * Synchronise and move up to cap records, oldest first, into out[0..cap-1];
 * *n_out receives the number written.  Records not returned stay queued for
 * the next call.  out may be NULL only when cap == 0 (then *n_out is the
 * number queued).
 */
int pyro_sw_moments(pyro_sw *h, pyro_sw_record *out, int64_t cap, int64_t *n_out);

/*
 * Copy the spins to / from host memory in the exchange layout: Ising int8
 * [N] (+1 / -1); O(n) float [n][N], component-major.  bytes must equal that
 * size.  set_spins also sets the global index of the next sweep (random
 * draws depend on it), and discards queued records.  Synchronising.
 *
 * Site dilution (the random-system extension of Sec. 4): a zero spin (Ising
 * 0, O(n) the zero vector) is a vacant site.  It carries no bond, stays its
 * own one-site cluster and stays zero; E sums over bonds with two occupied
 * ends and m = M/N counts all N sites.  For Ising, set_spins with a vacant
 * site allocates one library-owned device array of 8 bytes per cell (the
 * bonds with two occupied ends), kept until pyro_sw_destroy.  Errors:
 * PYRO_EINVAL for an Ising value other than +1, -1, 0; PYRO_ENOMEM.
 */
int pyro_sw_get_spins(pyro_sw *h, void *host, size_t bytes);
int pyro_sw_set_spins(pyro_sw *h, const void *host, size_t bytes, int64_t next_sweep);

/*
 * Cluster label of every site after the last sweep: the smallest site index
 * in its cluster.  n must equal N.  Before the first sweep: label[i] = i.
 * Synchronising.
 */
int pyro_sw_get_labels(pyro_sw *h, int32_t *host, size_t n);

/*
 * Change the temperature (takes effect from the next enqueued sweep).
 * Errors: PYRO_EINVAL for T <= 0 or NaN.
 */
int pyro_sw_set_temperature(pyro_sw *h, double T);

/*
 * Tile shape of the cluster labeling: the lattice is cut into boxes of cells,
 * each labelled in one workgroup's local memory before the boxes are merged.
 * The shape changes speed only, never results (labels are canonical and all
 * draws are keyed by sweep and site or bond).  A new handle uses 8x8x8
 * for L >= 96, 8x8x4 for 48 <= L < 96 and 8x4x4 below (a group without an
 * autotuned shape applies the same rule to its largest L).
 */
enum { PYRO_TILE_8x8x4 = 0, PYRO_TILE_8x4x4 = 1, PYRO_TILE_4x4x4 = 2, PYRO_TILE_8x8x8 = 3, PYRO_TILE_16x8x8 = 4 };
int pyro_sw_set_tile_shape(pyro_sw *h, int shape);

/* Number of sites N and global index of the next sweep. */
int pyro_sw_info(const pyro_sw *h, int64_t *n_sites, int64_t *next_sweep);

/*
 * Kernel timing.  kernel_mask selects kernels by their index in the list
 * pyro_sw_kernel_times returns (bit k = kernel k; -1 = all, 0 = off).  Every
 * launch of a selected kernel is bracketed by HIP events on the handle's
 * stream.  pyro_sw_kernel_times synchronises and returns, per kernel name,
 * the number of timed launches and their summed duration in milliseconds
 * since the last pyro_sw_set_timing call.  names[k] point to static strings;
 * *n_out receives the number of kernels.
 */
int pyro_sw_set_timing(pyro_sw *h, int kernel_mask);
int pyro_sw_kernel_times(pyro_sw *h, const char **names, int64_t *launches, double *ms,
                         int cap, int *n_out);

/*
 * Groups: many lattices (any mix of L, model, T, seed) swept together.  Each
 * sweep of a group is one captured HIP graph whose kernels cover every
 * member (one launch per step of the sweep for all lattices of a model),
 * replayed once per sweep on the group's stream.  Every member's trajectory
 * is bit-identical to sweeping it alone.
 *   pyro_sw_group_create   members stay owned by the caller and must outlive
 *                          the group; stream as in pyro_sw_init.  A lattice
 *                          may belong to several groups but must not be used
 *                          by two calls at once.
 *   pyro_sw_group_sweep    n_sweeps sweeps of every member, or, when
 *                          per_member is not NULL, per_member[i] sweeps of
 *                          member i (members with fewer sweeps idle while the
 *                          others run).  Records go to each member, read with
 *                          pyro_sw_moments on the member.
 *   pyro_sw_group_autotune times trial_sweeps (1..1000) sweeps of each model
 *                          with every tile shape, keeps the fastest per model
 *                          (also for later groups of the same lattice sizes
 *                          in this process), and restores every member's
 *                          spins, sweep index and records, so tuning changes
 *                          no result.  shapes_out[3] (may be NULL) receives
 *                          the shapes for Ising, XY, Heisenberg.
 *   pyro_sw_group_set_tile_shape  fix the shape of one model's lattices.
 *   pyro_sw_group_set_slices  run the members as nslices (1..8) slices,
 *                          each with its own captured sweep and internal
 *                          stream, forked from and joined to the group's
 *                          stream on every call, so that the latency-bound
 *                          passes of one slice overlap the arithmetic of
 *                          another (members are dealt largest first to the
 *                          lightest slice; default min(n, 8)).  Changes speed
 *                          only, never results.
 *   pyro_sw_group_set_mode how the Ising members are swept (the O(n)
 *                          members always use per-sweep graphs):
 *                          ising_mode PYRO_MODE_GRAPH: one captured graph of
 *                          the sweep's kernels per sweep (the default);
 *                          PYRO_MODE_PERSISTENT: every sweep of a call in one
 *                          persistent fused launch per slice (captured as a
 *                          graph), whose workgroups take (replica, phase,
 *                          tile) items so that the passes of different
 *                          replicas overlap.  resident != 0: Ising members of
 *                          L <= 16 without vacant sites run LDS-resident, one
 *                          workgroup per lattice holding it whole for every
 *                          sweep of a call, beside the slices.  Modes change
 *                          speed only, never results.
 *   pyro_sw_group_get_mode the current modes (either output may be NULL).
 *   pyro_sw_group_autotune also chooses the Ising modes (every combination
 *                          of mode and tile shape that applies is timed).
 *   pyro_sw_group_set_counting  on != 0: the unite pass of the tiled sweeps
 *                          counts its compare-and-swaps on the global forest
 *                          (a measurement mode: one more device atomic per
 *                          swap); the counters start at zero.
 *   pyro_sw_group_counts   synchronises; swaps tried and swaps that hooked a
 *                          root since counting was switched on (0 if never).
 *   pyro_sw_group_set_timing / pyro_sw_group_kernel_times  as for a handle.
 *   pyro_sw_group_destroy  frees the group only (NULL is a no-op).
 * Errors: PYRO_EINVAL (arguments), PYRO_ESTATE (a member failed or is busy),
 * PYRO_ENOMEM, PYRO_EDEVICE (also when a persistent launch gave up a wait:
 * reported by the next pyro_sw_moments of a member, whose device state then
 * disagrees with the host's).
 */
typedef struct pyro_sw_group pyro_sw_group;
enum { PYRO_MODE_GRAPH = 0, PYRO_MODE_PERSISTENT = 1 };
int pyro_sw_group_create(pyro_sw_group **out, pyro_sw *const *members, int n, void *stream);
int pyro_sw_group_sweep(pyro_sw_group *g, int64_t n_sweeps, const int64_t *per_member);
int pyro_sw_group_autotune(pyro_sw_group *g, int trial_sweeps, int *shapes_out);
int pyro_sw_group_set_tile_shape(pyro_sw_group *g, int model, int shape);
int pyro_sw_group_set_slices(pyro_sw_group *g, int nslices);
int pyro_sw_group_set_mode(pyro_sw_group *g, int ising_mode, int resident);
int pyro_sw_group_get_mode(const pyro_sw_group *g, int *ising_mode, int *resident);
int pyro_sw_group_set_counting(pyro_sw_group *g, int on);
int pyro_sw_group_counts(pyro_sw_group *g, int64_t *cas_tried, int64_t *cas_hooked);
int pyro_sw_group_set_timing(pyro_sw_group *g, int kernel_mask);
int pyro_sw_group_kernel_times(pyro_sw_group *g, const char **names, int64_t *launches, double *ms,
                               int cap, int *n_out);
int pyro_sw_group_destroy(pyro_sw_group *g);

/*
 * Serving: a job server for a stream of independent simulation jobs, each
 * the problem the paper states (model n, lattice size L, temperature T in
 * units of J, number of Monte Carlo sweeps; Sec. 2), plus seed and start.
 *
 * The server owns one device allocation of hbm_budget bytes.  A job's
 * footprint is its spin and workspace bytes (pyro_sw_workspace_size,
 * rounded up to 256); jobs are admitted in arrival order while their
 * footprint fits the free budget and fewer than max_running jobs run.  A
 * queued job that does not fit lets later jobs pass until it has waited
 * starve_ms; from then on no job is admitted before it.  Admitted jobs keep
 * spins, sweep index and records resident until they finish.
 *
 * Running jobs are swept in lanes by lattice size (L <= 16, <= 40, <= 72,
 * <= 136, larger): each lane is one group (pyro_sw_group_*) on its own
 * stream, advanced a quantum at a time, the quantum being as many group
 * sweeps as fit in quantum_ms by the lane's measured sweep time (each member
 * runs at most its remaining sweeps).  Lanes overlap on the device.  Jobs
 * join and leave a lane between its quanta, so work that arrives while
 * other jobs run starts as soon as a slot and memory free up (continuous
 * batching).  Every job's records and final spins are identical to a plain
 * pyro_sw_init + pyro_sw_sweep run with the same arguments.
 *
 *   pyro_sw_server_create   hbm_budget >= 1 MiB, max_running >= 1,
 *                           quantum_ms > 0, starve_ms >= 0.
 *   pyro_sw_server_job_bytes  footprint of a job (no device needed).
 *   pyro_sw_server_submit   validates and queues a job (sweeps 1..2^31-1;
 *                           keep_spins != 0 keeps the final spins for
 *                           pyro_sw_server_take); never waits for the device.
 *                           PYRO_ENOMEM if the footprint exceeds the budget.
 *   pyro_sw_server_step     one scheduling round: retire lanes whose quantum
 *                           ended (finished jobs release their memory),
 *                           admit queued jobs, start the next quantum of
 *                           every idle lane.  If nothing changed it waits up
 *                           to wait_ms for a quantum to end and repeats once.
 *                           n_queued / n_running (may be NULL) receive the
 *                           counts after the round.
 *   pyro_sw_server_status   state and times of a job (seconds on the server
 *                           clock, which starts at create; -1 = not yet).
 *   pyro_sw_server_take     records (cap as in pyro_sw_moments; cap = 0
 *                           gives the count only) and, when spins_host is
 *                           not NULL, the final spins (spin_bytes as in
 *                           pyro_sw_get_spins, job created with keep_spins)
 *                           of a finished job; the job is forgotten unless
 *                           cap = 0.  PYRO_ESTATE if the job is not done.
 *   pyro_sw_server_clock    seconds since create.
 *   pyro_sw_server_destroy  synchronises and frees everything (NULL no-op).
 * A server is used from one thread at a time.
 */
typedef struct pyro_sw_server pyro_sw_server;
typedef struct {
    int model;      /* PYRO_ISING, PYRO_XY, PYRO_HEISENBERG */
    int L;          /* 1..406 */
    double T, J;    /* as in pyro_sw_init */
    uint64_t seed;
    int start;      /* PYRO_START_COLD or PYRO_START_RANDOM */
    int keep_spins; /* nonzero: keep the final spins for pyro_sw_server_take */
    int64_t sweeps; /* 1 .. 2^31 - 1 */
} pyro_sw_job;
enum { PYRO_JOB_QUEUED = 0, PYRO_JOB_RUNNING = 1, PYRO_JOB_DONE = 2 };
typedef struct {
    int64_t id;
    int state;          /* PYRO_JOB_* */
    int lane;           /* -1 while queued */
    int64_t sweeps_done;
    int64_t footprint;  /* bytes */
    int error;          /* status of a job that failed on the device, else 0 */
    int reserved;
    double t_submit, t_admit, t_done;
} pyro_sw_job_status;
int pyro_sw_server_create(pyro_sw_server **out, size_t hbm_budget, int max_running, double quantum_ms,
                          double starve_ms);
int pyro_sw_server_job_bytes(const pyro_sw_job *job, size_t *bytes);
int pyro_sw_server_submit(pyro_sw_server *s, const pyro_sw_job *job, int64_t *id);
int pyro_sw_server_step(pyro_sw_server *s, double wait_ms, int *n_queued, int *n_running);
int pyro_sw_server_status(pyro_sw_server *s, int64_t id, pyro_sw_job_status *out);
int pyro_sw_server_take(pyro_sw_server *s, int64_t id, pyro_sw_record *out, int64_t cap, int64_t *n_out,
                        void *spins_host, size_t spin_bytes);
int pyro_sw_server_clock(pyro_sw_server *s, double *seconds);
int pyro_sw_server_destroy(pyro_sw_server *s);

/*
 * Measurement helper, not part of a sweep: throughput on the current device
 * of the Philox4x32-10 generator that every random draw of a sweep uses
 * (counter, key and rounds as in pyro_sw_init).  Draws `calls` blocks with
 * counters (i, 0x5EED, BOND stream, 0) for i = 0 .. calls-1 and key = seed,
 * spread over the whole GPU, and XOR-folds all their output words so that no
 * block is skipped; the launch is timed `repeats` times with HIP events.
 *   calls_per_second  blocks per second of the fastest launch (out)
 *   fold              XOR of every output word of every block (out), for a
 *                     check against a host implementation
 * Synchronous; allocates and frees a 4-byte device buffer and a stream.
 * EINVAL for calls outside [1, 2^32], repeats < 1 or NULL outputs.
 */
int pyro_sw_philox_rate(int64_t calls, int repeats, uint64_t seed, double *calls_per_second, uint32_t *fold);

/*
 * Measurement helper, not part of a sweep: device atomic throughput on the
 * current device, the ceiling of the global merge (a hook is a load and a
 * compare-and-swap of a label entry) and of work counters.
 *   mode 0   `ops` operations, each a load and a compare-and-swap from the
 *            loaded value v to v + 1 of a pseudo-random word of a zeroed
 *            array of `words` 32-bit words (a label array has one per site)
 *   mode 1   `ops` atomic adds of 1 to one word
 *   ops_per_second  operations per second of the fastest of `repeats`
 *                   launches (HIP events around the launch)
 *   succeeded  swaps that took effect (mode 0; ops in mode 1), and
 *   word_sum   the sum of the array after the last launch: equal to
 *              succeeded when no update was lost
 * Synchronous; allocates and frees the array, two counters and a stream.
 * EINVAL for a mode other than 0 or 1, words outside [1, 2^32], ops outside
 * [1, 2^40], repeats < 1 or NULL outputs.
 */
int pyro_sw_atomic_rate(int mode, int64_t words, int64_t ops, int repeats, double *ops_per_second,
                        int64_t *succeeded, int64_t *word_sum);

/*
 * Generic lattices: the same Swendsen-Wang sweep on any graph supplied as a
 * nearest-neighbour (bond) table, the generality the paper claims for its
 * algorithm (Sec. 2 and Sec. 4).  Bond b joins sites bond_a[b] and
 * bond_b[b]; its random draws are keyed by b and the sweep index exactly as
 * bond b of the pyrochlore sweep, and flip coins by the cluster's smallest
 * site, so the pyrochlore table of pyro_sw_bonds reproduces that sweep's
 * trajectory bit for bit.  No tiles: one thread per bond or site, with the
 * global union-find of the pyrochlore sweep; slower, for any lattice.
 *   pyro_sw_graph_init     n_sites in [1, 2^31 - 1], n_bonds in [0, 2^32 - 1];
 *                          ends in range and distinct (EINVAL otherwise);
 *                          host arrays are copied, the caller keeps them;
 *                          model, T, J, seed, start and stream as in
 *                          pyro_sw_init.  One device allocation: 12 B per
 *                          bond (ends and table position) and 4 B more per
 *                          bond inside a 4096-site window, spins, 4 B per
 *                          site of labels (O(n): 4 more of projections; 4
 *                          more for the window site lists when the windows
 *                          are breadth-first balls), partials, a record
 *                          ring.  The windows are chosen on the host at
 *                          set-up (a breadth-first pass over the table,
 *                          about 8 B per bond and 16 B per site of host
 *                          memory while it runs); they never change a
 *                          result.
 *   pyro_sw_graph_sweep    enqueue n_sweeps sweeps (records drained to the
 *                          host every 1024 sweeps).
 *   pyro_sw_graph_moments, _get_spins, _set_spins, _get_labels,
 *   _set_temperature, _destroy   as for a pyrochlore handle (spin layouts
 *                          int8 [N] or float [n][N]; a zero spin is a vacant
 *                          site; labels are the smallest site index of each
 *                          site's cluster after the last sweep).
 * pyro_sw_bonds writes the pyrochlore bond table of edge L (n = 48 L^3
 * entries per array, bond 48 cell + 6 t + e as in the site numbering above)
 * into host arrays.
 * pyro_sw_sc_bonds writes the periodic simple-cubic table of edge L, the
 * comparison lattice of Sec. 3.4 (coordination 6 like the pyrochlore):
 * site (z L + y) L + x, bond 3 i + d joins site i to its +x, +y, +z
 * neighbour for d = 0, 1, 2 (n = 3 L^3 entries per array; L in [1, 1290],
 * EINVAL otherwise or for a wrong n or NULL arrays).  Host code, no device.
 */
typedef struct pyro_sw_graph pyro_sw_graph;
int pyro_sw_graph_init(pyro_sw_graph **out, int64_t n_sites, int64_t n_bonds, const int32_t *bond_a,
                       const int32_t *bond_b, int model, double T, double J, uint64_t seed, int start, void *stream);
int pyro_sw_graph_sweep(pyro_sw_graph *g, int64_t n_sweeps);
int pyro_sw_graph_moments(pyro_sw_graph *g, pyro_sw_record *out, int64_t cap, int64_t *n_out);
int pyro_sw_graph_get_spins(pyro_sw_graph *g, void *host, size_t bytes);
int pyro_sw_graph_set_spins(pyro_sw_graph *g, const void *host, size_t bytes, int64_t next_sweep);
int pyro_sw_graph_get_labels(pyro_sw_graph *g, int32_t *host, size_t n);
int pyro_sw_graph_set_temperature(pyro_sw_graph *g, double T);
int pyro_sw_graph_destroy(pyro_sw_graph *g);
int pyro_sw_bonds(int L, int32_t *bond_a, int32_t *bond_b, int64_t n);
int pyro_sw_sc_bonds(int L, int32_t *bond_a, int32_t *bond_b, int64_t n);

/*
 * For callers that cannot allocate: code under HIP graph capture, serving
 * loops and harnesses that forbid device allocation.  Runs n_sweeps sweeps
 * of one lattice whose spins the caller holds in device memory, as a handle
 * made by pyro_sw_init_ext, given these spins by pyro_sw_set_spins with
 * next_sweep = first_sweep, would run them with pyro_sw_sweep (same kernels,
 * same tile shape, bit-identical results), and writes its records to the
 * caller's device buffer.  No handle: nothing persists between calls.
 *   dev_spins    device memory, int8 [N] (+1/-1; vacant sites are not
 *                supported here) or float [n][N]; read and overwritten in
 *                place; 16-byte aligned
 *   L, model, T, J, seed   as in pyro_sw_init
 *   first_sweep  global index of the first sweep (keys the random draws)
 *   n_sweeps     in [0, 2^31 - 1]; first_sweep + n_sweeps < 2^32
 *   dev_records  device memory for n_sweeps records of type pyro_sw_record,
 *                80 B each, 8-byte aligned: record k describes the state after sweep
 *                first_sweep + k
 *   stream       HIP stream (NULL = the default stream); the call only
 *                enqueues work and returns
 * Workspace: a static device array of 64 MiB per device (labels, crossing
 * lists, coins, partial sums), held until the process ends, which bounds L
 * at 80 for every model (EINVAL beyond).  The call allocates nothing: no
 * hipMalloc, hipFree, stream, event or graph; its first call on a device
 * looks the array's address up.  Every call on a device shares that array,
 * so calls whose work overlaps on one device race: serialise them (one
 * stream, or synchronise between calls).  EINVAL for bad arguments as in
 * pyro_sw_init, NULL or misaligned buffers, or a lattice beyond the limit;
 * EDEVICE if a launch fails.
 */
int pyro_sw_sweep_static(void *dev_spins, int L, int model, double T, double J, uint64_t seed, int64_t first_sweep,
                         int64_t n_sweeps, pyro_sw_record *dev_records, void *stream);

/* Synchronise and free everything the library allocated.  NULL is a no-op. */
int pyro_sw_destroy(pyro_sw *h);

/* Static text for a status code. */
const char *pyro_sw_strerror(int status);

/* Detail of the last error on the calling thread ("" if none). */
const char *pyro_sw_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PYRO_SW_H */
