#!/usr/bin/env python3
"""Throughput benchmark of the HIP Swendsen-Wang sweep on one MI355X.

Workload: Ising model on the periodic pyrochlore lattice, L = 128
(33,554,432 sites, 100,663,296 bonds), int8 spins and int32 labels, five
lattices resident at T = 4.205, 4.210, 4.2139, 4.218, 4.223 (seeds 1..5,
random start).  One step = one Swendsen-Wang sweep of each of the five
lattices (bond activation, cluster labeling, cluster flips, moments);
--steps 10000 --warmup 0 is the full five-temperature run (sweeps 1..10^4
from the random start, Binder U per temperature over sweeps 5001..10^4 and
over all sweeps).

Printed on one JSON line: spin-updates/s over the timed steps, the roofline
of the dominant kernel (algorithmic bytes per launch / its mean duration,
timed with HIP events on the stream it runs on), and the CPU oracle timed on
a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SW spin-updates/sec and % HBM roofline, Ising L=128; batched vs plain, p99 job latency"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s

# Algorithmic HBM bytes per site of one launch of each Ising kernel: every
# array element the kernel must touch, read or written once (halo re-reads,
# forest walks and L2/MALL hits not counted).  The crossing lists the local
# kernel writes and the forest passes read are data dependent and small
# (at most 3 pairs per down tetrahedron of a tile's low-face cells); they
# are not counted.


def bytes_per_site(shape):
    del shape  # the counted traffic does not depend on the tile shape
    return {
        "local": 1.0 + 4.0,            # read spins, write tile-local roots
        "unite": 0.0,                  # forest walks over the crossing lists (data dependent)
        "flip": 4.0 + 1.0 + 1.0,       # read labels, read and write spins (the settle step's walks and stores,
                                       # data dependent, and the coins drawn in the kernel are not counted)
        "persist": 11.0,               # the whole sweep (every pass), per sweep of each lattice
        "energy": 1.0,                 # read spins
        "finalize": 0.0,
    }


# Per-launch counter figures of the Ising kernels (one L=128 lattice, 8x8x8
# tiles) from rocprofv3 --pmc runs of `bench.py --pmc-probe`: HBM bytes
# (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter's reading for
# the probe's 256 MiB copy) and wave instructions (SQ_INSTS_VALU,
# SQ_INSTS_SALU, SQ_WAVES).  Valid only for the kernel sources they were
# taken with (fingerprint); the summaries are in profiles/.
COUNTER_FINGERPRINT = "bce8deb94f4062c8"
MEASURED_TRAFFIC = {  # kernel -> HBM bytes per launch
    "local": 216857639,
    "unite": 194594163,
    "flip": 269545072,
    "finalize": 73136,
}
MEASURED_ISSUE = {  # kernel -> (VALU wave instructions, SALU wave instructions, waves) per launch
    "local": (62134795, 28267641, 32768),
    "unite": (11532870, 12803987, 16384),
    "flip": (24889449, 10496674, 32768),
}

# Issue ceiling of the vector ALUs: a wave64 VALU instruction occupies a
# 16-lane SIMD for 4 cycles, so each of the 256 CUs (4 SIMDs) completes at
# most one wave instruction per cycle: 256 x 2.4 GHz.
VALU_ISSUE_PEAK = 256 * 2.4e9


def _code_tokens(text):
    """Source text without comments, whitespace runs collapsed (string and
    character literals kept as written)."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_fingerprint():
    """SHA-256 over the HIP sources of the library (names and code, comments
    and whitespace left out, so that a comment edit keeps the counters)."""
    import hashlib

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1612_08312_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".hpp")):
            h.update(name.encode())
            with open(os.path.join(csrc, name), encoding="utf-8") as f:
                h.update(_code_tokens(f.read()).encode())
    return h.hexdigest()[:16]


def pmc_probe():
    """Workload for counter collection: a 256 MiB device copy (calibration),
    then 4 sweeps of the bench's first L=128 lattice with every kernel
    launched directly (no graph) after 30 graph sweeps."""
    import torch

    from paper_1612_08312_amd import pyrosw, workloads

    torch.cuda.set_device(0)
    a = torch.ones(1 << 26, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    cfg = workloads.ISING_L128
    lt = pyrosw.Lattice(L=128, model=1, T=cfg["temps"][2], seed=cfg["seeds"][2], start=cfg["start"])
    lt.sweep(30)
    lt.moments()
    pyrosw.pyro_sw_set_timing(lt.h, -1)
    lt.sweep(4)
    pyrosw.pyro_sw_kernel_times(lt.h)
    lt.close()
    log("pmc probe done, kernel fingerprint", kernel_fingerprint())


SWEEP_BYTES_PER_SITE = 11.0  # whole-sweep model: read s, write/read labels, read/write s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(L, T, seed, sweeps):
    """Time the CPU oracle (single thread) on `sweeps` sweeps of one L
    lattice at temperature T; lattice construction is not timed."""
    import oracle

    o = oracle.Oracle(L=L, model=oracle.ISING, T=T, seed=seed, start=oracle.RANDOM)
    t0 = time.perf_counter()
    o.sweep(sweeps)
    dt = time.perf_counter() - t0
    return dict(value=o.N * sweeps / dt, unit="spin-updates/s", cores=1, kind="oracle",
                sample=f"{sweeps} sweeps of one Ising L={L} lattice at T={T} (N={o.N}), "
                       f"random start, single-threaded C oracle, lattice build not timed",
                host=cpu_model(), host_threads=os.cpu_count())


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def copy_peak_gbs(dev, mib=1024, reps=5):
    """Achievable HBM bandwidth: best of `reps` device-to-device copies of
    `mib` MiB (bytes read plus bytes written over the copy's duration)."""
    import torch

    a = torch.ones(mib << 18, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(reps):
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    return 2 * (mib << 20) / (best * 1e-3) / 1e9


def batch_modes(sweeps, stream, dev):
    """The 96-replica batch under each Ising mode of a group (per-sweep
    graphs; persistent fused launch; each with and without LDS-resident
    small lattices), autotuned tile shape: spin-updates/s of each, `sweeps`
    sweeps after 5 warm-up sweeps."""
    import torch

    from paper_1612_08312_amd import pyrosw, workloads

    specs = workloads.batch_replicas()
    lats = [pyrosw.Lattice(L=r["L"], model=r["model"], T=r["T"], J=r["J"], seed=r["seed"], start=r["start"],
                           device=dev, stream=stream) for r in specs]
    sites = sum(lt.N for lt in lats)
    group = pyrosw.Group(lats, stream)
    shape = group.autotune(trial_sweeps=3)[0]
    out = {"tile_shape": pyrosw.TILE_SHAPES[shape]}
    for name, mode, res in (("graph", pyrosw.PYRO_MODE_GRAPH, False), ("graph_resident", pyrosw.PYRO_MODE_GRAPH, True),
                            ("persistent", pyrosw.PYRO_MODE_PERSISTENT, False),
                            ("persistent_resident", pyrosw.PYRO_MODE_PERSISTENT, True)):
        group.set_mode(mode, res)
        group.sweep(5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        group.sweep(sweeps)
        torch.cuda.synchronize()
        out[name] = sites * sweeps / (time.perf_counter() - t0)
        for lt in lats:
            lt.moments()
    group.close()
    for lt in lats:
        lt.close()
    return out


def batched_vs_plain(sweeps, stream, dev):
    """The 96-replica batch (L in {8,12,16,24,32,48} x 16 temperatures in
    [4.19, 4.24]) swept `sweeps` times as one group (one captured graph per
    sweep, autotuned tile shape), then the same replicas one at a time, each
    from its own captured graph on the same stream.  Records must agree
    bit for bit."""
    import numpy as np
    import torch

    from paper_1612_08312_amd import pyrosw, workloads

    specs = workloads.batch_replicas()

    def build():
        return [pyrosw.Lattice(L=r["L"], model=r["model"], T=r["T"], J=r["J"], seed=r["seed"],
                               start=r["start"], device=dev, stream=stream) for r in specs]

    lats = build()
    sites = sum(lt.N for lt in lats)
    group = pyrosw.Group(lats, stream)
    shape = pyrosw.TILE_SHAPES[group.autotune(trial_sweeps=3)[0]]
    mode, resident = group.mode()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    group.sweep(sweeps)
    torch.cuda.synchronize()
    t_batched = time.perf_counter() - t0
    rec_b = [lt.moments() for lt in lats]
    group.close()
    for lt in lats:
        lt.close()

    lats = build()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for lt in lats:
        lt.sweep(sweeps)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    rec_p = [lt.moments() for lt in lats]
    for lt in lats:
        lt.close()
    identical = all(np.array_equal(a, b) for a, b in zip(rec_b, rec_p)) and all(len(a) == sweeps for a in rec_b)
    return {
        "workload": "ising_batch_96_replicas",
        "replicas": len(specs),
        "sites_per_sweep": sites,
        "sweeps": sweeps,
        "tile_shape": shape,
        "ising_mode": "persistent" if mode == pyrosw.PYRO_MODE_PERSISTENT else "graph",
        "lds_resident_small_lattices": bool(resident),
        "batched_spin_updates_per_s": sites * sweeps / t_batched,
        "plain_spin_updates_per_s": sites * sweeps / t_plain,
        "speedup": t_plain / t_batched,
        "records_identical": bool(identical),
    }


def serving_vs_plain(n_jobs, budget_gb, quantum_ms, dev):
    """The first `n_jobs` jobs of the Poisson serving stream (20 jobs/s;
    models, sizes, temperatures and sweep counts as drawn by
    workloads.serving_jobs, including one Ising L=256 job) through the job
    server, then the same jobs run plain, one at a time in arrival order.
    Plain latencies replay the measured plain durations through a FIFO queue
    with the same arrival times."""
    import numpy as np
    import torch

    from paper_1612_08312_amd import pyrosw, serving, workloads

    jobs = workloads.serving_jobs(n_jobs=n_jobs)
    srv = pyrosw.Server(hbm_budget=int(budget_gb * (1 << 30)), max_running=64, quantum_ms=quantum_ms)
    results, summary = serving.run_stream(srv, jobs)
    srv.close()
    log(f"bench: served {len(jobs)} jobs in {summary['makespan_s']:.1f} s; running them plain")

    durations, identical, mismatches = [], True, []
    for idx, r in enumerate(results):
        if idx and idx % 25 == 0:
            log(f"bench: {idx} plain jobs done")
        j = r["job"]
        lt = pyrosw.Lattice(L=j["L"], model=j["model"], T=j["T"], J=j["J"], seed=j["seed"], start=j["start"],
                            device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lt.sweep(j["sweeps"])
        torch.cuda.synchronize()
        durations.append(time.perf_counter() - t0)
        rec = lt.moments()
        lt.close()
        a, b = r["records"], rec
        same = len(a) == len(b)
        if same:
            for f in ("sweep", "bond_sum", "M_int", "E", "m2", "m4"):
                exact = f in ("sweep", "bond_sum", "M_int") or j["model"] == 1
                ok = np.array_equal(a[f], b[f]) if exact else np.allclose(a[f], b[f], rtol=1e-12, atol=1e-12)
                if not ok:
                    bad = np.nonzero(a[f] != b[f])[0]
                    mismatches.append(dict(job=j["job_id"], model=j["model"], L=j["L"], field=f,
                                           first_sweep=int(bad[0]) if len(bad) else -1, n_bad=int(len(bad))))
                same &= bool(ok)
        else:
            mismatches.append(dict(job=j["job_id"], lengths=[len(a), len(b)]))
        if not same:  # which side moves: run the job plain once more
            lt = pyrosw.Lattice(L=j["L"], model=j["model"], T=j["T"], J=j["J"], seed=j["seed"],
                                start=j["start"], device=dev)
            lt.sweep(j["sweeps"])
            again = lt.moments()
            lt.close()
            mismatches[-1]["plain_repeat_equal"] = bool(
                len(again) == len(b) and all(np.array_equal(again[f], b[f]) for f in ("bond_sum", "M_int", "E")))
        identical &= bool(same)
    t_free, lat = 0.0, []
    for j, d in sorted(zip(jobs, durations), key=lambda p: p[0]["arrival"]):
        start = max(j["arrival"], t_free)
        t_free = start + d
        lat.append(t_free - j["arrival"])
    updates = summary["spin_updates"]
    return {
        "workload": "poisson_20_jobs_per_s_mixed_models",
        "jobs": len(jobs),
        "models": {m: sum(1 for j in jobs if j["model"] == m) for m in (1, 2, 3)},
        "largest_L": max(j["L"] for j in jobs),
        "spin_updates": updates,
        "hbm_budget_gb": budget_gb,
        "quantum_ms": quantum_ms,
        "served_p50_latency_s": summary["p50_latency_s"],
        "served_p99_latency_s": summary["p99_latency_s"],
        "served_spin_updates_per_s": summary["spin_updates_per_s"],
        "served_makespan_s": summary["makespan_s"],
        "plain_p50_latency_s": serving.percentile_nearest_rank(lat, 50),
        "plain_p99_latency_s": serving.percentile_nearest_rank(lat, 99),
        "plain_spin_updates_per_s": updates / sum(durations),
        "plain_makespan_s": t_free,
        "records_identical": bool(identical),
        "mismatches": mismatches[:20],
    }


def on_throughput(sweeps, stream, dev):
    """XY (T = 2.0285) and Heisenberg (T = 1.31695) on the L = 64 pyrochlore
    lattice (4,194,304 sites each, random start, FP32 spins, FP64 moments):
    spin-updates/s of each, one lattice at a time, after 20 warm-up sweeps."""
    import torch

    from paper_1612_08312_amd import pyrosw, workloads

    out = {}
    for cfg in workloads.ON_L64:
        name = "xy" if cfg["model"] == 2 else "heisenberg"
        lt = pyrosw.Lattice(L=cfg["L"], model=cfg["model"], T=cfg["T"], J=cfg["J"], seed=cfg["seed"],
                            start=cfg["start"], device=dev, stream=stream)
        lt.sweep(20)
        lt.moments()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lt.sweep(sweeps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rec = lt.moments()
        lt.close()
        out[name] = {"T": cfg["T"], "spin_updates_per_s": lt.N * sweeps / dt, "us_per_sweep": dt / sweeps * 1e6,
                     "mean_m2": float(rec["m2"].mean())}
    out.update(workload="on_pyrochlore_L64", L=64, sweeps=sweeps)
    return out


def diluted_throughput(sweeps, stream, dev):
    """Site-diluted Ising lattice (L = 128, 10% vacant sites, T = 3.8) against
    the pure lattice at the same temperature: spin-updates/s of each (all N
    sites counted), one lattice at a time, after 20 warm-up sweeps."""
    import torch

    from paper_1612_08312_amd import pyrosw, workloads

    c = workloads.DILUTED_ISING_L128
    N = workloads.n_sites(c["L"])
    out = {}
    for name, vac in (("diluted", c["vacancy"]), ("pure", 0.0)):
        lt = pyrosw.Lattice(L=c["L"], model=c["model"], T=c["T"], J=c["J"], seed=c["seed"],
                            start=pyrosw.PYRO_START_COLD, device=dev, stream=stream)
        lt.set_spins(workloads.diluted_spins(N, c["model"], vac, c["seed"]), 0)
        lt.sweep(20)
        lt.moments()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lt.sweep(sweeps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rec = lt.moments()
        lt.close()
        out[name] = {"vacancy": vac, "spin_updates_per_s": N * sweeps / dt, "us_per_sweep": dt / sweeps * 1e6,
                     "mean_m2": float(rec["m2"].mean())}
    out.update(workload="ising_pyrochlore_L128_site_diluted", L=c["L"], T=c["T"], sweeps=sweeps)
    return out


def graph_throughput(sweeps, stream, dev):
    """The generic graph path (any bond table): simple-cubic Ising L = 256 at
    its T_c, the pyrochlore L = 128 table at T = 4.2139 for comparison with
    the tiled sweep, and XY on the simple-cubic L = 128 table at its T_c;
    spin-updates/s after 10 warm-up sweeps."""
    import torch

    from paper_1612_08312_amd import pyrosw, workloads

    sc = workloads.SC_ISING_L256
    cases = (("simple_cubic_L256", pyrosw.simple_cubic_bonds(sc["L"]), sc["L"] ** 3, 1, sc["T"], sc["seed"]),
             ("pyrochlore_L128", pyrosw.pyro_sw_bonds(128), 16 * 128 ** 3, 1, 4.2139, 3),
             ("xy_simple_cubic_L128", pyrosw.simple_cubic_bonds(128), 128 ** 3, 2, 2.20182, 4))
    out = {}
    for name, bonds, n, model, T, seed in cases:
        g = pyrosw.Graph(bonds, n, model, T, seed=seed, device=dev, stream=stream)
        g.sweep(10)
        g.moments()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.sweep(sweeps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rec = g.moments()
        g.close()
        out[name] = {"model": model, "sites": n, "bonds": len(bonds[0]), "T": T, "spin_updates_per_s": n * sweeps / dt,
                     "us_per_sweep": dt / sweeps * 1e6, "mean_m2": float(rec["m2"].mean())}
    out.update(workload="ising_graph_path", sweeps=sweeps)
    return out


def kernel_bounds(kt, N, cas_per_launch, hooks_per_launch, cas_ceiling, copy_gbs, counters_valid):
    """Each Ising pass of one L=128 lattice (per-sweep launches, mean over the
    probe): its duration, what bounds it, and the fraction of that bound it
    reaches.  The tile pass is bound by VALU issue (wave instructions per
    launch from the counters / duration, against one wave instruction per CU
    and cycle); the settle-and-flip pass by HBM streaming (counter bytes /
    duration, against 8 TB/s and the measured copy bandwidth: its 6 B/site
    of labels and spins plus the settle step's walks) and by the latency of
    its settle walks; the
    unite pass by device atomics
    (compare-and-swaps per launch / duration, against the measured random
    compare-and-swap rate); the finalize by launch latency (one workgroup
    per lattice).  There is no store pass: each tile settles its own hooked
    roots at the start of its flip."""
    out = {}
    for k, (n, ms) in kt.items():
        if not n:
            continue
        us = ms / n * 1e3
        row = {"us": round(us, 2)}
        if k == "local":
            row["bound"] = "VALU issue"
            if counters_valid and k in MEASURED_ISSUE:
                valu, salu, waves = MEASURED_ISSUE[k]
                row.update(valu_per_wave=round(valu / waves), salu_per_wave=round(salu / waves),
                           achieved_wave_instr_per_s=valu / (us * 1e-6), peak_wave_instr_per_s=VALU_ISSUE_PEAK,
                           frac=valu / (us * 1e-6) / VALU_ISSUE_PEAK)
            row["hbm_alg_frac"] = 5.0 * N / (us * 1e-6) / (HBM_PEAK_GBS * 1e9)
        elif k == "unite":
            row.update(bound="device atomics", cas_per_launch=round(cas_per_launch),
                       hooks_per_launch=round(hooks_per_launch), achieved_cas_per_s=cas_per_launch / (us * 1e-6),
                       peak_cas_per_s=cas_ceiling, frac=cas_per_launch / (us * 1e-6) / cas_ceiling)
        elif k == "flip":
            row["bound"] = "HBM streaming (labels and spins) and the settle step's walk latency"
            row.update(alg_bytes_per_site=6.0, hbm_alg_frac=6.0 * N / (us * 1e-6) / (HBM_PEAK_GBS * 1e9))
            if counters_valid and k in MEASURED_TRAFFIC:
                gbs = MEASURED_TRAFFIC[k] / (us * 1e-6) / 1e9
                row.update(achieved_GBps=gbs, peak_GBps=HBM_PEAK_GBS, frac=gbs / HBM_PEAK_GBS,
                           frac_of_copy=gbs / copy_gbs)
            if counters_valid and k in MEASURED_ISSUE:
                valu, salu, waves = MEASURED_ISSUE[k]
                row.update(valu_per_wave=round(valu / waves), salu_per_wave=round(salu / waves),
                           valu_issue_frac=valu / (us * 1e-6) / VALU_ISSUE_PEAK)
        elif k == "finalize":
            row["bound"] = "launch latency (one workgroup per lattice)"
        if counters_valid and k in MEASURED_TRAFFIC:
            row["counter_bytes_per_launch"] = MEASURED_TRAFFIC[k]
        out[k] = row
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--L", type=int, default=128)
    ap.add_argument("--cpu-sweeps", type=int, default=4, help="oracle sweeps for cpu_baseline (0: skip)")
    ap.add_argument("--tile-shape", type=int, default=-1, help="tile shape id (-1: autotune)")
    ap.add_argument("--slices", type=int, default=0,
                    help="concurrent slices of the five-lattice group (0: the group's default, one per lattice)")
    ap.add_argument("--cas-count-sweeps", type=int, default=4,
                    help="sweeps of the unite-pass counting run (0: skip; it adds one atomic per swap)")
    ap.add_argument("--ising-mode", choices=("auto", "graph", "persistent"), default="auto",
                    help="Ising sweep mode of the group (auto: the autotuner's choice)")
    ap.add_argument("--batch-sweeps", type=int, default=2000,
                    help="sweeps of the 96-replica batched-vs-plain comparison (0: skip)")
    ap.add_argument("--serve-jobs", type=int, default=100,
                    help="jobs of the Poisson serving stream for the served-vs-plain comparison (0: skip)")
    ap.add_argument("--serve-budget-gb", type=float, default=64.0, help="HBM budget of the job server")
    ap.add_argument("--serve-quantum-ms", type=float, default=20.0, help="lane quantum of the job server")
    ap.add_argument("--on-sweeps", type=int, default=500, help="sweeps of the XY and Heisenberg L=64 leg (0: skip)")
    ap.add_argument("--graph-sweeps", type=int, default=200,
                    help="sweeps of the generic graph-path leg (simple cubic L=256, pyrochlore L=128; 0: skip)")
    ap.add_argument("--diluted-sweeps", type=int, default=500,
                    help="sweeps of the site-diluted Ising L=128 leg and its pure twin (0: skip)")
    ap.add_argument("--batch-modes-sweeps", type=int, default=0,
                    help="sweeps of the 96-replica batch timed under each Ising mode (0: skip)")
    ap.add_argument("--pmc-probe", action="store_true", help="run the counter-collection workload and exit")
    ap.add_argument("--roofline-steps", type=int, default=200,
                    help="steps of the pass that times the dominant kernel with HIP events")
    args = ap.parse_args()

    if args.pmc_probe:
        pmc_probe()
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(independent lattices would shard by replica, one lattice as slabs along z)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1612_08312_amd import pyrosw, workloads

    cfg = workloads.ISING_L128
    L = args.L
    temps, seeds = cfg["temps"], cfg["seeds"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    log(f"bench: building {len(temps)} Ising L={L} lattices")
    lats = [pyrosw.Lattice(L=L, model=1, T=T, seed=s, start=cfg["start"], device=dev, stream=stream)
            for T, s in zip(temps, seeds)]
    N = lats[0].N
    group = pyrosw.Group(lats, stream)
    if args.slices > 0:
        group.set_slices(args.slices)
    if args.tile_shape >= 0 or args.ising_mode != "auto":
        tshape = args.tile_shape if args.tile_shape >= 0 else pyrosw.PYRO_TILE_8x8x8
        group.set_tile_shape(1, tshape)
        shape = pyrosw.TILE_SHAPES[tshape]
        if args.ising_mode != "auto":
            group.set_mode(pyrosw.PYRO_MODE_PERSISTENT if args.ising_mode == "persistent" else pyrosw.PYRO_MODE_GRAPH)
    else:
        shapes = group.autotune(trial_sweeps=3)
        shape = pyrosw.TILE_SHAPES[shapes[0]]
        log("bench: autotuned tile shape", shape)
    ising_mode = "persistent" if group.mode()[0] == pyrosw.PYRO_MODE_PERSISTENT else "graph"
    log("bench: Ising mode", ising_mode)
    byte_model = bytes_per_site(shape)

    # Warmup, then the timed region.
    group.sweep(args.warmup)
    for lt in lats:
        lt.moments()  # discard warmup records
    torch.cuda.synchronize()
    log(f"bench: timing {args.steps} steps")
    t0 = time.perf_counter()
    group.sweep(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    recs = [lt.moments() for lt in lats]
    # Per-pass breakdown (HIP events on every kernel of per-sweep launches,
    # ten sweeps), then the dominant kernel of the timed mode: the
    # persistent launch itself, or the slowest pass.
    saved_mode = group.mode()
    group.set_mode(pyrosw.PYRO_MODE_GRAPH, saved_mode[1])
    pyrosw.pyro_sw_group_set_timing(group.g, -1)
    group.sweep(10)
    kt = {k: list(v) for k, v in pyrosw.pyro_sw_group_kernel_times(group.g).items()}
    pyrosw.pyro_sw_group_set_timing(group.g, 0)
    group.set_mode(*saved_mode)
    names = list(kt)
    dominant = "persist" if ising_mode == "persistent" else max(kt, key=lambda k: kt[k][1])
    log("bench: mean us per launch over probe sweeps:",
        {k: round(v[1] / v[0] * 1e3, 1) for k, v in kt.items() if v[0]})
    # Mean duration of the dominant kernel: HIP events around each of its
    # launches on the group's stream (direct launches instead of the graph).
    roof_steps = max(1, min(args.steps, args.roofline_steps))
    pyrosw.pyro_sw_group_set_timing(group.g, 1 << names.index(dominant))
    group.sweep(roof_steps)
    dom_n, dom_ms = pyrosw.pyro_sw_group_kernel_times(group.g)[dominant]
    pyrosw.pyro_sw_group_set_timing(group.g, 0)

    # Compare-and-swaps of the unite pass per launch (a counting run of
    # per-sweep launches: one more atomic per swap, so it is not timed) and
    # the device's random compare-and-swap ceiling on a label-sized array.
    count_sweeps = args.cas_count_sweeps
    cas_tried = cas_hooked = 0
    if count_sweeps > 0:
        group.set_mode(pyrosw.PYRO_MODE_GRAPH, saved_mode[1])
        pyrosw.pyro_sw_group_set_counting(group.g, True)
        group.sweep(count_sweeps)
        cas_tried, cas_hooked = pyrosw.pyro_sw_group_counts(group.g)
        pyrosw.pyro_sw_group_set_counting(group.g, False)
        group.set_mode(*saved_mode)
        for lt in lats:
            lt.moments()
    cas_ceiling, cas_ok, cas_sum = pyrosw.pyro_sw_atomic_rate(0, N, 1 << 26, 3)
    group.close()
    for lt in lats:
        lt.close()

    # Outside the timed region: the achievable copy bandwidth and the Philox
    # throughput (the ALU side of the tile pass: 3 blocks per cell and sweep,
    # plus a rare fourth for near-threshold bonds).
    copy_gbs = copy_peak_gbs(dev)
    philox_rate, philox_fold = pyrosw.pyro_sw_philox_rate(1 << 28, 3, 1)
    philox_blocks = 3 * (N // 16)

    updates = N * len(lats) * args.steps
    value = updates / dt
    dom_avg_s = dom_ms / max(dom_n, 1) / 1e3
    # a group runs its lattices in concurrent slices, one launch per kernel
    # and slice: the launches of one step together cover every lattice once
    launches_per_step = max(dom_n, 1) / roof_steps
    bytes_per_launch = byte_model.get(dominant, 0.0) * N * len(lats) / launches_per_step
    achieved = bytes_per_launch / dom_avg_s / 1e9 if dom_avg_s > 0 else 0.0
    counters_valid = COUNTER_FINGERPRINT == kernel_fingerprint()
    traffic = MEASURED_TRAFFIC.get(dominant) if counters_valid and launches_per_step == len(lats) else None
    binder, binder_all = {}, {}
    for T, r in zip(temps, recs):
        half = r[len(r) // 2:]
        if len(half):
            binder[str(T)] = float(np.mean(half["m4"]) / np.mean(half["m2"]) ** 2)
            binder_all[str(T)] = float(np.mean(r["m4"]) / np.mean(r["m2"]) ** 2)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "spin-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8",
        "data": "synthetic",
        "config": {
            "workload": f"ising_pyrochlore_L{L}_5T",
            "L": L,
            "sites_per_lattice": N,
            "lattices": len(lats),
            "temperatures": list(temps),
            "seeds": list(seeds),
            "start": "random",
            "sweeps_per_lattice": args.steps,
            "step": ("one SW sweep of each lattice (every sweep of the timed call in one persistent launch)"
                     if ising_mode == "persistent" else
                     "one SW sweep of each lattice (one captured graph per lattice and sweep, run concurrently)"),
            "tile_shape": shape,
            "ising_mode": ising_mode,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dominant,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "alg_bytes_per_site": byte_model.get(dominant, 0.0),
            "mean_launch_us": dom_avg_s * 1e6,
            "timed_launches": dom_n,
            "launches_per_step": launches_per_step,
            "copy_GBps": copy_gbs,
            "frac_of_copy": achieved / copy_gbs,
            "limiter": ("the whole sweep in one launch: see kernels" if dominant == "persist" else
                        "VALU issue and LDS-walk latency, not HBM bandwidth: see kernels.local"),
        },
        "philox": {
            "blocks_per_s": philox_rate,
            "blocks_per_lattice_sweep": philox_blocks,
            "us_per_lattice_sweep": philox_blocks / philox_rate * 1e6,
            "share_of_step": philox_blocks * len(lats) / philox_rate / (dt / args.steps),
            "fold": philox_fold,
        },
        "sweep_alg_roofline_frac": value * SWEEP_BYTES_PER_SITE / (HBM_PEAK_GBS * 1e9),
        "kernels": kernel_bounds(kt, N, cas_tried / max(count_sweeps * len(lats), 1),
                                 cas_hooked / max(count_sweeps * len(lats), 1), cas_ceiling, copy_gbs, counters_valid),
        "binder_U_second_half": binder,
        "binder_U_all_sweeps": binder_all,
        "kernel_mean_us_probe": {k: round(v[1] / v[0] * 1e3, 2) for k, v in kt.items() if v[0]},
    }
    if args.on_sweeps > 0:
        log(f"bench: XY and Heisenberg L=64, {args.on_sweeps} sweeps each")
        out["on"] = on_throughput(args.on_sweeps, stream, dev)
    if args.diluted_sweeps > 0:
        log(f"bench: site-diluted and pure Ising L=128, {args.diluted_sweeps} sweeps each")
        out["diluted"] = diluted_throughput(args.diluted_sweeps, stream, dev)
    if args.graph_sweeps > 0:
        log(f"bench: generic graph path, {args.graph_sweeps} sweeps per lattice")
        out["graph"] = graph_throughput(args.graph_sweeps, stream, dev)
    if args.batch_modes_sweeps > 0:
        log(f"bench: 96-replica batch under each Ising mode, {args.batch_modes_sweeps} sweeps")
        out["batch_modes"] = batch_modes(args.batch_modes_sweeps, stream, dev)
    if args.batch_sweeps > 0:
        log(f"bench: 96-replica batch, {args.batch_sweeps} sweeps, batched then plain")
        out["batched"] = batched_vs_plain(args.batch_sweeps, stream, dev)
    if args.serve_jobs > 0:
        log(f"bench: serving {args.serve_jobs} jobs, then the same jobs plain")
        out["serving"] = serving_vs_plain(args.serve_jobs, args.serve_budget_gb, args.serve_quantum_ms, dev)
    if args.cpu_sweeps > 0:
        log("bench: timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(L, temps[2], seeds[2], args.cpu_sweeps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
