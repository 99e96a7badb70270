"""Drive a job server with a timed arrival stream and summarise latency.

``run_stream`` submits each job when the server clock passes its arrival
time (relative to the first call), lets the server schedule in between, and
collects every job's status and results.  The scheduling itself (admission
by HBM footprint, lanes, quanta) is native (``pyro_sw_server_*``); this
module only paces submissions and reads results back.
"""
from __future__ import annotations

import math

import numpy as np

_JOB_KEYS = ("model", "L", "T", "J", "seed", "start", "sweeps", "keep_spins")


def spin_bytes(job: dict) -> int:
    n = 16 * int(job["L"]) ** 3
    return n if int(job["model"]) == 1 else 4 * int(job["model"]) * n


def percentile_nearest_rank(values, q: float) -> float:
    """Smallest value v with at least q% of the values <= v (nearest rank)."""
    v = sorted(values)
    if not v:
        return float("nan")
    k = max(1, math.ceil(q / 100.0 * len(v)))
    return float(v[k - 1])


def run_stream(server, jobs, keep_spins: bool = False, max_wait_ms: float = 2.0, take: bool = True):
    """Submit `jobs` (dicts with an ``arrival`` time in seconds) at their
    arrival times and run until every job is done.

    Returns (results, summary): results[k] = dict(job=..., id=..., status=...,
    records=..., spins=...) in the order of `jobs`; summary holds latency
    percentiles (seconds, submit to done, nearest rank), the makespan and the
    aggregate spin-updates per second.
    """
    order = sorted(range(len(jobs)), key=lambda k: jobs[k]["arrival"])
    ids = [None] * len(jobs)
    t_start = server.clock()
    nxt = 0
    n_queued = n_running = 0
    while True:
        now = server.clock() - t_start
        while nxt < len(order) and jobs[order[nxt]]["arrival"] <= now:
            k = order[nxt]
            spec = {key: jobs[k][key] for key in _JOB_KEYS if key in jobs[k]}
            spec["keep_spins"] = keep_spins
            ids[k] = server.submit(spec)
            nxt += 1
        if nxt == len(order) and n_queued == 0 and n_running == 0 and all(i is not None for i in ids):
            # the previous step reported nothing left; confirm with a fresh round
            n_queued, n_running = server.step(0.0)
            if n_queued == 0 and n_running == 0:
                break
            continue
        wait = max_wait_ms
        if nxt < len(order):
            wait = min(wait, max(0.0, (jobs[order[nxt]]["arrival"] - now) * 1e3))
        n_queued, n_running = server.step(wait)
    results = []
    for k, job in enumerate(jobs):
        st = server.status(ids[k])
        rec, spins = (server.take(ids[k], spin_bytes(job) if keep_spins else 0) if take else (None, None))
        results.append(dict(job=job, id=ids[k], status=st, records=rec, spins=spins))
    lat = [r["status"]["t_done"] - r["status"]["t_submit"] for r in results]
    first = min(r["status"]["t_submit"] for r in results)
    last = max(r["status"]["t_done"] for r in results)
    updates = sum(16 * int(j["L"]) ** 3 * int(j["sweeps"]) for j in jobs)
    summary = {
        "jobs": len(jobs),
        "p50_latency_s": percentile_nearest_rank(lat, 50),
        "p99_latency_s": percentile_nearest_rank(lat, 99),
        "mean_latency_s": float(np.mean(lat)) if lat else float("nan"),
        "makespan_s": last - first,
        "spin_updates": updates,
        "spin_updates_per_s": updates / (last - first) if last > first else float("nan"),
    }
    return results, summary
