"""Host-side pieces of the serving path, no GPU: the arena allocator that
carves the server's HBM budget (compiled with g++ and checked against a byte
map), the stream driver against a simulated server, and the latency
percentile definition."""
import os
import subprocess

import numpy as np
import pytest

from paper_1612_08312_amd import serving, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1612_08312_amd", "csrc")


def test_arena_allocator(tmp_path):
    exe = str(tmp_path / "arena_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I", CSRC, os.path.join(ROOT, "tests", "arena_check.cpp"),
                    "-o", exe], check=True)
    out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode == 0, out.stderr
    assert "arena ok" in out.stdout


def test_percentile_nearest_rank():
    v = list(range(1, 101))
    assert serving.percentile_nearest_rank(v, 50) == 50
    assert serving.percentile_nearest_rank(v, 99) == 99
    assert serving.percentile_nearest_rank(v, 100) == 100
    assert serving.percentile_nearest_rank([3.0], 99) == 3.0
    assert serving.percentile_nearest_rank([5, 1, 4, 2, 3], 50) == 3


class FakeServer:
    """Single-queue simulation: one job at a time, duration proportional to
    its spin updates; the clock advances only inside step()."""

    def __init__(self, rate=1e9):
        self.t = 0.0
        self.rate = rate
        self.jobs = {}
        self.queue = []
        self.current = None
        self.next_id = 1
        self.submit_times = {}

    def clock(self):
        return self.t

    def submit(self, spec):
        jid = self.next_id
        self.next_id += 1
        self.jobs[jid] = dict(spec=spec, t_submit=self.t, t_admit=-1.0, t_done=-1.0, state=0)
        self.queue.append(jid)
        return jid

    def _advance(self, dt):
        end = self.t + dt
        while True:
            if self.current is None and self.queue:
                self.current = self.queue.pop(0)
                self.jobs[self.current].update(t_admit=self.t, state=1)
            if self.current is None:
                self.t = end
                return
            j = self.jobs[self.current]
            finish = j["t_admit"] + 16 * j["spec"]["L"] ** 3 * j["spec"]["sweeps"] / self.rate
            if finish <= end:
                self.t = max(self.t, finish)
                j.update(t_done=self.t, state=2)
                self.current = None
            else:
                self.t = end
                return

    def step(self, wait_ms):
        self._advance(max(wait_ms, 0.05) * 1e-3)
        return len(self.queue), int(self.current is not None)

    def status(self, jid):
        j = self.jobs[jid]
        return dict(id=jid, state=j["state"], t_submit=j["t_submit"], t_admit=j["t_admit"], t_done=j["t_done"])

    def take(self, jid, spin_bytes=0):
        return np.zeros(self.jobs[jid]["spec"]["sweeps"]), None


def test_stream_driver_against_a_simulated_server():
    jobs = workloads.serving_jobs(n_jobs=12, rate=50.0, seed=7, big_job_index=-1)
    for j in jobs:
        j["L"] = 8
        j["sweeps"] = 100
    srv = FakeServer(rate=2e8)
    results, summary = serving.run_stream(srv, jobs)
    assert len(results) == len(jobs)
    for r in results:
        st = r["status"]
        assert st["state"] == 2
        # submitted no earlier than its arrival, and within a couple of ms of it
        assert st["t_submit"] >= r["job"]["arrival"] - 1e-12
        assert st["t_submit"] <= r["job"]["arrival"] + 3e-3
        assert st["t_submit"] <= st["t_admit"] <= st["t_done"]
        assert len(r["records"]) == r["job"]["sweeps"]
    lat = sorted(r["status"]["t_done"] - r["status"]["t_submit"] for r in results)
    assert summary["p50_latency_s"] == pytest.approx(lat[5])
    assert summary["p99_latency_s"] == pytest.approx(lat[-1])
    assert summary["spin_updates"] == sum(16 * 8 ** 3 * 100 for _ in jobs)


def test_serving_workload_shape():
    jobs = workloads.serving_jobs()
    assert len(jobs) == 200
    arr = np.array([j["arrival"] for j in jobs])
    assert arr[0] == 0 and np.all(np.diff(arr) >= 0)
    assert 0.5 / 20 < np.mean(np.diff(arr)) < 2.0 / 20
    big = [j for j in jobs if j["L"] == 256]
    assert len(big) == 1 and big[0]["model"] == 1
    for j in jobs:
        assert j["model"] in (1, 2, 3) and 500 <= j["sweeps"] <= 5000
        if j["L"] != 256:
            assert j["L"] % 8 == 0 and 8 <= j["L"] <= 128
        assert abs(j["T"] / workloads.TC[j["model"]] - 1) <= 0.02 + 1e-12
