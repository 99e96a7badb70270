"""Seeded synthetic workloads.

Inputs only: lattice sizes, temperatures, seeds, sweep counts and seeded
random spin configurations.  Nothing here performs any step of the
Swendsen-Wang method; both the HIP path and the CPU oracle receive the same
values from this module.

Shapes follow the paper's finite-size-scaling runs (Sec. 2: L x L x L cubic
cells of 16 sites, periodic; Sec. 3: temperatures around each model's T_c,
in units of J).
"""
from __future__ import annotations

import numpy as np

ISING, XY, HEISENBERG = 1, 2, 3
COLD, RANDOM = 0, 1

# Critical temperatures the paper estimates (Sec. 3.1-3.3, in units of J).
TC = {ISING: 4.21394, XY: 2.02850, HEISENBERG: 1.31695}


def n_sites(L: int) -> int:
    """Sites of an L x L x L lattice of 16-site cubic cells (Sec. 2)."""
    return 16 * L ** 3


# Small Ising lattice the oracle finishes in well under a second.
SMALL_ISING = dict(L=4, model=ISING, T=4.2139, J=1.0, seed=1, start=COLD, sweeps=1000)

# Ising L = 128 at five temperatures around T_c, random start.
ISING_L128 = dict(L=128, model=ISING, temps=(4.205, 4.210, 4.2139, 4.218, 4.223),
                  seeds=(1, 2, 3, 4, 5), J=1.0, start=RANDOM, sweeps=10000)

# Continuous-spin lattices, L = 64, random start.
ON_L64 = (
    dict(L=64, model=XY, T=2.0285, J=1.0, seed=1, start=RANDOM, sweeps=5000),
    dict(L=64, model=HEISENBERG, T=1.31695, J=1.0, seed=1, start=RANDOM, sweeps=5000),
)


def batch_replicas():
    """96 Ising replicas: L in {8,12,16,24,32,48} x 16 temperatures spaced
    evenly over [4.19, 4.24] (end points included); replica k = 16*l + i has
    seed 1 + k; random start; 2000 sweeps."""
    Ls = (8, 12, 16, 24, 32, 48)
    temps = np.linspace(4.19, 4.24, 16)
    out = []
    for li, L in enumerate(Ls):
        for ti, T in enumerate(temps):
            k = 16 * li + ti
            out.append(dict(L=L, model=ISING, T=float(T), J=1.0, seed=1 + k, start=RANDOM))
    return out


BATCH_SWEEPS = 2000


def serving_jobs(n_jobs: int = 200, rate: float = 20.0, seed: int = 12345,
                 big_job_index: int = 9, big_L: int = 256):
    """Poisson stream of simulation jobs.

    Each job: model uniform over {Ising, XY, Heisenberg}; L uniform over
    8, 16, ..., 128; T = T_c(model) * (1 + 0.04 * (u - 0.5)); sweeps uniform
    over [500, 5000]; arrival times from exponential gaps of mean 1/rate.
    The job at ``big_job_index`` is replaced by an Ising L = ``big_L`` job.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n_jobs)
    arrivals = np.cumsum(gaps) - gaps[0]
    jobs = []
    for k in range(n_jobs):
        model = int(rng.integers(1, 4))
        L = int(8 * rng.integers(1, 17))
        u = float(rng.random())
        sweeps = int(rng.integers(500, 5001))
        if k == big_job_index:
            model, L = ISING, big_L
        T = TC[model] * (1.0 + 0.04 * (u - 0.5))
        jobs.append(dict(job_id=k, arrival=float(arrivals[k]), model=model, L=L, T=T,
                         J=1.0, seed=1000 + k, start=RANDOM, sweeps=sweeps))
    return jobs


def random_ising_spins(N: int, seed: int) -> np.ndarray:
    """Seeded +-1 int8 configuration of N sites."""
    rng = np.random.default_rng(seed)
    return np.where(rng.random(N) < 0.5, 1, -1).astype(np.int8)


def random_unit_vectors(N: int, n: int, seed: int) -> np.ndarray:
    """Seeded unit n-vectors, float32, component-major [n][N]."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, N))
    v /= np.linalg.norm(v, axis=0, keepdims=True)
    return v.astype(np.float32)


def diluted_spins(N: int, model: int, vacancy: float, seed: int) -> np.ndarray:
    """Seeded site-diluted configuration: each site is vacant (zero spin)
    independently with probability ``vacancy``; the others hold a random
    +-1 (Ising, int8 [N]) or a random unit vector (float32 [n][N])."""
    rng = np.random.default_rng(seed)
    vac = rng.random(N) < vacancy
    if model == ISING:
        s = random_ising_spins(N, seed + 1)
        s[vac] = 0
    else:
        s = random_unit_vectors(N, model, seed + 1)
        s[:, vac] = 0.0
    return s


# Site-diluted Ising lattice: L = 128, 10% vacant sites, T = 3.8 (the pure
# lattice orders there, T_c = 4.21394; the diluted one does not).
DILUTED_ISING_L128 = dict(L=128, model=ISING, T=3.8, J=1.0, seed=7, vacancy=0.1)

# Simple-cubic Ising lattice for the generic graph path: L = 256
# (16,777,216 sites, 3 bonds per site) at the simple-cubic T_c the paper
# quotes (Sec. 3.1), random start.
SC_ISING_L256 = dict(L=256, model=ISING, T=4.511524, J=1.0, seed=3)
