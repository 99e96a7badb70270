"""Pins of the oracle on site-diluted lattices (the random-system extension
named in Sec. 4; the sweep of Sec. 2 with vacant sites).

A vacant site is a zero spin: Ising 0, O(n) the zero vector.  It carries no
bond, remains a one-site cluster and stays zero; m = M/N with N counting all
sites.  The pins:
  * exact enumeration of the Ising model on the occupied sites of the
    16-site L = 1 lattice (Eqs. 1-2);
  * O(n) on the same diluted lattice against an independent Metropolis
    sampler of the occupied subgraph;
  * T -> 0 from the cold start: the clusters are exactly the connected
    components of the occupied sites (a library connected-components
    routine), every vacancy its own cluster; a planted mistake (two vacant
    sites may activate their bond) fails it;
  * invariants at T_c: vacancies stay zero, occupied Ising spins stay +-1,
    the record's bond sum and magnetisation are the sums over the lattice;
  * a fully vacant lattice has E = M = 0 and one cluster per site.
"""
import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

import oracle
from tests import pins

VACANT_L1 = np.array([1, 6, 11, 12])  # four of the 16 sites of the L = 1 lattice


def vacancies(N, frac, seed):
    rng = np.random.default_rng(seed)
    return np.flatnonzero(rng.random(N) < frac)


def diluted_ising(N, vac, seed, cold=False):
    rng = np.random.default_rng(seed)
    s = np.ones(N, dtype=np.int8) if cold else rng.choice(np.array([-1, 1], dtype=np.int8), N)
    s[vac] = 0
    return s


def diluted_on(N, n, vac, seed):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, N))
    v /= np.linalg.norm(v, axis=0, keepdims=True)
    v = v.astype(np.float32)
    v[:, vac] = 0.0
    return v


def occupied_subgraph(N, a, b, vac):
    occ = np.ones(N, dtype=bool)
    occ[vac] = False
    keep = occ[a] & occ[b]
    idx = -np.ones(N, dtype=np.int64)
    idx[occ] = np.arange(occ.sum())
    return int(occ.sum()), idx[a[keep]], idx[b[keep]]


@pytest.mark.parametrize("T", [4.2139, 2.0])
def test_diluted_l1_exact_enumeration(T):
    o = oracle.Oracle(L=1, T=T, seed=41, start=oracle.RANDOM)
    a, b = o.bonds()
    n_occ, sa, sb = occupied_subgraph(16, a, b, VACANT_L1)
    exact = pins.ising_exact(n_occ, sa, sb, T, norm=16)
    o.set_spins(diluted_ising(16, VACANT_L1, 1), 0)
    rec = o.sweep(300_000)
    ok, info = pins.check_against_exact(rec, exact)
    assert ok, info
    assert np.all(o.spins()[VACANT_L1] == 0)


@pytest.mark.parametrize("n,T", [(2, 2.0285), (3, 1.31695)])
def test_diluted_on_l1_against_metropolis(n, T):
    o = oracle.Oracle(L=1, model=n, T=T, seed=43, start=oracle.RANDOM)
    a, b = o.bonds()
    n_occ, sa, sb = occupied_subgraph(16, a, b, VACANT_L1)
    (Em, eE), (m2m, em2) = pins.metropolis_on(n_occ, sa, sb, n, T, chains=1500, sweeps=1500, discard=200)
    o.set_spins(diluted_on(16, n, VACANT_L1, 2), 0)
    rec = o.sweep(200_000)[200:]
    Eo, eEo = pins.binned_mean(rec["E"])
    m2o, em2o = pins.binned_mean(rec["m2"])
    scale = (n_occ / 16.0) ** 2  # the sampler normalises m by its own site count
    assert abs(Eo - Em) < 4.5 * np.hypot(eE, eEo), (Eo, eEo, Em, eE)
    assert abs(m2o - scale * m2m) < 4.5 * np.hypot(scale * em2, em2o), (m2o, em2o, m2m, em2)
    assert np.all(o.spins()[:, VACANT_L1] == 0.0)


def _zero_t_components(plant=oracle.PLANT_NONE):
    L = 3
    o = oracle.Oracle(L=L, T=1e-3, seed=5, start=oracle.COLD)
    assert o.threshold == 2 ** 32
    N = o.N
    vac = vacancies(N, 0.35, 7)
    if plant:
        o.plant(plant)
    o.set_spins(diluted_ising(N, vac, 3, cold=True), 0)
    o.sweep(1)
    a, b = o.bonds()
    occ = np.ones(N, dtype=bool)
    occ[vac] = False
    keep = occ[a] & occ[b]
    g = coo_matrix((np.ones(int(keep.sum())), (a[keep], b[keep])), shape=(N, N))
    _, comp = connected_components(g, directed=False)
    want = np.zeros(N, dtype=np.int64)
    first = {}
    for i in range(N):  # smallest site of each component
        first.setdefault(comp[i], i)
        want[i] = first[comp[i]]
    return np.array_equal(o.labels(), want), o, vac


def test_diluted_zero_temperature_clusters_are_occupied_components():
    ok, o, vac = _zero_t_components()
    assert ok
    lab = o.labels()
    assert np.array_equal(lab[vac], vac)
    # some vacancies are neighbours, so the planted join below has teeth
    a, b = o.bonds()
    v = np.zeros(o.N, dtype=bool)
    v[vac] = True
    assert np.any(v[a] & v[b])


def test_diluted_zero_temperature_catches_vacant_join():
    ok, _, _ = _zero_t_components(plant=oracle.PLANT_VACANT_JOIN)
    assert not ok


@pytest.mark.parametrize("model", [1, 2, 3])
def test_diluted_invariants_at_tc(model):
    L = 3
    T = {1: 4.2139, 2: 2.0285, 3: 1.31695}[model]
    o = oracle.Oracle(L=L, model=model, T=T, seed=9, start=oracle.RANDOM)
    N = o.N
    vac = vacancies(N, 0.2, 11)
    s0 = diluted_ising(N, vac, 4) if model == 1 else diluted_on(N, model, vac, 4)
    o.set_spins(s0, 0)
    rec = o.sweep(60)
    s = o.spins()
    a, b = o.bonds()
    if model == 1:
        assert np.all(s[vac] == 0)
        occ = np.ones(N, dtype=bool)
        occ[vac] = False
        assert np.all(np.abs(s[occ]) == 1)
        assert int(rec["M_int"][-1]) == int(s.astype(np.int64).sum())
        assert int(rec["bond_sum"][-1]) == int((s[a].astype(np.int64) * s[b]).sum())
    else:
        assert np.all(s[:, vac] == 0.0)
        E = -float((s[:, a].astype(np.float64) * s[:, b]).sum())
        assert rec["E"][-1] == pytest.approx(E, rel=1e-12, abs=1e-9)
    lab = o.labels()
    assert np.array_equal(lab[vac], vac)


@pytest.mark.parametrize("model", [1, 2])
def test_fully_vacant_lattice(model):
    o = oracle.Oracle(L=2, model=model, T=4.0, seed=1, start=oracle.RANDOM)
    N = o.N
    o.set_spins(np.zeros(N, dtype=np.int8) if model == 1 else np.zeros((model, N), dtype=np.float32), 0)
    rec = o.sweep(5)
    assert np.all(rec["E"] == 0.0) and np.all(rec["m2"] == 0.0)
    assert np.array_equal(o.labels(), np.arange(N))
    assert not o.active().any()
