"""Pins of the oracle's Swendsen-Wang sweep against exact results.

* exact enumeration of the 16-site L = 1 lattice (2^16 states) for the Ising
  model of Eq. (1), moments of Eq. (2);
* the exact SW transition matrix of one tetrahedron (K4): detailed balance
  with the Boltzmann weights of Eq. (1), and a chi-square test of the
  oracle's one-step transitions;
* the limits of the moment ratio quoted after Eq. (2) (U -> 1 as T -> 0,
  U -> (n+2)/n as T -> infinity, with its exact finite-N form);
* two spins on one bond: closed forms of <s1.s2> for n = 1, 2, 3;
* O(n) on the L = 1 lattice against an independent Metropolis sampler;
* simple cubic and pyrochlore near their critical temperatures (Sec. 3.1,
  Sec. 3.4: metric factor D1 = 1.0 for Ising, so U(T_c) is shared).

Each pin is also shown to fail when a mistake is planted in the oracle.
"""
import json
import os

import numpy as np
import pytest

import oracle
from tests import pins

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


def _l1_graph():
    o = oracle.Oracle(L=1)
    return o.bonds()


# ---------------------------------------------------------------- L = 1 --
def _l1_enumeration_pin(T, plant=oracle.PLANT_NONE, sweeps=300_000, seed=3):
    a, b = _l1_graph()
    exact = pins.ising_exact(16, a, b, T)
    o = oracle.Oracle(L=1, T=T, seed=seed, start=oracle.RANDOM)
    if plant:
        o.plant(plant)
    rec = o.sweep(sweeps)
    return pins.check_against_exact(rec, exact)


@pytest.mark.parametrize("T", [4.2139, 10.0, 2.0])
def test_l1_exact_enumeration(T):
    ok, info = _l1_enumeration_pin(T)
    assert ok, info


@pytest.mark.parametrize("plant", [oracle.PLANT_HALF_BETA, oracle.PLANT_DROP_BONDS, oracle.PLANT_ANTI])
def test_l1_enumeration_catches_planted_mistakes(plant):
    ok, info = _l1_enumeration_pin(4.2139, plant=plant, sweeps=50_000)
    assert not ok, info


# ------------------------------------------------------------------ K4 --
K4 = (np.array([0, 0, 0, 1, 1, 2]), np.array([1, 2, 3, 2, 3, 3]))


def test_k4_transition_matrix_detailed_balance():
    for T in (0.7, 2.0, 4.2139):
        P = pins.sw_transition_matrix(4, *K4, T)
        assert np.allclose(P.sum(axis=1), 1.0)
        pi = pins.boltzmann(4, *K4, T)
        flux = pi[:, None] * P
        assert np.allclose(flux, flux.T, atol=1e-14)
        assert np.allclose(pi @ P, pi, atol=1e-14)


def _k4_chi2(plant=oracle.PLANT_NONE, T=2.0, samples=20_000, start_state=0b0010):
    P = pins.sw_transition_matrix(4, *K4, T)
    o = oracle.Oracle(model=oracle.ISING, T=T, seed=99, lattice="edges", edges=K4, n_sites=4)
    if plant:
        o.plant(plant)
    s0 = np.array([1 - 2 * ((start_state >> k) & 1) for k in range(4)], dtype=np.int8)
    counts = np.zeros(16, dtype=np.int64)
    for t in range(samples):
        o.set_spins(s0, t)
        o.sweep(1)
        s = o.spins()
        counts[int(sum(((1 - int(s[k])) // 2) << k for k in range(4)))] += 1
    return pins.chi2_row(counts, P[start_state])


def test_k4_one_step_transitions():
    ok, info = _k4_chi2()
    assert ok, info


@pytest.mark.parametrize("plant", [oracle.PLANT_FLIP_ALL, oracle.PLANT_HALF_BETA, oracle.PLANT_ANTI])
def test_k4_catches_planted_mistakes(plant):
    ok, info = _k4_chi2(plant=plant)
    assert not ok, info


# -------------------------------------------------------------- limits --
@pytest.mark.parametrize("model", [1, 2, 3])
def test_infinite_temperature(model):
    """beta = 0: no bond is ever active, every site is its own cluster and
    is flipped (reflected) independently; after one sweep the spins are
    i.i.d.  For Ising <m^2> = 1/N and <m^4> = (3N - 2)/N^3 exactly, so
    U = 3 - 2/N -> 3 (Sec. 3.1).  For n > 1 the reflections keep the
    configuration isotropic; U -> (n + 2)/n as N grows."""
    L = 1 if model == 1 else 2
    o = oracle.Oracle(L=L, model=model, T=float("inf"), seed=5, start=oracle.RANDOM)
    rec = o.sweep(1)
    assert np.array_equal(o.labels(), np.arange(o.N))
    assert not o.active().any()
    N = o.N
    if model == 1:
        rec = o.sweep(200_000)
        m2, e2 = pins.binned_mean(rec["m2"])
        assert abs(m2 - 1.0 / N) < 4.5 * e2
        U, eU = pins.binned_binder(rec["m2"], rec["m4"])
        assert abs(U - (3.0 - 2.0 / N)) < 4.5 * eU
        assert abs(3.0 - GOLD["binder_high_T_limit"]["1"]) == 0.0
    else:
        # random start is already isotropic, and reflections through random
        # planes keep it so; compare with the Gaussian limit of Sec. 3.2/3.3
        rec = o.sweep(20_000)
        U, eU = pins.binned_binder(rec["m2"], rec["m4"])
        n = model
        exact_finite = (n + 2) / n - 2.0 / (n * N)  # i.i.d. uniform unit vectors
        assert abs(U - exact_finite) < 4.5 * eU + 1e-3
        assert abs(exact_finite - GOLD["binder_high_T_limit"][str(n)]) < 0.02


def test_zero_temperature_limit():
    """T -> 0 from the cold start: every parallel bond is active, one
    cluster, |m| = 1, E = -3N J and U = 1 exactly (Sec. 3.1)."""
    o = oracle.Oracle(L=2, T=1e-3, seed=1, start=oracle.COLD)
    assert o.threshold == 2 ** 32
    rec = o.sweep(50)
    assert np.all(o.labels() == 0)
    assert np.all(rec["m2"] == 1.0) and np.all(rec["m4"] == 1.0)
    assert np.all(rec["E"] == -3.0 * o.N)
    assert oracle.binder(rec) == GOLD["binder_low_T_limit"]["value"]
    # both signs occur: the one cluster is flipped with probability 1/2
    assert set(np.sign(rec["M_int"]).tolist()) == {-1, 1}


# --------------------------------------------------------- single bond --
def _single_bond_pin(n, T, plant=oracle.PLANT_NONE, sweeps=200_000):
    o = oracle.Oracle(model=n, T=T, seed=17, start=oracle.RANDOM, lattice="edges",
                      edges=(np.array([0]), np.array([1])), n_sites=2)
    if plant:
        o.plant(plant)
    rec = o.sweep(sweeps)
    corr, err = pins.binned_mean(-rec["E"])
    exact = pins.single_bond_correlation(n, 1.0 / T)
    return abs(corr - exact) < 4.5 * err, dict(corr=corr, err=err, exact=exact)


@pytest.mark.parametrize("n,T", [(1, 4.2139), (2, 2.0285), (3, 1.31695), (2, 0.7), (3, 0.5)])
def test_single_bond_closed_form(n, T):
    ok, info = _single_bond_pin(n, T)
    assert ok, info


@pytest.mark.parametrize("n,plant", [(2, oracle.PLANT_REFLECT_SIGN), (3, oracle.PLANT_HALF_BETA),
                                     (3, oracle.PLANT_FLIP_ALL)])
def test_single_bond_catches_planted_mistakes(n, plant):
    ok, info = _single_bond_pin(n, 1.31695 if n == 3 else 2.0285, plant=plant, sweeps=50_000)
    assert not ok, info


# ------------------------------------------------- O(n) vs Metropolis --
@pytest.mark.parametrize("n,T", [(2, 2.0285), (3, 1.31695)])
def test_on_l1_against_metropolis(n, T):
    a, b = _l1_graph()
    (Em, eE), (m2m, em2) = pins.metropolis_on(16, a, b, n, T, chains=1500, sweeps=1500, discard=200)
    o = oracle.Oracle(L=1, model=n, T=T, seed=23, start=oracle.RANDOM)
    rec = o.sweep(200_000)[200:]
    Eo, eEo = pins.binned_mean(rec["E"])
    m2o, em2o = pins.binned_mean(rec["m2"])
    assert abs(Eo - Em) < 4.5 * np.hypot(eE, eEo), (Eo, eEo, Em, eE)
    assert abs(m2o - m2m) < 4.5 * np.hypot(em2, em2o), (m2o, em2o, m2m, em2)
    # spin norms stay at 1 within float32 rounding drift
    s = o.spins().astype(np.float64)
    assert np.max(np.abs(np.sqrt((s * s).sum(0)) - 1)) < 1e-4


# ------------------------------------------------- near criticality --
def test_simple_cubic_and_pyrochlore_share_U_at_Tc():
    """At T_c the moment ratio approaches a universal value for large L.
    The paper finds metric factor D1 = 1.0 for Ising (Sec. 3.4), so the
    pyrochlore U(T_c) and simple-cubic U(T_c) agree.  Loose band around the
    3D Ising value (about 1.60) to allow corrections to scaling at small L."""
    Tsc = GOLD["simple_cubic_critical_temperature"]["1"]
    Tpy = GOLD["critical_temperature"]["1"]
    o = oracle.Oracle(L=8, T=Tsc, seed=2, start=oracle.RANDOM, lattice="sc")
    rec = o.sweep(20_000)
    Usc, esc = pins.binned_binder(rec["m2"][1000:], rec["m4"][1000:])
    o = oracle.Oracle(L=3, T=Tpy, seed=2, start=oracle.RANDOM)
    rec = o.sweep(20_000)
    Upy, epy = pins.binned_binder(rec["m2"][1000:], rec["m4"][1000:])
    assert 1.50 < Usc < 1.70, (Usc, esc)
    assert 1.50 < Upy < 1.70, (Upy, epy)
    assert abs(Usc - Upy) < 0.06 + 4 * np.hypot(esc, epy)


def test_critical_temperature_ratio():
    """T_c(pyrochlore)/T_c(simple cubic) printed as 93.4, 92.1, 91.3 percent."""
    for n in ("1", "2", "3"):
        r = 100 * GOLD["critical_temperature"][n] / GOLD["simple_cubic_critical_temperature"][n]
        assert abs(r - GOLD["ratio_to_simple_cubic_percent"][n]) < 0.05
