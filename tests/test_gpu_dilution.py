"""Site-diluted lattices (the random-system extension of Sec. 4; a zero spin
is a vacant site) on the GPU against the oracle: Ising records, spins and
labels bit for bit; O(n) spins and labels bit for bit, records within 1e-5;
groups mixing diluted and pure lattices; clearing the dilution; and, at
L = 64, properties that hold at any size."""
import sys

import numpy as np
import pytest

import oracle
from paper_1612_08312_amd import pyrosw, workloads

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def both(L, model, T, seed, vacancy, sweeps):
    say("GPU case: diluted L=%d model=%d T=%g seed=%d vacancy=%g sweeps=%d" % (L, model, T, seed, vacancy, sweeps))
    s0 = workloads.diluted_spins(16 * L ** 3, model, vacancy, seed)
    g = pyrosw.Lattice(L=L, model=model, T=T, seed=seed, start=pyrosw.PYRO_START_COLD)
    o = oracle.Oracle(L=L, model=model, T=T, seed=seed, start=oracle.COLD)
    g.set_spins(s0, 0)
    o.set_spins(s0, 0)
    g.sweep(sweeps)
    return g, o, g.moments(), o.sweep(sweeps), s0


# L = 16 and 24 take the flip's keyed paths (8x4x4 tiles dividing L: bit
# fields for the power of two, the rounding decode for 24)
@pytest.mark.parametrize("L,vacancy", [(4, 0.1), (5, 0.5), (7, 0.25), (2, 1.0), (16, 0.1), (24, 0.2)])
def test_diluted_ising_bit_exact(L, vacancy):
    g, o, gr, orr, s0 = both(L, 1, 4.0, 300 + L, vacancy, 120)
    for f in ("sweep", "bond_sum", "M_int", "E", "m2", "m4"):
        np.testing.assert_array_equal(gr[f], orr[f], err_msg=f)
    s = g.spins()
    np.testing.assert_array_equal(s, o.spins())
    np.testing.assert_array_equal(g.labels(), o.labels())
    vac = np.flatnonzero(s0 == 0)
    assert np.all(s[vac] == 0)
    g.close()


@pytest.mark.parametrize("model,L", [(2, 4), (3, 5), (2, 24)])
def test_diluted_on_parity(model, L):
    T = workloads.TC[model]
    g, o, gr, orr, s0 = both(L, model, T, 400 + L, 0.2, 60)
    np.testing.assert_array_equal(g.spins(), o.spins())
    np.testing.assert_array_equal(g.labels(), o.labels())
    np.testing.assert_array_equal(gr["sweep"], orr["sweep"])
    np.testing.assert_allclose(gr["E"], orr["E"], rtol=1e-5, atol=1e-9)
    np.testing.assert_allclose(gr["m2"], orr["m2"], rtol=1e-5, atol=1e-12)
    g.close()


def test_group_with_diluted_member_equals_solo():
    L, sweeps = 6, 50
    specs = [(1, 4.1, 11, 0.2), (1, 4.2139, 12, 0.0), (2, 2.0285, 13, 0.3)]
    say("GPU case: group of diluted and pure lattices", specs)
    lats, solo = [], []
    for model, T, seed, vac in specs:
        for dst in (lats, solo):
            lt = pyrosw.Lattice(L=L, model=model, T=T, seed=seed, start=pyrosw.PYRO_START_COLD)
            lt.set_spins(workloads.diluted_spins(16 * L ** 3, model, vac, seed), 0)
            dst.append(lt)
    g = pyrosw.Group(lats)
    g.sweep(sweeps)
    for lt, ref in zip(lats, solo):
        ref.sweep(sweeps)
        a, b = lt.moments(), ref.moments()
        for f in ("sweep", "bond_sum", "M_int", "E", "m2", "m4"):
            np.testing.assert_array_equal(a[f], b[f], err_msg=f)
        np.testing.assert_array_equal(lt.spins(), ref.spins())
    g.close()
    for lt in lats + solo:
        lt.close()


def test_clearing_the_dilution_restores_the_pure_lattice():
    L, T, seed = 4, 4.2139, 21
    g = pyrosw.Lattice(L=L, model=1, T=T, seed=seed, start=pyrosw.PYRO_START_COLD)
    g.set_spins(workloads.diluted_spins(16 * L ** 3, 1, 0.3, seed), 0)
    g.sweep(10)
    g.moments()
    pure = workloads.random_ising_spins(16 * L ** 3, seed)
    g.set_spins(pure, 0)
    o = oracle.Oracle(L=L, model=1, T=T, seed=seed, start=oracle.COLD)
    o.set_spins(pure, 0)
    g.sweep(40)
    np.testing.assert_array_equal(g.moments()["bond_sum"], o.sweep(40)["bond_sum"])
    np.testing.assert_array_equal(g.spins(), o.spins())
    with pytest.raises(pyrosw.PyroSWError):
        bad = pure.copy()
        bad[3] = 2
        g.set_spins(bad, 0)
    g.close()


def test_diluted_l64_properties():
    """L = 64, 10% vacant, one sweep at T = 3.8: vacancies keep spin 0 and
    their own label; labels are canonical; the label of every occupied site
    is an occupied site of equal pre-flip spin; the record's M and bond sum
    are the sums over the lattice."""
    c = workloads.DILUTED_ISING_L128
    L = 64
    N = 16 * L ** 3
    say("GPU case: diluted Ising L=%d vacancy=%g T=%g" % (L, c["vacancy"], c["T"]))
    s0 = workloads.diluted_spins(N, 1, c["vacancy"], c["seed"])
    g = pyrosw.Lattice(L=L, model=1, T=c["T"], seed=c["seed"], start=pyrosw.PYRO_START_COLD)
    g.set_spins(s0, 0)
    g.sweep(3)
    before = g.spins()
    g.sweep(1)
    rec = g.moments()
    after, lab = g.spins(), g.labels()
    g.close()
    vac = s0 == 0
    assert np.array_equal(after == 0, vac)
    np.testing.assert_array_equal(lab[vac], np.flatnonzero(vac))
    assert np.all(lab <= np.arange(N)) and np.array_equal(lab[lab], lab)
    occ = ~vac
    assert np.all(before[lab[occ]] == before[occ])
    assert np.all(lab[occ] >= 0) and not np.any(vac[lab[occ]])
    assert int(rec["M_int"][-1]) == int(after.astype(np.int64).sum())
    from tests.test_gpu_large import bond_sum, cell_bond_table
    assert int(rec["bond_sum"][-1]) == bond_sum(L, after.astype(np.int64), cell_bond_table())
    # no occupied site is labelled by a vacancy: every vacant site is a cluster of one
    sizes = np.bincount(lab, minlength=N)
    assert sizes[np.flatnonzero(vac)].max() == 1
