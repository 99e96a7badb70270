"""Group modes for Ising members: the persistent fused launch (every sweep of
a call in one launch whose workgroups take (replica, phase, tile) items) and
LDS-resident small lattices (one workgroup holds a lattice of L <= 16 for
every sweep of a call).  Neither may change any result: records, spins and
labels are compared bit for bit with each lattice swept alone (and with the
oracle), across tile shapes, split calls, per-member sweep counts and mixes
with O(n) members."""
import sys

import numpy as np
import pytest

import oracle
from paper_1612_08312_amd import pyrosw

pytestmark = pytest.mark.gpu

GRAPH, PERSIST = pyrosw.PYRO_MODE_GRAPH, pyrosw.PYRO_MODE_PERSISTENT


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def lat(**kw):
    return pyrosw.Lattice(**kw)


def same(a, b, e_rtol=0.0):
    assert len(a) == len(b)
    for f in ("sweep", "bond_sum", "M_int", "M", "m2", "m4"):
        np.testing.assert_array_equal(a[f], b[f], err_msg=f)
    if e_rtol:
        np.testing.assert_allclose(a["E"], b["E"], rtol=e_rtol, atol=0)
    else:
        np.testing.assert_array_equal(a["E"], b["E"], err_msg="E")


ISING_MIX = [dict(L=1, model=1, T=4.2, seed=31, start=1), dict(L=2, model=1, T=50.0, seed=32, start=1),
             dict(L=3, model=1, T=4.2139, seed=33, start=1), dict(L=5, model=1, T=4.0, seed=34, start=1),
             dict(L=8, model=1, T=4.3, seed=35, start=1), dict(L=9, model=1, T=4.2139, seed=36, start=0),
             dict(L=12, model=1, T=4.19, seed=37, start=1), dict(L=16, model=1, T=4.2139, seed=38, start=1),
             dict(L=17, model=1, T=4.22, seed=39, start=1), dict(L=24, model=1, T=3.5, seed=40, start=1)]


def solo_runs(cfgs, calls):
    out = []
    for c in cfgs:
        s = lat(**c)
        for n in calls:
            s.sweep(n)
        out.append((s.moments(), s.spins(), s.labels()))
        s.close()
    return out


@pytest.mark.parametrize("mode,resident,shape", [
    (PERSIST, False, pyrosw.PYRO_TILE_8x8x8), (PERSIST, False, pyrosw.PYRO_TILE_8x8x4),
    (PERSIST, False, pyrosw.PYRO_TILE_8x4x4), (PERSIST, True, pyrosw.PYRO_TILE_8x8x8),
    (GRAPH, True, pyrosw.PYRO_TILE_8x4x4)])
def test_modes_equal_solo(mode, resident, shape):
    say("mode case:", mode, resident, pyrosw.TILE_SHAPES[shape])
    calls = (10, 1, 14)
    ref = solo_runs(ISING_MIX, calls)
    grp_l = [lat(**c) for c in ISING_MIX]
    g = pyrosw.Group(grp_l)
    g.set_tile_shape(1, shape)
    g.set_mode(mode, resident)
    assert g.mode() == (mode, resident)
    for n in calls:
        g.sweep(n)
    for (r, s, l), q in zip(ref, grp_l):
        same(q.moments(), r)
        np.testing.assert_array_equal(q.spins(), s)
        np.testing.assert_array_equal(q.labels(), l)
    g.close()


def test_modes_per_member_counts_and_oracle():
    cfgs = [ISING_MIX[i] for i in (3, 6, 7, 9)]
    grp_l = [lat(**c) for c in cfgs]
    g = pyrosw.Group(grp_l)
    g.set_tile_shape(1, pyrosw.PYRO_TILE_8x8x4)
    g.set_mode(PERSIST, True)
    counts = [7, 0, 13, 4]
    g.sweep(0, per_member=counts)
    for c, q, k in zip(cfgs, grp_l, counts):
        o = oracle.Oracle(L=c["L"], model=1, T=c["T"], seed=c["seed"], start=c["start"])
        same(q.moments(), o.sweep(k))
        np.testing.assert_array_equal(q.spins(), o.spins())
        if k:
            np.testing.assert_array_equal(q.labels(), o.labels())
        assert q.next_sweep == k
    g.close()


def test_resident_l16_against_oracle():
    """The largest LDS-resident lattice (65,536 sites, 16-bit forest) over 60
    sweeps near T_c, records, spins and labels against the oracle."""
    c = dict(L=16, model=1, T=4.2139, seed=41, start=1)
    q = lat(**c)
    g = pyrosw.Group([q])
    g.set_mode(GRAPH, True)
    g.sweep(60)
    o = oracle.Oracle(L=16, model=1, T=c["T"], seed=c["seed"], start=1)
    same(q.moments(), o.sweep(60))
    np.testing.assert_array_equal(q.spins(), o.spins())
    np.testing.assert_array_equal(q.labels(), o.labels())
    g.close()


def test_persistent_with_on_members_and_slices():
    """Ising members persistent, O(n) members on per-sweep graphs in the same
    slices; 1 and 3 slices."""
    cfgs = ISING_MIX[3:8] + [dict(L=5, model=2, T=2.0285, seed=51, start=1),
                             dict(L=4, model=3, T=1.31695, seed=52, start=1)]
    ref = solo_runs(cfgs, (12,))
    for nslices in (1, 3):
        grp_l = [lat(**c) for c in cfgs]
        g = pyrosw.Group(grp_l)
        g.set_slices(nslices)
        g.set_mode(PERSIST, True)
        g.sweep(12)
        for (r, s, l), q, c in zip(ref, grp_l, cfgs):
            same(q.moments(), r, e_rtol=1e-13 if c["model"] > 1 else 0.0)
            np.testing.assert_array_equal(q.spins(), s)
            np.testing.assert_array_equal(q.labels(), l)
        g.close()


def test_autotune_chooses_modes_without_changing_results():
    cfgs = [dict(L=L, model=1, T=T, seed=60 + 3 * i + j, start=1)
            for i, L in enumerate((8, 12, 16, 24)) for j, T in enumerate((4.19, 4.2139, 4.24))]
    ref = solo_runs(cfgs, (20,))
    grp_l = [lat(**c) for c in cfgs]
    g = pyrosw.Group(grp_l)
    shapes = g.autotune(trial_sweeps=2)
    say("autotuned:", pyrosw.TILE_SHAPES[shapes[0]], g.mode())
    g.sweep(20)
    for (r, s, l), q in zip(ref, grp_l):
        same(q.moments(), r)
        np.testing.assert_array_equal(q.spins(), s)
        np.testing.assert_array_equal(q.labels(), l)
    g.close()
