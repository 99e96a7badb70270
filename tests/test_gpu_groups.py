"""Groups (many lattices per captured graph), tile shapes and the autotuner:
none of them may change any result.  Spins, labels, magnetisations and the
Ising energy are compared bit for bit (O(n) included: same FP32 operations
in the same order).  The O(n) energy is an FP64 sum of per-tile partials, so
its last bit follows the tile shape: it is compared to 1e-13 relative when
the tiling differs."""
import sys

import numpy as np
import pytest

import oracle
from paper_1612_08312_amd import pyrosw, workloads

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def lat(**kw):
    say("GPU case:", kw)
    return pyrosw.Lattice(**kw)


def same_records(a, b, e_rtol=0.0):
    assert len(a) == len(b)
    for f in ("sweep", "bond_sum", "M_int", "M", "m2", "m4"):
        np.testing.assert_array_equal(a[f], b[f], err_msg=f)
    if e_rtol:
        np.testing.assert_allclose(a["E"], b["E"], rtol=e_rtol, atol=0)
    else:
        np.testing.assert_array_equal(a["E"], b["E"], err_msg="E")


MIX = [dict(L=3, model=1, T=4.2139, seed=11, start=1), dict(L=8, model=1, T=4.0, seed=12, start=1),
       dict(L=5, model=2, T=2.0285, seed=13, start=1), dict(L=4, model=3, T=1.31695, seed=14, start=1),
       dict(L=9, model=1, T=4.3, seed=15, start=0), dict(L=2, model=3, T=1.0, seed=16, start=1)]


def test_group_matches_solo_mixed_models():
    solo = [lat(**c) for c in MIX]
    for s in solo:
        s.sweep(30)
    grp_l = [lat(**c) for c in MIX]
    g = pyrosw.Group(grp_l)
    g.sweep(10)
    g.sweep(20)
    for s, q in zip(solo, grp_l):
        same_records(s.moments(), q.moments())
        np.testing.assert_array_equal(s.spins(), q.spins())
        np.testing.assert_array_equal(s.labels(), q.labels())
    g.close()


def test_group_per_member_counts_and_oracle():
    cfgs = MIX[:4]
    grp_l = [lat(**c) for c in cfgs]
    g = pyrosw.Group(grp_l)
    counts = [5, 0, 17, 9]
    g.sweep(0, per_member=counts)
    for c, q, k in zip(cfgs, grp_l, counts):
        o = oracle.Oracle(L=c["L"], model=c["model"], T=c["T"], seed=c["seed"], start=c["start"])
        orec = o.sweep(k)
        grec = q.moments()
        assert q.next_sweep == k
        if c["model"] == 1:
            same_records(grec, orec)
            np.testing.assert_array_equal(q.spins(), o.spins())
        else:
            np.testing.assert_allclose(grec["E"], orec["E"], rtol=1e-5)
            np.testing.assert_allclose(q.spins(), o.spins(), rtol=0, atol=1e-5)
        if k:
            np.testing.assert_array_equal(q.labels(), o.labels())
    g.close()


@pytest.mark.parametrize("model,L", [(1, 6), (1, 9), (2, 5), (3, 4)])
def test_tile_shapes_do_not_change_results(model, L):
    ref = None
    for shape in range(len(pyrosw.TILE_SHAPES)):
        x = lat(L=L, model=model, T=workloads.TC[model], seed=21, start=1)
        x.set_tile_shape(shape)
        x.sweep(25)
        out = (x.moments(), x.spins(), x.labels())
        if ref is None:
            ref = out
        else:
            same_records(ref[0], out[0], e_rtol=0.0 if model == 1 else 1e-13)
            np.testing.assert_array_equal(ref[1], out[1])
            np.testing.assert_array_equal(ref[2], out[2])


def test_autotune_changes_no_result():
    cfgs = [dict(L=8, model=1, T=4.2, seed=31, start=1), dict(L=12, model=1, T=4.22, seed=32, start=1),
            dict(L=6, model=2, T=2.0, seed=33, start=1)]
    a = [lat(**c) for c in cfgs]
    b = [lat(**c) for c in cfgs]
    for x in a:
        x.sweep(7)
    ga = pyrosw.Group(a)
    ga.sweep(13)
    gb = pyrosw.Group(b)
    gb.sweep(7)
    shapes = gb.autotune(trial_sweeps=3)
    say("autotuned shapes", shapes)
    gb.sweep(13)
    for x, y in zip(a, b):
        same_records(x.moments(), y.moments(), e_rtol=0.0 if x.model == 1 else 1e-13)
        np.testing.assert_array_equal(x.spins(), y.spins())
    ga.close()
    gb.close()


def test_long_run_ring_drains():
    """More sweeps than the device record ring holds (drains in between)."""
    a = lat(L=1, model=1, T=4.2139, seed=41, start=1)
    o = oracle.Oracle(L=1, model=1, T=4.2139, seed=41, start=1)
    a.sweep(20000)
    same_records(a.moments(), o.sweep(20000))


@pytest.mark.parametrize("nslices", [1, 3, 8])
def test_slices_change_no_result(nslices):
    """The members of a group run as concurrent slices (own stream and
    captured sweep each); any slice count gives the same records."""
    ref = [lat(**kw) for kw in MIX]
    g0 = pyrosw.Group(ref)
    g0.set_slices(1)
    g0.sweep(17)
    want = [lt.moments() for lt in ref]
    g0.close()
    lats = [lat(**kw) for kw in MIX]
    g = pyrosw.Group(lats)
    g.set_slices(nslices)
    g.sweep(9)
    g.set_slices(max(1, nslices - 1))  # re-dealing between calls keeps every trajectory
    g.sweep(8)
    for lt, w in zip(lats, want):
        same_records(lt.moments(), w)
    g.close()
    for lt in ref + lats:
        lt.close()


@pytest.mark.parametrize("T", [3.0, 4.2139, 6.0])
def test_large_tiles_with_long_crossing_lists(T):
    """16x8x8 tiles on a ragged L = 100 lattice: 609 crossing tetrahedra per
    tile, each emitting up to 3 pairs; in the ordered phase (T = 3) most emit
    2 or 3, so a tile's list exceeds the unite pass's 1024 LDS pair slots and
    the direct unions run (and, with many distinct roots, those beyond the
    LDS root table).  Results must equal the 8x8x8 tiling."""
    out = []
    for shape in (3, 4):
        x = lat(L=100, model=1, T=T, seed=31, start=1)
        x.set_tile_shape(shape)
        x.sweep(3)
        out.append((x.moments(), x.spins(), x.labels()))
        x.close()
    same_records(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])
    np.testing.assert_array_equal(out[0][2], out[1][2])
