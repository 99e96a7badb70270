"""Full-size Ising lattices, too large for the oracle to sweep: one GPU sweep is
checked through properties that hold at any size, on sampled sites and
bonds, with the oracle's own Philox and lattice routines.

For the sweep with index t (Swendsen-Wang update of the Ising model, the
cluster construction and flip of the method's update step):
  * labels are canonical: label[i] <= i, label[label[i]] == label[i], and a
    site shares its spin (before the flip) with its cluster's root;
  * every active bond joins two sites of one cluster (bond b is active iff
    its spins are equal and r32(b) < thr, r32 drawn from the BOND / BOND_LO
    streams);
  * each site's new spin is its old spin times -1 exactly when the flip coin
    of its cluster's label is set (FLIP stream);
  * the record's M_int and bond_sum equal the sums over the whole lattice.
L = 406 is the largest lattice the library accepts (N < 2^30): it exercises
the top of the site-index range and ragged tiles of every tile shape.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1612_08312_amd import pyrosw

torch = pytest.importorskip("torch")

ST_BOND, ST_FLIP, ST_BOND_LO = 0, 1, 4


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def cell_bond_table():
    """Bond k (0..47) of cell (x, y, z): (dx_a, dy_a, dz_a, r_a, dx_b, dy_b, dz_b, r_b)
    with site index 16 cell + r, read off the oracle's bond list of a 4^3
    lattice at the interior cell (1, 1, 1)."""
    o = oracle.Oracle(L=4, model=1, T=4.0, seed=1, start=0)
    a, b = o.bonds()
    c0 = (1 * 4 + 1) * 4 + 1
    rows = []
    for k in range(48):
        row = []
        for s in (a[48 * c0 + k], b[48 * c0 + k]):
            c, r = divmod(int(s), 16)
            x, y, z = c % 4, (c // 4) % 4, c // 16
            row += [x - 1, y - 1, z - 1, r]
        rows.append(row)
    return np.array(rows, dtype=np.int64)


def bond_ends(L, bonds, table):
    bonds = np.asarray(bonds, dtype=np.int64)
    cell, k = np.divmod(bonds, 48)
    x, y, z = cell % L, (cell // L) % L, cell // (L * L)
    t = table[k]
    ends = []
    for o in (0, 4):
        xe, ye, ze = (x + t[:, o]) % L, (y + t[:, o + 1]) % L, (z + t[:, o + 2]) % L
        ends.append(16 * ((ze * L + ye) * L + xe) + t[:, o + 3])
    return ends[0], ends[1]


def bond_sum(L, spins, table):
    """Sum over all bonds of s_i s_j, one bond class at a time."""
    s = spins.reshape(L, L, L, 16)  # [z, y, x, r]
    total = 0
    for dxa, dya, dza, ra, dxb, dyb, dzb, rb in table:
        sa = np.roll(s[..., ra], shift=(-dza, -dya, -dxa), axis=(0, 1, 2))
        sb = np.roll(s[..., rb], shift=(-dzb, -dyb, -dxb), axis=(0, 1, 2))
        total += int(np.sum(sa * sb, dtype=np.int64))
    return total


def key_of(seed):
    return [seed & 0xFFFFFFFF, seed >> 32]


def r32(seed, b, t):
    w = oracle.philox([(b >> 4) & 0xFFFFFFFF, t, ST_BOND, 0], key_of(seed))
    hi = (int(w[(b & 15) >> 2]) >> (8 * (b & 3))) & 0xFF
    v = oracle.philox([(b >> 2) & 0xFFFFFFFF, t, ST_BOND_LO, 0], key_of(seed))
    return (hi << 24) | (int(v[b & 3]) & 0xFFFFFF)


def coin(seed, r, t):
    w = oracle.philox([(r >> 7) & 0xFFFFFFFF, t, ST_FLIP, 0], key_of(seed))
    return (int(w[(r >> 5) & 3]) >> (r & 31)) & 1


def test_bond_table_matches_oracle_bonds():
    """The translated cell bond table reproduces the oracle's bond list and
    its bond sum at other sizes (including the 2-cell wrap)."""
    table = cell_bond_table()
    for L in (2, 3, 5):
        o = oracle.Oracle(L=L, model=1, T=4.2139, seed=11, start=1)
        a, b = o.bonds()
        ea, eb = bond_ends(L, np.arange(48 * L ** 3), table)
        np.testing.assert_array_equal(ea, a)
        np.testing.assert_array_equal(eb, b)
        rec = o.sweep(1)
        assert bond_sum(L, o.spins(), table) == int(rec["bond_sum"][0])


def test_coin_and_r32_match_oracle_at_small_size():
    """The sampled-property helpers reproduce the oracle's own sweep on a
    small lattice: flips follow coin(label), active bonds follow r32."""
    L, seed = 3, 21
    o = oracle.Oracle(L=L, model=1, T=4.2139, seed=seed, start=1)
    o.sweep(1)
    before, t = o.spins().copy(), o.t
    o.sweep(1)
    after, lab, act = o.spins(), o.labels(), o.active()
    N = 16 * L ** 3
    flip = np.array([coin(seed, int(lab[i]), t) for i in range(N)])
    np.testing.assert_array_equal(after, before * np.where(flip == 1, -1, 1))
    table = cell_bond_table()
    ea, eb = bond_ends(L, np.arange(48 * L ** 3), table)
    thr = oracle.ising_threshold(4.2139)
    want = np.array([before[i] == before[j] and r32(seed, b, t) < thr
                     for b, (i, j) in enumerate(zip(ea, eb))])
    np.testing.assert_array_equal(act.astype(bool), want)


@pytest.mark.gpu
@pytest.mark.parametrize("L", [256, 406])
def test_full_size_sweep_properties(L):
    T, seed = 4.2139, 31337 + L
    say("GPU case: Ising L=%d T=%g seed=%d random start" % (L, T, seed))
    lt = pyrosw.Lattice(L=L, model=1, T=T, seed=seed, start=pyrosw.PYRO_START_RANDOM)
    N = 16 * L ** 3
    lt.sweep(1)
    before = lt.spins()
    t = lt.next_sweep
    lt.sweep(1)
    rec = lt.moments()
    after = lt.spins()
    lab = lt.labels()
    lt.close()
    say("swept; checking samples")
    assert len(rec) == 2 and int(rec["sweep"][-1]) == t

    rng = np.random.default_rng(L)
    sites = np.concatenate([[0, 1, 15, 16, N - 16, N - 1], rng.integers(0, N, 6000)])
    # sites of the last cell row of every axis (tile and wrap seams)
    cells = np.array([(L - 1), (L - 1) * L, (L - 1) * L * L, L ** 3 - 1, 8 * 8 * 8 - 1])
    sites = np.concatenate([sites, (16 * cells[:, None] + np.arange(16)).ravel()])
    li = lab[sites]
    assert np.all(li <= sites) and np.all(li >= 0)
    np.testing.assert_array_equal(lab[li], li)
    np.testing.assert_array_equal(before[li], before[sites])
    flip = np.array([coin(seed, int(r), t) for r in li])
    np.testing.assert_array_equal(after[sites], before[sites] * np.where(flip == 1, -1, 1))

    table = cell_bond_table()
    thr = oracle.ising_threshold(T)
    bonds = rng.integers(0, 48 * L ** 3, 6000)
    ea, eb = bond_ends(L, bonds, table)
    n_active = 0
    for b, i, j in zip(bonds, ea, eb):
        if before[i] == before[j] and r32(seed, int(b), t) < thr:
            n_active += 1
            assert lab[i] == lab[j], (int(b), int(i), int(j))
    assert n_active > 1000  # near T_c about half the bonds are parallel and ~70% of those active

    assert int(rec["M_int"][-1]) == int(np.sum(after, dtype=np.int64))
    assert int(rec["bond_sum"][-1]) == bond_sum(L, after, table)
