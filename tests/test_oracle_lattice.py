"""Pins of the oracle's lattice against geometry and the paper's numbers
(Sec. 2: 16-site cubic cell, L^3 cells, periodic, N = 16 L^3, coordination
six; Fig. 1: corner-sharing tetrahedra)."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1612_08312_amd import workloads
from tests import pins

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")


@pytest.mark.parametrize("L", [1, 2, 3])
def test_bonds_are_exactly_the_nearest_neighbour_pairs(L):
    o = oracle.Oracle(L=L)
    a, b = o.bonds()
    pos = pins.pyro_positions(L)
    assert o.N == 16 * L ** 3 == len(pos)
    # the oracle's own positions agree with the numbering
    for i in range(o.N):
        assert np.array_equal(oracle.pyro_position(L, i), pos[i])
    # all positions distinct on the periodic box
    assert len({tuple(p % (4 * L)) for p in pos}) == o.N
    brute = pins.nn_pairs_brute_force(pos, 4 * L)
    mine = {(min(x, y), max(x, y)) for x, y in zip(a.tolist(), b.tolist())}
    assert len(mine) == o.NB == 3 * o.N  # no multi-edges
    assert mine == brute


@pytest.mark.parametrize("L", [1, 2, 3])
def test_corner_sharing_tetrahedra(L):
    o = oracle.Oracle(L=L)
    a, b = o.bonds()
    deg = np.bincount(np.concatenate([a, b]), minlength=o.N)
    assert np.all(deg == 6)  # coordination number six (Sec. 2)
    tets = []
    for t in range(o.NB // 6):
        verts = set(a[6 * t:6 * t + 6].tolist()) | set(b[6 * t:6 * t + 6].tolist())
        pairs = {(min(x, y), max(x, y)) for x, y in zip(a[6 * t:6 * t + 6], b[6 * t:6 * t + 6])}
        assert len(verts) == 4 and len(pairs) == 6  # a complete K4
        tets.append(verts)
    # every site lies in exactly two tetrahedra, which share only that site
    member = [[] for _ in range(o.N)]
    for k, v in enumerate(tets):
        for s in v:
            member[s].append(k)
    for s in range(o.N):
        assert len(member[s]) == 2
        t1, t2 = member[s]
        assert tets[t1] & tets[t2] == {s}
    # 8 tetrahedra per cubic cell, bond b in tetrahedron b // 6
    assert len(tets) == 8 * L ** 3


def test_paper_system_sizes():
    g = json.load(open(GOLD))["sites_per_L"]
    for L in (32, 48, 64, 96):
        assert workloads.n_sites(L) == g[str(L)]
    o = oracle.Oracle(L=32)
    assert o.N == g["32"]
    assert o.NB == 3 * g["32"]


def test_simple_cubic_lattice():
    o = oracle.Oracle(L=4, lattice="sc")
    a, b = o.bonds()
    assert o.N == 64 and o.NB == 192
    assert np.all(np.bincount(np.concatenate([a, b]), minlength=64) == 6)
    assert len({(min(x, y), max(x, y)) for x, y in zip(a, b)}) == 192
