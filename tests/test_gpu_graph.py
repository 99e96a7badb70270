"""The generic graph path (any nearest-neighbour table; Sec. 2 and Sec. 4 of
the paper) on the GPU against the oracle: the pyrochlore table of
pyro_sw_bonds reproduces the oracle's pyrochlore trajectory, the simple-cubic
table the oracle's simple-cubic one, and a random graph the oracle's
edge-list mode.  Ising: records, spins and labels bit for bit; O(n): spins
and labels bit for bit, records within 1e-5."""
import sys

import numpy as np
import pytest

import oracle
from paper_1612_08312_amd import pyrosw, workloads

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def compare(g, o, sweeps, model, chunks=2):
    gr, orr = [], []
    for _ in range(chunks):
        g.sweep(sweeps // chunks)
        gr.append(g.moments())
        orr.append(o.sweep(sweeps // chunks))
    gr, orr = np.concatenate(gr), np.concatenate(orr)
    assert len(gr) == len(orr) == sweeps
    np.testing.assert_array_equal(g.spins(), o.spins())
    np.testing.assert_array_equal(g.labels(), o.labels())
    np.testing.assert_array_equal(gr["sweep"], orr["sweep"])
    if model == 1:
        for f in ("bond_sum", "M_int", "E", "m2", "m4"):
            np.testing.assert_array_equal(gr[f], orr[f], err_msg=f)
    else:
        np.testing.assert_allclose(gr["E"], orr["E"], rtol=1e-5, atol=1e-9)
        np.testing.assert_allclose(gr["m2"], orr["m2"], rtol=1e-5, atol=1e-12)


@pytest.mark.parametrize("model,L,T", [(1, 3, 4.2139), (1, 5, 4.0), (2, 3, 2.0285), (3, 4, 1.31695)])
def test_pyrochlore_table_equals_oracle(model, L, T):
    say("GPU case: graph path, pyrochlore table L=%d model=%d T=%g" % (L, model, T))
    bonds = pyrosw.pyro_sw_bonds(L)
    g = pyrosw.Graph(bonds, 16 * L ** 3, model, T, seed=50 + L, start=pyrosw.PYRO_START_RANDOM)
    o = oracle.Oracle(L=L, model=model, T=T, seed=50 + L, start=oracle.RANDOM)
    np.testing.assert_array_equal(g.spins(), o.spins())
    compare(g, o, 120, model)
    g.close()


@pytest.mark.parametrize("model,L,T", [(1, 8, 4.511524), (1, 5, 10.0), (2, 6, 2.20182), (3, 5, 1.4430)])
def test_simple_cubic_equals_oracle(model, L, T):
    say("GPU case: graph path, simple cubic L=%d model=%d T=%g" % (L, model, T))
    g = pyrosw.Graph(pyrosw.simple_cubic_bonds(L), L ** 3, model, T, seed=70 + L)
    o = oracle.Oracle(L=L, model=model, T=T, seed=70 + L, start=oracle.RANDOM, lattice="sc")
    compare(g, o, 200, model)
    g.close()


@pytest.mark.parametrize("model,L,T", [(1, 24, 4.511524), (2, 17, 2.20182)])
def test_simple_cubic_across_windows_equals_oracle(model, L, T):
    """Lattices of several 4096-site windows: bonds inside a window are
    united in LDS, the others in the global forest."""
    say("GPU case: graph path, simple cubic across windows L=%d model=%d" % (L, model))
    g = pyrosw.Graph(pyrosw.simple_cubic_bonds(L), L ** 3, model, T, seed=30 + L)
    o = oracle.Oracle(L=L, model=model, T=T, seed=30 + L, start=oracle.RANDOM, lattice="sc")
    compare(g, o, 60, model)
    g.close()


def ball_cut_fewer(n, a, b, window=4096):
    """The library's window rule, restated: windows grown breadth first from
    the smallest free site, 4096 sites each, are used when they cut fewer
    bonds than windows of consecutive indices.  True when they do."""
    import collections
    adj = [[] for _ in range(n)]
    for x, y in zip(a.tolist(), b.tolist()):
        adj[x].append(y)
        adj[y].append(x)
    win = [-1] * n
    w, fill, nxt, taken = 0, 0, 0, 0
    while taken < n:
        while win[nxt] >= 0:
            nxt += 1
        q = collections.deque([nxt])
        win[nxt] = w
        taken += 1
        fill += 1
        full = fill == window
        while q and not full:
            x = q.popleft()
            for y in adj[x]:
                if win[y] < 0:
                    win[y] = w
                    taken += 1
                    fill += 1
                    q.append(y)
                    if fill == window:
                        full = True
                        break
        if full:
            w, fill = w + 1, 0
    win = np.asarray(win)
    return int(np.sum(win[a] != win[b])) < int(np.sum(a // window != b // window))


@pytest.mark.parametrize("lattice,model,L,T", [("sc", 1, 48, 4.511524), ("sc", 2, 40, 2.20182),
                                               ("pyro", 1, 12, 4.2139)])
def test_breadth_first_windows_equal_oracle(lattice, model, L, T):
    """Tables that breadth-first windows cut less than consecutive ones (so
    the window pass gathers its sites through the window's site list): the
    trajectory is still the oracle's."""
    say("GPU case: graph path, breadth-first windows, %s L=%d model=%d" % (lattice, L, model))
    bonds = pyrosw.simple_cubic_bonds(L) if lattice == "sc" else pyrosw.pyro_sw_bonds(L)
    n = L ** 3 if lattice == "sc" else 16 * L ** 3
    assert ball_cut_fewer(n, np.asarray(bonds[0], np.int64), np.asarray(bonds[1], np.int64))
    g = pyrosw.Graph(bonds, n, model, T, seed=90 + L)
    o = oracle.Oracle(L=L, model=model, T=T, seed=90 + L, start=oracle.RANDOM, lattice=lattice)
    compare(g, o, 20, model)
    g.close()


def test_pyrochlore_table_across_windows_equals_oracle():
    L, T = 7, 4.2139  # 5488 sites: two windows
    say("GPU case: graph path, pyrochlore table across windows L=%d" % L)
    g = pyrosw.Graph(pyrosw.pyro_sw_bonds(L), 16 * L ** 3, 1, T, seed=77)
    o = oracle.Oracle(L=L, model=1, T=T, seed=77, start=oracle.RANDOM)
    compare(g, o, 60, 1)
    g.close()


# N = 6000, NB = 40000: a dense graph (mean degree 13) whose first window
# holds about 21,000 inside bonds
@pytest.mark.parametrize("model,N,NB", [(1, 600, 1800), (2, 600, 1800), (1, 20000, 60000), (3, 20000, 60000),
                                        (1, 6000, 40000)])
def test_random_graph_equals_oracle(model, N, NB):
    rng = np.random.default_rng(9)
    a = rng.integers(0, N, NB)
    b = (a + 1 + rng.integers(0, N - 1, NB)) % N  # never a self-loop; repeated pairs allowed
    T = 2.5 if model == 1 else 1.2
    say("GPU case: graph path, random graph N=%d NB=%d model=%d" % (N, NB, model))  # N = 20000: five windows
    g = pyrosw.Graph((a, b), N, model, T, seed=123)
    o = oracle.Oracle(model=model, T=T, seed=123, start=oracle.RANDOM, lattice="edges", edges=(a, b), n_sites=N)
    compare(g, o, 300, model)
    g.close()


def test_graph_without_bonds_and_with_vacancies():
    say("GPU case: graph path, no bonds; diluted simple cubic")
    N = 1000
    g = pyrosw.Graph((np.zeros(0, np.int32), np.zeros(0, np.int32)), N, 1, 3.0, seed=4)
    o = oracle.Oracle(model=1, T=3.0, seed=4, start=oracle.RANDOM, lattice="edges",
                      edges=(np.zeros(0, np.int32), np.zeros(0, np.int32)), n_sites=N)
    compare(g, o, 50, 1)
    assert np.array_equal(g.labels(), np.arange(N))
    g.close()
    L = 7
    s0 = workloads.diluted_spins(L ** 3, 1, 0.3, 8)
    g = pyrosw.Graph(pyrosw.simple_cubic_bonds(L), L ** 3, 1, 3.5, seed=8, start=pyrosw.PYRO_START_COLD)
    o = oracle.Oracle(L=L, model=1, T=3.5, seed=8, start=oracle.COLD, lattice="sc")
    g.set_spins(s0, 0)
    o.set_spins(s0, 0)
    compare(g, o, 100, 1)
    assert np.all(g.spins()[s0 == 0] == 0)
    g.close()


def test_large_simple_cubic_properties():
    """L = 128 simple cubic (2,097,152 sites) at its T_c: canonical labels,
    equal pre-flip spins within a cluster, exact M and bond sum."""
    L, T, seed = 128, 4.511524, 5
    N = L ** 3
    say("GPU case: graph path, simple cubic L=%d" % L)
    g = pyrosw.Graph(pyrosw.simple_cubic_bonds(L), N, 1, T, seed=seed)
    g.sweep(5)
    before = g.spins()
    g.sweep(1)
    rec = g.moments()
    after, lab = g.spins(), g.labels()
    g.close()
    assert np.all(lab <= np.arange(N)) and np.array_equal(lab[lab], lab)
    assert np.array_equal(before[lab], before)
    s = after.astype(np.int64).reshape(L, L, L)
    bsum = sum(int((s * np.roll(s, -1, axis=ax)).sum()) for ax in (0, 1, 2))
    assert int(rec["M_int"][-1]) == int(s.sum())
    assert int(rec["bond_sum"][-1]) == bsum
