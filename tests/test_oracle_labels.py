"""Pin of the oracle's cluster labeling: connected components of the active
bond graph (scipy), labelled by the smallest site index in each cluster."""
import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

import oracle


def _reference_labels(N, a, b, act):
    m = act.astype(bool)
    g = coo_matrix((np.ones(m.sum()), (a[m], b[m])), shape=(N, N))
    _, comp = connected_components(g, directed=False)
    lab = np.empty(N, dtype=np.int64)
    for c in np.unique(comp):
        idx = np.nonzero(comp == c)[0]
        lab[idx] = idx.min()
    return lab


@pytest.mark.parametrize("seed", range(6))
def test_labels_match_connected_components(seed):
    rng = np.random.default_rng(seed)
    N = int(rng.integers(1, 400))
    NB = int(rng.integers(0, 3 * N))
    a = rng.integers(0, N, NB).astype(np.int32)
    b = rng.integers(0, N, NB).astype(np.int32)
    act = (rng.random(NB) < rng.random()).astype(np.uint8)
    lab = oracle.label_components(N, a, b, act)
    assert np.array_equal(lab, _reference_labels(N, a, b, act))


def test_sweep_labels_are_components_of_sweep_bonds():
    o = oracle.Oracle(L=3, T=4.2139, seed=11, start=oracle.RANDOM)
    a, b = o.bonds()
    for _ in range(3):
        o.sweep(1)
        assert np.array_equal(o.labels(), _reference_labels(o.N, a, b, o.active()))
