"""Pins of the oracle's counter-based generator (Philox4x32-10, Salmon et al.
SC'11) and of the way the oracle consumes it."""
import os

import numpy as np

import oracle

KAT = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")

_M = 0xFFFFFFFF


def _philox_py(ctr, key):
    """Independent pure-Python Philox4x32-10 (test only)."""
    x = list(ctr)
    k0, k1 = key
    for _ in range(10):
        p0 = 0xD2511F53 * x[0]
        p1 = 0xCD9E8D57 * x[2]
        x = [((p1 >> 32) ^ x[1] ^ k0) & _M, p1 & _M, ((p0 >> 32) ^ x[3] ^ k1) & _M, p0 & _M]
        k0 = (k0 + 0x9E3779B9) & _M
        k1 = (k1 + 0xBB67AE85) & _M
    return x


def test_known_answers():
    n = 0
    for line in open(KAT):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(v, 16) for v in line.split()]
        out = oracle.philox(w[0:4], w[4:6])
        assert list(out) == w[6:10]
        assert _philox_py(w[0:4], w[4:6]) == w[6:10]
        n += 1
    assert n == 3


def test_oracle_matches_python_twin_on_random_counters():
    rng = np.random.default_rng(5)
    for _ in range(200):
        c = [int(v) for v in rng.integers(0, 2 ** 32, 4, dtype=np.uint64)]
        k = [int(v) for v in rng.integers(0, 2 ** 32, 2, dtype=np.uint64)]
        assert list(oracle.philox(c, k)) == _philox_py(c, k)


def test_random_start_uses_init_stream_bits():
    seed = 0x1234_5678_9ABC
    o = oracle.Oracle(L=2, seed=seed, start=oracle.RANDOM)
    s = o.spins()
    key = (seed & _M, seed >> 32)
    for i in range(o.N):
        w = _philox_py((i >> 7, 0, 2, 0), key)
        bit = (w[(i >> 5) & 3] >> (i & 31)) & 1
        assert s[i] == (-1 if bit else 1)
    # roughly balanced
    assert abs(int(s.sum())) < 4 * np.sqrt(o.N)


def test_axis_is_unit_and_isotropic():
    for n in (2, 3):
        r = np.array([oracle.axis(3, t, n) for t in range(4000)], dtype=np.float64)
        norms = np.linalg.norm(r, axis=1)
        assert np.all(np.abs(norms - 1) < 1e-6)
        if n == 2:
            assert np.all(r[:, 2] == 0)
        # isotropy: each component has mean 0 and variance 1/n
        assert np.all(np.abs(r[:, :n].mean(0)) < 4 * np.sqrt(1.0 / n / len(r)))
        assert np.all(np.abs((r[:, :n] ** 2).mean(0) - 1.0 / n) < 0.03)


def test_ising_threshold_limits():
    assert oracle.ising_threshold(float("inf")) == 0
    assert oracle.ising_threshold(1e-3) == 2 ** 32
    p = 1 - np.exp(-2 / 4.2139)
    assert abs(oracle.ising_threshold(4.2139) - p * 2 ** 32) <= 1.0
