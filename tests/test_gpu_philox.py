"""Philox4x32-10 on the device against the oracle's generator, through the
library's throughput probe: the XOR fold of every output word of blocks
(i, 0x5EED, BOND, 0), i < calls, must equal the fold the oracle computes
block by block, for several seeds (including one with a nonzero high key
word) and a call count that is not a multiple of the probe's grid."""
import numpy as np
import pytest

import oracle
from paper_1612_08312_amd import pyrosw

pytestmark = pytest.mark.gpu

ST_BOND = 0


def oracle_fold(calls, seed):
    key = [seed & 0xFFFFFFFF, seed >> 32]
    f = 0
    for i in range(calls):
        w = oracle.philox([i, 0x5EED, ST_BOND, 0], key)
        f ^= int(w[0]) ^ int(w[1]) ^ int(w[2]) ^ int(w[3])
    return f


@pytest.mark.parametrize("seed", [1, 2024, (7 << 32) | 99])
def test_device_philox_fold_matches_oracle(seed):
    calls = 3001
    rate, fold = pyrosw.pyro_sw_philox_rate(calls, repeats=1, seed=seed)
    assert rate > 0
    assert fold == oracle_fold(calls, seed)


def test_atomic_rate_loses_no_update():
    """The atomic-throughput probe: every successful compare-and-swap shows
    in the array's sum, and one-address adds count every operation."""
    rate, ok, total = pyrosw.pyro_sw_atomic_rate(0, 1 << 20, 1 << 22, 1)
    assert rate > 0 and 0 < ok <= 1 << 22 and total == ok
    rate, ok, total = pyrosw.pyro_sw_atomic_rate(1, 1, 1 << 20, 1)
    assert rate > 0 and ok == 1 << 20 and total == 1 << 20
