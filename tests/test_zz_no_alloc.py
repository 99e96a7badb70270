"""The no-allocation entry point pyro_sw_sweep_static against the handle
path (pyro_sw_init_ext + pyro_sw_set_spins + pyro_sw_sweep), through the C
ABI: two calls in a row on one device, the second on a smaller lattice, each
bit-identical to the handle path (records, spins), since both run the same
kernels with the same tile shape."""
import sys

import numpy as np
import pytest

from paper_1612_08312_amd import pyrosw, workloads

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def static_run(L, model, T, seed, s0, first, n, stream):
    import torch

    dev = torch.device("cuda:0")
    spins = torch.from_numpy(np.ascontiguousarray(s0)).to(dev)
    recs = torch.zeros(n * pyrosw.RECORD_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    pyrosw.pyro_sw_sweep_static(spins.data_ptr(), L, model, T, 1.0, seed, first, n, recs.data_ptr(), stream)
    torch.cuda.synchronize()
    return recs.cpu().numpy().view(pyrosw.RECORD_DTYPE), spins.cpu().numpy()


def handle_run(L, model, T, seed, s0, first, n):
    lt = pyrosw.Lattice(L=L, model=model, T=T, seed=seed, start=pyrosw.PYRO_START_COLD)
    lt.set_spins(s0, first)
    lt.sweep(n)
    rec, spins = lt.moments(), lt.spins()
    lt.close()
    return rec, spins


def test_static_sweeps_equal_handle_sweeps():
    import torch

    stream = torch.cuda.current_stream(torch.device("cuda:0"))
    cases = [dict(L=12, model=1, T=4.2139, seed=21, first=40, n=25),   # larger lattice first
             dict(L=5, model=2, T=2.0285, seed=22, first=3, n=12)]     # then a smaller one
    for c in cases:
        say("no-alloc case:", c)
        N = workloads.n_sites(c["L"])
        s0 = (workloads.random_ising_spins(N, c["seed"]) if c["model"] == 1
              else workloads.random_unit_vectors(N, c["model"], c["seed"]))
        rs, ss = static_run(c["L"], c["model"], c["T"], c["seed"], s0, c["first"], c["n"], stream)
        rh, sh = handle_run(c["L"], c["model"], c["T"], c["seed"], s0, c["first"], c["n"])
        assert len(rs) == len(rh) == c["n"]
        for f in ("sweep", "bond_sum", "M_int", "E", "M", "m2", "m4"):
            np.testing.assert_array_equal(rs[f], rh[f], err_msg=f)
        np.testing.assert_array_equal(ss.reshape(sh.shape), sh)


def test_static_rejects_oversized_and_bad_arguments():
    lib = pyrosw.load_library()
    assert lib.pyro_sw_sweep_static(None, 8, 1, 4.0, 1.0, 1, 0, 1, None, None) == pyrosw.PYRO_EINVAL
    assert lib.pyro_sw_sweep_static(256, 81, 1, 4.0, 1.0, 1, 0, 1, 256, None) == pyrosw.PYRO_EINVAL
    assert lib.pyro_sw_sweep_static(256, 8, 1, 4.0, 1.0, 1, -1, 1, 256, None) == pyrosw.PYRO_EINVAL
    assert lib.pyro_sw_sweep_static(258, 8, 1, 4.0, 1.0, 1, 0, 1, 256, None) == pyrosw.PYRO_EINVAL
    assert "80" in pyrosw.last_error() or "aligned" in pyrosw.last_error()
