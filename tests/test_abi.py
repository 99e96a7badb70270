"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

from paper_1612_08312_amd import pyrosw

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "pyro_sw.h")).read()
    return sorted(set(re.findall(r"\b(pyro_sw_\w+)\s*\(", text)))


def test_header_and_binding_agree():
    assert _declared_symbols() == sorted(pyrosw.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = pyrosw.load_library()
    for name in _declared_symbols():
        assert hasattr(lib, name), name


def test_record_layout():
    assert pyrosw.RECORD_DTYPE.itemsize == 80


@pytest.mark.parametrize("args", [
    dict(L=0, model=1, T=4.0), dict(L=407, model=1, T=4.0), dict(L=4, model=0, T=4.0),
    dict(L=4, model=4, T=4.0), dict(L=4, model=1, T=0.0), dict(L=4, model=1, T=-1.0),
    dict(L=4, model=1, T=float("nan")), dict(L=4, model=1, T=4.0, J=0.0),
    dict(L=4, model=1, T=4.0, J=float("inf")), dict(L=4, model=1, T=4.0, start=2),
])
def test_init_rejects_bad_arguments_without_a_device(args):
    with pytest.raises(pyrosw.PyroSWError) as ei:
        pyrosw.pyro_sw_init(**args)
    assert ei.value.status == pyrosw.PYRO_EINVAL


def test_workspace_size():
    s, w = pyrosw.pyro_sw_workspace_size(4, 1)
    assert s == 1024 and s % 256 == 0 and w % 256 == 0
    s3, _ = pyrosw.pyro_sw_workspace_size(4, 3)
    assert s3 == 3 * 4 * 1024
    with pytest.raises(pyrosw.PyroSWError):
        pyrosw.pyro_sw_workspace_size(4, 5)


def test_null_handle_calls():
    lib = pyrosw.load_library()
    assert lib.pyro_sw_sweep(None, 1) == pyrosw.PYRO_EINVAL
    assert lib.pyro_sw_destroy(None) == pyrosw.PYRO_OK
    n = ctypes.c_int64()
    assert lib.pyro_sw_moments(None, None, 0, ctypes.byref(n)) == pyrosw.PYRO_EINVAL
    assert pyrosw.pyro_sw_strerror(pyrosw.PYRO_EDEVICE) == "HIP device error"


@pytest.mark.parametrize("args", [
    dict(hbm_budget=1000), dict(hbm_budget=1 << 30, max_running=0),
    dict(hbm_budget=1 << 30, quantum_ms=0.0), dict(hbm_budget=1 << 30, quantum_ms=float("nan")),
    dict(hbm_budget=1 << 30, starve_ms=-1.0),
])
def test_server_create_rejects_bad_arguments_without_a_device(args):
    with pytest.raises(pyrosw.PyroSWError) as ei:
        pyrosw.pyro_sw_server_create(**args)
    assert ei.value.status == pyrosw.PYRO_EINVAL


def test_server_job_bytes():
    s, w = pyrosw.pyro_sw_workspace_size(8, 2)
    up = lambda v: (v + 255) // 256 * 256
    assert pyrosw.pyro_sw_server_job_bytes(dict(model=2, L=8, T=2.0, sweeps=1)) == up(s) + up(w)
    for bad in (dict(model=1, L=407, T=4.0, sweeps=1), dict(model=4, L=8, T=4.0, sweeps=1)):
        with pytest.raises(pyrosw.PyroSWError):
            pyrosw.pyro_sw_server_job_bytes(bad)


def test_server_null_calls():
    lib = pyrosw.load_library()
    jid = ctypes.c_int64()
    spec = pyrosw.JobSpec(model=1, L=4, T=4.0, J=1.0, seed=1, start=0, keep_spins=0, sweeps=10)
    assert lib.pyro_sw_server_submit(None, ctypes.byref(spec), ctypes.byref(jid)) == pyrosw.PYRO_EINVAL
    assert lib.pyro_sw_server_step(None, 0.0, None, None) == pyrosw.PYRO_EINVAL
    assert lib.pyro_sw_server_destroy(None) == pyrosw.PYRO_OK
    assert ctypes.sizeof(pyrosw.JobSpec) == 48 and ctypes.sizeof(pyrosw.JobStatus) == 64


def test_group_set_slices_null():
    lib = pyrosw.load_library()
    assert lib.pyro_sw_group_set_slices(None, 2) == pyrosw.PYRO_EINVAL


@pytest.mark.parametrize("calls,repeats", [(0, 1), (-5, 1), ((1 << 32) + 1, 1), (16, 0)])
def test_philox_rate_rejects_bad_arguments_without_a_device(calls, repeats):
    with pytest.raises(pyrosw.PyroSWError) as ei:
        pyrosw.pyro_sw_philox_rate(calls, repeats)
    assert ei.value.status == pyrosw.PYRO_EINVAL


def test_philox_rate_null_outputs():
    lib = pyrosw.load_library()
    assert lib.pyro_sw_philox_rate(16, 1, 1, None, None) == pyrosw.PYRO_EINVAL


def test_bond_tables_match_the_oracle():
    """pyro_sw_bonds and pyro_sw_sc_bonds (host code of the library) give the
    oracle's bond lists, bond for bond."""
    import numpy as np

    import oracle

    for L in (1, 2, 3, 5):
        a, b = pyrosw.pyro_sw_bonds(L)
        oa, ob = oracle.Oracle(L=L).bonds()
        np.testing.assert_array_equal(a, oa)
        np.testing.assert_array_equal(b, ob)
    for L in (2, 3, 6):
        a, b = pyrosw.simple_cubic_bonds(L)
        oa, ob = oracle.Oracle(L=L, lattice="sc").bonds()
        np.testing.assert_array_equal(a, oa)
        np.testing.assert_array_equal(b, ob)
    with pytest.raises(pyrosw.PyroSWError):
        pyrosw.pyro_sw_bonds(0)
    with pytest.raises(pyrosw.PyroSWError):
        pyrosw.simple_cubic_bonds(0)
    lib = pyrosw.load_library()
    a = np.zeros(3 * 8, np.int32)
    assert lib.pyro_sw_sc_bonds(2, a.ctypes.data, a.ctypes.data, 3 * 8 - 1) == pyrosw.PYRO_EINVAL
    assert lib.pyro_sw_sc_bonds(2, None, a.ctypes.data, 3 * 8) == pyrosw.PYRO_EINVAL


@pytest.mark.parametrize("bonds,n,model", [
    (([0], [0]), 4, 1),      # a site joined to itself
    (([0], [4]), 4, 1),      # an end out of range
    (([-1], [2]), 4, 1),
    (([0], [1]), 0, 1),      # no sites
    (([0], [1]), 4, 5),      # bad model
])
def test_graph_init_rejects_bad_arguments_without_a_device(bonds, n, model):
    import numpy as np

    lib = pyrosw.load_library()
    a = np.asarray(bonds[0], np.int32)
    b = np.asarray(bonds[1], np.int32)
    h = ctypes.c_void_p()
    rc = lib.pyro_sw_graph_init(ctypes.byref(h), n, len(a), a.ctypes.data_as(ctypes.c_void_p),
                                b.ctypes.data_as(ctypes.c_void_p), model, 4.0, 1.0, 1, 0, None)
    assert rc == pyrosw.PYRO_EINVAL and not h.value


@pytest.mark.parametrize("args", [(2, 16, 16, 1), (0, 0, 16, 1), (0, (1 << 32) + 1, 16, 1), (0, 16, 0, 1),
                                  (1, 16, 16, 0)])
def test_atomic_rate_rejects_bad_arguments_without_a_device(args):
    with pytest.raises(pyrosw.PyroSWError) as ei:
        pyrosw.pyro_sw_atomic_rate(*args)
    assert ei.value.status == pyrosw.PYRO_EINVAL
