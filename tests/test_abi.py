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
