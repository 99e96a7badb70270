"""CPU oracle for the pyrochlore Swendsen-Wang sweep -- TEST INFRASTRUCTURE.

A ctypes front end for ``pyro_oracle.c``: a plain, slow, single-threaded
restatement of the method of Soldatov, Nefedev, Komura and Okabe (Sec. 2:
model and simulation method; Eq. 1: Hamiltonian; Eq. 2: moment ratio).
Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The HIP library never uses it.

Build: ``python -m oracle.build`` (or ``oracle.build.build()``), which runs
gcc on ``pyro_oracle.c`` with no fast-math and no FP contraction.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

ISING, XY, HEISENBERG = 1, 2, 3
COLD, RANDOM = 0, 1

PLANT_NONE = 0
PLANT_HALF_BETA = 1
PLANT_FLIP_ALL = 2
PLANT_DROP_BONDS = 3
PLANT_REFLECT_SIGN = 4
PLANT_ANTI = 5
PLANT_VACANT_JOIN = 6

# Per-sweep record, same field order as the C struct ``orc_record``.
RECORD_DTYPE = np.dtype(
    [
        ("sweep", "<i8"),
        ("bond_sum", "<i8"),
        ("M_int", "<i8"),
        ("pad", "<i8"),
        ("E", "<f8"),
        ("M", "<f8", (3,)),
        ("m2", "<f8"),
        ("m4", "<f8"),
    ]
)

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _b

        _b.build()
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, u64, i32, f64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int, ctypes.c_double
    lib.orc_philox.argtypes = [vp, vp, vp]
    lib.orc_philox.restype = None
    lib.orc_axis.argtypes = [u64, i64, i32, vp]
    lib.orc_axis.restype = None
    lib.orc_ising_threshold.argtypes = [f64, f64]
    lib.orc_ising_threshold.restype = u64
    lib.orc_pyro_position.argtypes = [i32, i64, vp]
    lib.orc_pyro_position.restype = None
    for name in ("orc_create_pyro", "orc_create_sc"):
        getattr(lib, name).argtypes = [ctypes.POINTER(vp), i32, i32, f64, f64, u64, i32]
        getattr(lib, name).restype = i32
    lib.orc_create_edges.argtypes = [ctypes.POINTER(vp), i64, i64, vp, vp, i32, f64, f64, u64, i32]
    lib.orc_create_edges.restype = i32
    lib.orc_destroy.argtypes = [vp]
    lib.orc_destroy.restype = None
    for name in ("orc_num_sites", "orc_num_bonds", "orc_sweep_index"):
        getattr(lib, name).argtypes = [vp]
        getattr(lib, name).restype = i64
    lib.orc_threshold.argtypes = [vp]
    lib.orc_threshold.restype = u64
    lib.orc_x0.argtypes = [vp]
    lib.orc_x0.restype = ctypes.c_float
    lib.orc_bonds.argtypes = [vp, vp, vp]
    lib.orc_bonds.restype = None
    lib.orc_get_spins.argtypes = [vp, vp]
    lib.orc_get_spins.restype = None
    lib.orc_set_spins.argtypes = [vp, vp, i64]
    lib.orc_set_spins.restype = None
    lib.orc_get_labels.argtypes = [vp, vp]
    lib.orc_get_labels.restype = None
    lib.orc_get_active.argtypes = [vp, vp]
    lib.orc_get_active.restype = None
    lib.orc_label_components.argtypes = [i64, i64, vp, vp, vp, vp]
    lib.orc_label_components.restype = None
    lib.orc_sweep.argtypes = [vp, i64, vp]
    lib.orc_sweep.restype = i32
    lib.orc_measure.argtypes = [vp, vp]
    lib.orc_measure.restype = None
    lib.orc_set_temperature.argtypes = [vp, f64]
    lib.orc_set_temperature.restype = None
    lib.orc_set_plant.argtypes = [vp, i32]
    lib.orc_set_plant.restype = None
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def philox(ctr, key) -> np.ndarray:
    """Philox4x32-10 block for a 4-word counter and 2-word key."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().orc_philox(_ptr(c), _ptr(k), _ptr(out))
    return out


def axis(seed: int, t: int, n: int) -> np.ndarray:
    """Embedding axis of sweep t (uniform unit n-vector, float32[3])."""
    r = np.zeros(3, dtype=np.float32)
    _load().orc_axis(seed, t, n, _ptr(r))
    return r


def ising_threshold(T: float, J: float = 1.0) -> int:
    return int(_load().orc_ising_threshold(T, J))


def pyro_position(L: int, i: int) -> np.ndarray:
    p = np.zeros(3, dtype=np.int32)
    _load().orc_pyro_position(L, i, _ptr(p))
    return p


def label_components(N: int, a, b, active) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.int32)
    b = np.ascontiguousarray(b, dtype=np.int32)
    act = np.ascontiguousarray(active, dtype=np.uint8)
    lab = np.zeros(N, dtype=np.int32)
    _load().orc_label_components(N, len(a), _ptr(a), _ptr(b), _ptr(act), _ptr(lab))
    return lab


class Oracle:
    """One lattice (pyrochlore, simple cubic or an edge list) and its state."""

    def __init__(self, L=None, model=ISING, T=1.0, J=1.0, seed=1, start=COLD, *,
                 lattice="pyro", edges=None, n_sites=None):
        lib = _load()
        h = ctypes.c_void_p()
        if lattice == "pyro":
            rc = lib.orc_create_pyro(ctypes.byref(h), int(L), model, float(T), float(J), seed, start)
        elif lattice == "sc":
            rc = lib.orc_create_sc(ctypes.byref(h), int(L), model, float(T), float(J), seed, start)
        elif lattice == "edges":
            a = np.ascontiguousarray(edges[0], dtype=np.int32)
            b = np.ascontiguousarray(edges[1], dtype=np.int32)
            rc = lib.orc_create_edges(ctypes.byref(h), int(n_sites), len(a), _ptr(a), _ptr(b),
                                      model, float(T), float(J), seed, start)
        else:
            raise ValueError(lattice)
        if rc != 0 or not h.value:
            raise ValueError("oracle: invalid arguments")
        self._h = h
        self._lib = lib
        self.model = model
        self.n = model
        self.N = int(lib.orc_num_sites(h))
        self.NB = int(lib.orc_num_bonds(h))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.orc_destroy(h)
            self._h = None

    @property
    def t(self) -> int:
        return int(self._lib.orc_sweep_index(self._h))

    @property
    def threshold(self) -> int:
        return int(self._lib.orc_threshold(self._h))

    @property
    def x0(self) -> float:
        return float(self._lib.orc_x0(self._h))

    def bonds(self):
        a = np.zeros(self.NB, dtype=np.int32)
        b = np.zeros(self.NB, dtype=np.int32)
        self._lib.orc_bonds(self._h, _ptr(a), _ptr(b))
        return a, b

    def sweep(self, n: int = 1) -> np.ndarray:
        rec = np.zeros(n, dtype=RECORD_DTYPE)
        if self._lib.orc_sweep(self._h, n, _ptr(rec)) != 0:
            raise ValueError("oracle sweep failed")
        return rec

    def measure(self) -> np.ndarray:
        rec = np.zeros(1, dtype=RECORD_DTYPE)
        self._lib.orc_measure(self._h, _ptr(rec))
        return rec[0]

    def spins(self) -> np.ndarray:
        if self.model == ISING:
            out = np.zeros(self.N, dtype=np.int8)
        else:
            out = np.zeros((self.n, self.N), dtype=np.float32)
        self._lib.orc_get_spins(self._h, _ptr(out))
        return out

    def set_spins(self, s: np.ndarray, sweep_index: int) -> None:
        if self.model == ISING:
            s = np.ascontiguousarray(s, dtype=np.int8).reshape(self.N)
        else:
            s = np.ascontiguousarray(s, dtype=np.float32).reshape(self.n, self.N)
        self._lib.orc_set_spins(self._h, _ptr(s), sweep_index)

    def labels(self) -> np.ndarray:
        out = np.zeros(self.N, dtype=np.int32)
        self._lib.orc_get_labels(self._h, _ptr(out))
        return out

    def active(self) -> np.ndarray:
        out = np.zeros(self.NB, dtype=np.uint8)
        self._lib.orc_get_active(self._h, _ptr(out))
        return out

    def set_temperature(self, T: float) -> None:
        self._lib.orc_set_temperature(self._h, float(T))

    def plant(self, which: int) -> None:
        """Plant a deliberate mistake (tests of the pins only)."""
        self._lib.orc_set_plant(self._h, int(which))


def binder(records: np.ndarray, discard: int = 0) -> float:
    """U = <m^4>/<m^2>^2 over the records after the first ``discard`` (Eq. 2)."""
    r = records[discard:]
    return float(np.mean(r["m4"]) / np.mean(r["m2"]) ** 2)
