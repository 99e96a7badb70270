"""Python binding of the C ABI in ``include/pyro_sw.h`` (argument marshalling
only; every step of the sweep runs in the HIP library ``libpyrosw.so``).

Functions carry the C names.  ``Lattice`` is a convenience wrapper whose
device memory (spins and workspace) is owned by PyTorch tensors and whose
work runs on a PyTorch (HIP) stream.

If the library has not been built, loading fails loudly: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpyrosw.so")

PYRO_ISING, PYRO_XY, PYRO_HEISENBERG = 1, 2, 3
PYRO_START_COLD, PYRO_START_RANDOM = 0, 1
PYRO_OK, PYRO_EINVAL, PYRO_ENOMEM, PYRO_EDEVICE, PYRO_ESTATE = 0, -1, -2, -3, -4

# Same field order and size (80 bytes) as pyro_sw_record.
RECORD_DTYPE = np.dtype(
    [
        ("sweep", "<i8"),
        ("bond_sum", "<i8"),
        ("M_int", "<i8"),
        ("reserved", "<i8"),
        ("E", "<f8"),
        ("M", "<f8", (3,)),
        ("m2", "<f8"),
        ("m4", "<f8"),
    ]
)

# Every symbol the header declares.
EXPORTS = (
    "pyro_sw_init", "pyro_sw_workspace_size", "pyro_sw_init_ext", "pyro_sw_sweep",
    "pyro_sw_moments", "pyro_sw_get_spins", "pyro_sw_set_spins", "pyro_sw_get_labels",
    "pyro_sw_set_temperature", "pyro_sw_info", "pyro_sw_set_timing", "pyro_sw_kernel_times",
    "pyro_sw_destroy", "pyro_sw_strerror", "pyro_sw_last_error", "pyro_sw_set_tile_shape",
    "pyro_sw_group_create", "pyro_sw_group_sweep", "pyro_sw_group_autotune",
    "pyro_sw_group_set_tile_shape", "pyro_sw_group_set_timing", "pyro_sw_group_kernel_times",
    "pyro_sw_group_destroy", "pyro_sw_group_set_slices", "pyro_sw_group_set_mode", "pyro_sw_group_get_mode",
    "pyro_sw_group_set_counting", "pyro_sw_group_counts",
    "pyro_sw_server_create", "pyro_sw_server_job_bytes", "pyro_sw_server_submit", "pyro_sw_server_step",
    "pyro_sw_server_status", "pyro_sw_server_take", "pyro_sw_server_clock", "pyro_sw_server_destroy",
    "pyro_sw_philox_rate", "pyro_sw_sweep_static", "pyro_sw_atomic_rate",
    "pyro_sw_graph_init", "pyro_sw_graph_sweep", "pyro_sw_graph_moments", "pyro_sw_graph_get_spins",
    "pyro_sw_graph_set_spins", "pyro_sw_graph_get_labels", "pyro_sw_graph_set_temperature",
    "pyro_sw_graph_destroy", "pyro_sw_bonds", "pyro_sw_sc_bonds",
)

PYRO_JOB_QUEUED, PYRO_JOB_RUNNING, PYRO_JOB_DONE = 0, 1, 2
PYRO_MODE_GRAPH, PYRO_MODE_PERSISTENT = 0, 1


class JobSpec(ctypes.Structure):
    """pyro_sw_job."""
    _fields_ = [("model", ctypes.c_int), ("L", ctypes.c_int), ("T", ctypes.c_double), ("J", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("start", ctypes.c_int), ("keep_spins", ctypes.c_int),
                ("sweeps", ctypes.c_int64)]


class JobStatus(ctypes.Structure):
    """pyro_sw_job_status."""
    _fields_ = [("id", ctypes.c_int64), ("state", ctypes.c_int), ("lane", ctypes.c_int),
                ("sweeps_done", ctypes.c_int64), ("footprint", ctypes.c_int64), ("error", ctypes.c_int),
                ("reserved", ctypes.c_int), ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double)]

PYRO_TILE_8x8x4, PYRO_TILE_8x4x4, PYRO_TILE_4x4x4, PYRO_TILE_8x8x8, PYRO_TILE_16x8x8 = 0, 1, 2, 3, 4
TILE_SHAPES = {0: "8x8x4", 1: "8x4x4", 2: "4x4x4", 3: "8x8x8", 4: "16x8x8"}


class PyroSWError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {pyro_sw_strerror(status)} ({status}): {last_error()}")


_lib = None


def load_library():
    """Load ``libpyrosw.so``; raises if it is missing (build it first with
    ``python -m paper_1612_08312_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                           "(run python -m paper_1612_08312_amd.build)")
    # PyTorch ships its own HIP runtime under the same soname.  Loading it
    # first makes the library bind to that one, so that the library and
    # PyTorch share one runtime and one device context; loaded the other way
    # round, the library's first stream creation has reported no device.
    import torch  # noqa: F401

    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, u64, i32, f64, sz = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int,
                                  ctypes.c_double, ctypes.c_size_t)
    P = ctypes.POINTER
    lib.pyro_sw_init.argtypes = [P(vp), i32, i32, f64, f64, u64, i32, vp]
    lib.pyro_sw_workspace_size.argtypes = [i32, i32, P(sz), P(sz)]
    lib.pyro_sw_init_ext.argtypes = [P(vp), i32, i32, f64, f64, u64, i32, vp, vp, sz, vp, sz]
    lib.pyro_sw_sweep.argtypes = [vp, i64]
    lib.pyro_sw_moments.argtypes = [vp, vp, i64, P(i64)]
    lib.pyro_sw_get_spins.argtypes = [vp, vp, sz]
    lib.pyro_sw_set_spins.argtypes = [vp, vp, sz, i64]
    lib.pyro_sw_get_labels.argtypes = [vp, vp, sz]
    lib.pyro_sw_set_temperature.argtypes = [vp, f64]
    lib.pyro_sw_info.argtypes = [vp, P(i64), P(i64)]
    lib.pyro_sw_set_timing.argtypes = [vp, i32]
    lib.pyro_sw_kernel_times.argtypes = [vp, P(ctypes.c_char_p), P(i64), P(f64), i32, P(i32)]
    lib.pyro_sw_destroy.argtypes = [vp]
    lib.pyro_sw_philox_rate.argtypes = [i64, i32, u64, P(f64), P(ctypes.c_uint32)]
    lib.pyro_sw_sweep_static.argtypes = [vp, i32, i32, f64, f64, u64, i64, i64, vp, vp]
    lib.pyro_sw_atomic_rate.argtypes = [i32, i64, i64, i32, P(f64), P(i64), P(i64)]
    lib.pyro_sw_set_tile_shape.argtypes = [vp, i32]
    lib.pyro_sw_group_create.argtypes = [P(vp), P(vp), i32, vp]
    lib.pyro_sw_group_sweep.argtypes = [vp, i64, P(i64)]
    lib.pyro_sw_group_autotune.argtypes = [vp, i32, P(i32)]
    lib.pyro_sw_group_set_tile_shape.argtypes = [vp, i32, i32]
    lib.pyro_sw_group_set_slices.argtypes = [vp, i32]
    lib.pyro_sw_group_set_mode.argtypes = [vp, i32, i32]
    lib.pyro_sw_group_get_mode.argtypes = [vp, P(i32), P(i32)]
    lib.pyro_sw_group_set_counting.argtypes = [vp, i32]
    lib.pyro_sw_group_counts.argtypes = [vp, P(i64), P(i64)]
    lib.pyro_sw_group_set_timing.argtypes = [vp, i32]
    lib.pyro_sw_group_kernel_times.argtypes = [vp, P(ctypes.c_char_p), P(i64), P(f64), i32, P(i32)]
    lib.pyro_sw_group_destroy.argtypes = [vp]
    lib.pyro_sw_server_create.argtypes = [P(vp), sz, i32, f64, f64]
    lib.pyro_sw_server_job_bytes.argtypes = [P(JobSpec), P(sz)]
    lib.pyro_sw_server_submit.argtypes = [vp, P(JobSpec), P(i64)]
    lib.pyro_sw_server_step.argtypes = [vp, f64, P(i32), P(i32)]
    lib.pyro_sw_server_status.argtypes = [vp, i64, P(JobStatus)]
    lib.pyro_sw_server_take.argtypes = [vp, i64, vp, i64, P(i64), vp, sz]
    lib.pyro_sw_server_clock.argtypes = [vp, P(f64)]
    lib.pyro_sw_server_destroy.argtypes = [vp]
    lib.pyro_sw_graph_init.argtypes = [P(vp), i64, i64, vp, vp, i32, f64, f64, u64, i32, vp]
    lib.pyro_sw_graph_sweep.argtypes = [vp, i64]
    lib.pyro_sw_graph_moments.argtypes = [vp, vp, i64, P(i64)]
    lib.pyro_sw_graph_get_spins.argtypes = [vp, vp, sz]
    lib.pyro_sw_graph_set_spins.argtypes = [vp, vp, sz, i64]
    lib.pyro_sw_graph_get_labels.argtypes = [vp, vp, sz]
    lib.pyro_sw_graph_set_temperature.argtypes = [vp, f64]
    lib.pyro_sw_graph_destroy.argtypes = [vp]
    lib.pyro_sw_bonds.argtypes = [i32, vp, vp, i64]
    lib.pyro_sw_sc_bonds.argtypes = [i32, vp, vp, i64]
    lib.pyro_sw_strerror.argtypes = [i32]
    lib.pyro_sw_strerror.restype = ctypes.c_char_p
    lib.pyro_sw_last_error.argtypes = []
    lib.pyro_sw_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("pyro_sw_strerror", "pyro_sw_last_error"):
            getattr(lib, name).restype = i32
    _lib = lib
    return lib


def pyro_sw_strerror(status: int) -> str:
    return load_library().pyro_sw_strerror(int(status)).decode()


def last_error() -> str:
    return load_library().pyro_sw_last_error().decode()


def _check(rc: int, where: str):
    if rc != PYRO_OK:
        raise PyroSWError(rc, where)


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # torch.cuda.Stream


def pyro_sw_init(L, model, T, J=1.0, seed=1, start=PYRO_START_RANDOM, stream=None):
    h = ctypes.c_void_p()
    _check(load_library().pyro_sw_init(ctypes.byref(h), int(L), int(model), float(T), float(J),
                                       int(seed), int(start), _stream_ptr(stream)), "pyro_sw_init")
    return h


def pyro_sw_workspace_size(L, model):
    s, w = ctypes.c_size_t(), ctypes.c_size_t()
    _check(load_library().pyro_sw_workspace_size(int(L), int(model), ctypes.byref(s), ctypes.byref(w)),
           "pyro_sw_workspace_size")
    return s.value, w.value


def pyro_sw_init_ext(L, model, T, J, seed, start, stream, dev_spins, spin_bytes, dev_work, work_bytes):
    h = ctypes.c_void_p()
    _check(load_library().pyro_sw_init_ext(ctypes.byref(h), int(L), int(model), float(T), float(J),
                                           int(seed), int(start), _stream_ptr(stream), int(dev_spins),
                                           int(spin_bytes), int(dev_work), int(work_bytes)),
           "pyro_sw_init_ext")
    return h


def pyro_sw_sweep(h, n_sweeps):
    _check(load_library().pyro_sw_sweep(h, int(n_sweeps)), "pyro_sw_sweep")


def pyro_sw_moments(h, cap=None) -> np.ndarray:
    lib = load_library()
    n = ctypes.c_int64()
    if cap is None:
        _check(lib.pyro_sw_moments(h, None, 0, ctypes.byref(n)), "pyro_sw_moments")
        cap = n.value
    out = np.zeros(int(cap), dtype=RECORD_DTYPE)
    if cap == 0:
        return out
    _check(lib.pyro_sw_moments(h, out.ctypes.data_as(ctypes.c_void_p), int(cap), ctypes.byref(n)),
           "pyro_sw_moments")
    return out[: n.value]


def pyro_sw_info(h):
    n, t = ctypes.c_int64(), ctypes.c_int64()
    _check(load_library().pyro_sw_info(h, ctypes.byref(n), ctypes.byref(t)), "pyro_sw_info")
    return n.value, t.value


def pyro_sw_get_spins(h, model) -> np.ndarray:
    N, _ = pyro_sw_info(h)
    out = np.zeros(N, np.int8) if model == PYRO_ISING else np.zeros((model, N), np.float32)
    _check(load_library().pyro_sw_get_spins(h, out.ctypes.data_as(ctypes.c_void_p), out.nbytes),
           "pyro_sw_get_spins")
    return out


def pyro_sw_set_spins(h, spins: np.ndarray, next_sweep: int):
    a = np.ascontiguousarray(spins)
    _check(load_library().pyro_sw_set_spins(h, a.ctypes.data_as(ctypes.c_void_p), a.nbytes, int(next_sweep)),
           "pyro_sw_set_spins")


def pyro_sw_get_labels(h) -> np.ndarray:
    N, _ = pyro_sw_info(h)
    out = np.zeros(N, np.int32)
    _check(load_library().pyro_sw_get_labels(h, out.ctypes.data_as(ctypes.c_void_p), N), "pyro_sw_get_labels")
    return out


def pyro_sw_set_temperature(h, T):
    _check(load_library().pyro_sw_set_temperature(h, float(T)), "pyro_sw_set_temperature")


def pyro_sw_set_timing(h, kernel_mask: int = -1):
    """Bracket launches of the selected kernels with HIP events (bit k =
    kernel k of pyro_sw_kernel_times; -1 all; 0 off)."""
    _check(load_library().pyro_sw_set_timing(h, int(kernel_mask)), "pyro_sw_set_timing")


def _kernel_times(fn, h, where) -> dict:
    cap = 32
    names = (ctypes.c_char_p * cap)()
    launches = (ctypes.c_int64 * cap)()
    ms = (ctypes.c_double * cap)()
    n = ctypes.c_int()
    _check(fn(h, names, launches, ms, cap, ctypes.byref(n)), where)
    return {names[k].decode(): (int(launches[k]), float(ms[k])) for k in range(n.value)}


def pyro_sw_kernel_times(h) -> dict:
    """{kernel name: (timed launches, total ms)} since the last set_timing."""
    return _kernel_times(load_library().pyro_sw_kernel_times, h, "pyro_sw_kernel_times")


def pyro_sw_set_tile_shape(h, shape: int):
    _check(load_library().pyro_sw_set_tile_shape(h, int(shape)), "pyro_sw_set_tile_shape")


def pyro_sw_group_create(handles, stream=None):
    arr = (ctypes.c_void_p * len(handles))(*[h.value for h in handles])
    g = ctypes.c_void_p()
    _check(load_library().pyro_sw_group_create(ctypes.byref(g), arr, len(handles), _stream_ptr(stream)),
           "pyro_sw_group_create")
    return g


def pyro_sw_group_sweep(g, n_sweeps, per_member=None):
    arr = None
    if per_member is not None:
        arr = (ctypes.c_int64 * len(per_member))(*[int(v) for v in per_member])
    _check(load_library().pyro_sw_group_sweep(g, int(n_sweeps), arr), "pyro_sw_group_sweep")


def pyro_sw_group_autotune(g, trial_sweeps=5):
    out = (ctypes.c_int * 3)()
    _check(load_library().pyro_sw_group_autotune(g, int(trial_sweeps), out), "pyro_sw_group_autotune")
    return list(out)


def pyro_sw_group_set_tile_shape(g, model, shape):
    _check(load_library().pyro_sw_group_set_tile_shape(g, int(model), int(shape)), "pyro_sw_group_set_tile_shape")


def pyro_sw_group_set_timing(g, kernel_mask: int = -1):
    _check(load_library().pyro_sw_group_set_timing(g, int(kernel_mask)), "pyro_sw_group_set_timing")


def pyro_sw_group_kernel_times(g) -> dict:
    return _kernel_times(load_library().pyro_sw_group_kernel_times, g, "pyro_sw_group_kernel_times")


def pyro_sw_group_set_slices(g, nslices: int):
    _check(load_library().pyro_sw_group_set_slices(g, int(nslices)), "pyro_sw_group_set_slices")


def pyro_sw_group_set_mode(g, ising_mode: int, resident: bool = False):
    _check(load_library().pyro_sw_group_set_mode(g, int(ising_mode), int(bool(resident))), "pyro_sw_group_set_mode")


def pyro_sw_group_get_mode(g):
    m, r = ctypes.c_int(), ctypes.c_int()
    _check(load_library().pyro_sw_group_get_mode(g, ctypes.byref(m), ctypes.byref(r)), "pyro_sw_group_get_mode")
    return m.value, bool(r.value)


def pyro_sw_group_set_counting(g, on: bool):
    _check(load_library().pyro_sw_group_set_counting(g, int(bool(on))), "pyro_sw_group_set_counting")


def pyro_sw_group_counts(g):
    """(compare-and-swaps the unite pass tried, those that hooked a root)."""
    a, b = ctypes.c_int64(), ctypes.c_int64()
    _check(load_library().pyro_sw_group_counts(g, ctypes.byref(a), ctypes.byref(b)), "pyro_sw_group_counts")
    return a.value, b.value


def pyro_sw_group_destroy(g):
    if g is not None and g.value:
        _check(load_library().pyro_sw_group_destroy(g), "pyro_sw_group_destroy")
        g.value = None


def pyro_sw_philox_rate(calls: int, repeats: int = 3, seed: int = 1):
    """Philox4x32-10 blocks per second on the current device, and the XOR fold
    of all output words of blocks (i, 0x5EED, BOND, 0), i < calls, key seed."""
    rate, fold = ctypes.c_double(), ctypes.c_uint32()
    _check(load_library().pyro_sw_philox_rate(int(calls), int(repeats), int(seed), ctypes.byref(rate),
                                              ctypes.byref(fold)), "pyro_sw_philox_rate")
    return rate.value, fold.value


def pyro_sw_sweep_static(dev_spins: int, L, model, T, J, seed, first_sweep, n_sweeps, dev_records: int,
                         stream=None):
    """Enqueue n_sweeps sweeps of the lattice whose spins are at device
    address dev_spins, records to device address dev_records (80 B each),
    using the library's static workspace (no allocation)."""
    _check(load_library().pyro_sw_sweep_static(int(dev_spins), int(L), int(model), float(T), float(J), int(seed),
                                               int(first_sweep), int(n_sweeps), int(dev_records),
                                               _stream_ptr(stream)), "pyro_sw_sweep_static")


def pyro_sw_atomic_rate(mode: int, words: int, ops: int, repeats: int = 3):
    """Device atomic operations per second (mode 0: load + compare-and-swap
    of random words of a `words`-word array; mode 1: adds to one word), the
    number of operations that took effect and the array's sum afterwards."""
    rate, ok, total = ctypes.c_double(), ctypes.c_int64(), ctypes.c_int64()
    _check(load_library().pyro_sw_atomic_rate(int(mode), int(words), int(ops), int(repeats), ctypes.byref(rate),
                                              ctypes.byref(ok), ctypes.byref(total)), "pyro_sw_atomic_rate")
    return rate.value, ok.value, total.value


def pyro_sw_destroy(h):
    if h is not None and h.value:
        _check(load_library().pyro_sw_destroy(h), "pyro_sw_destroy")
        h.value = None


class Lattice:
    """One simulated lattice whose device memory belongs to PyTorch tensors.

    The library enqueues all work on ``stream`` (default: PyTorch's current
    stream of ``device``)."""

    def __init__(self, L, model, T, J=1.0, seed=1, start=PYRO_START_RANDOM, device="cuda:0", stream=None):
        import torch

        load_library()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.L, self.model, self.T, self.J, self.seed, self.start = L, model, T, J, seed, start
        sb, wb = pyro_sw_workspace_size(L, model)
        with torch.cuda.device(self.device):
            self.spin_mem = torch.empty(sb, dtype=torch.uint8, device=self.device)
            self.work_mem = torch.empty(wb, dtype=torch.uint8, device=self.device)
        self.h = pyro_sw_init_ext(L, model, T, J, seed, start, self.stream, self.spin_mem.data_ptr(), sb,
                                  self.work_mem.data_ptr(), wb)
        self.N = 16 * L ** 3

    def sweep(self, n=1):
        pyro_sw_sweep(self.h, n)

    def moments(self, cap=None) -> np.ndarray:
        return pyro_sw_moments(self.h, cap)

    def spins(self) -> np.ndarray:
        return pyro_sw_get_spins(self.h, self.model)

    def set_spins(self, s, next_sweep):
        pyro_sw_set_spins(self.h, s, next_sweep)

    def labels(self) -> np.ndarray:
        return pyro_sw_get_labels(self.h)

    def set_temperature(self, T):
        self.T = T
        pyro_sw_set_temperature(self.h, T)

    @property
    def next_sweep(self) -> int:
        return pyro_sw_info(self.h)[1]

    def spins_tensor(self):
        """Device view of the spins (int8 [N] or float32 [n, N])."""
        import torch

        if self.model == PYRO_ISING:
            return self.spin_mem[: self.N].view(torch.int8)
        return self.spin_mem[: 4 * self.model * self.N].view(torch.float32).view(self.model, self.N)

    def set_tile_shape(self, shape):
        pyro_sw_set_tile_shape(self.h, shape)

    def close(self):
        if getattr(self, "h", None) is not None:
            pyro_sw_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Group:
    """Lattices swept together from one captured graph per sweep (the
    members keep their own records, spins and sweep indices)."""

    def __init__(self, lattices, stream=None):
        self.lattices = list(lattices)
        if stream is None and self.lattices:
            stream = self.lattices[0].stream
        self.stream = stream
        self.g = pyro_sw_group_create([lt.h for lt in self.lattices], stream)

    def sweep(self, n, per_member=None):
        pyro_sw_group_sweep(self.g, n, per_member)

    def autotune(self, trial_sweeps=5):
        return pyro_sw_group_autotune(self.g, trial_sweeps)

    def set_tile_shape(self, model, shape):
        pyro_sw_group_set_tile_shape(self.g, model, shape)

    def set_slices(self, nslices):
        pyro_sw_group_set_slices(self.g, nslices)

    def set_mode(self, ising_mode, resident=False):
        pyro_sw_group_set_mode(self.g, ising_mode, resident)

    def mode(self):
        """(Ising mode, LDS-resident small lattices)."""
        return pyro_sw_group_get_mode(self.g)

    def close(self):
        if getattr(self, "g", None) is not None:
            pyro_sw_group_destroy(self.g)
            self.g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ serving --

def _job_spec(job: dict) -> JobSpec:
    return JobSpec(model=int(job["model"]), L=int(job["L"]), T=float(job["T"]), J=float(job.get("J", 1.0)),
                   seed=int(job.get("seed", 1)), start=int(job.get("start", PYRO_START_RANDOM)),
                   keep_spins=int(bool(job.get("keep_spins", False))), sweeps=int(job["sweeps"]))


def pyro_sw_server_job_bytes(job: dict) -> int:
    b = ctypes.c_size_t()
    _check(load_library().pyro_sw_server_job_bytes(ctypes.byref(_job_spec(job)), ctypes.byref(b)),
           "pyro_sw_server_job_bytes")
    return b.value


def pyro_sw_server_create(hbm_budget: int, max_running: int = 64, quantum_ms: float = 20.0,
                          starve_ms: float = 2000.0):
    s = ctypes.c_void_p()
    _check(load_library().pyro_sw_server_create(ctypes.byref(s), int(hbm_budget), int(max_running),
                                                float(quantum_ms), float(starve_ms)), "pyro_sw_server_create")
    return s


def pyro_sw_server_submit(s, job: dict) -> int:
    jid = ctypes.c_int64()
    _check(load_library().pyro_sw_server_submit(s, ctypes.byref(_job_spec(job)), ctypes.byref(jid)),
           "pyro_sw_server_submit")
    return jid.value


def pyro_sw_server_step(s, wait_ms: float = 0.0):
    nq, nr = ctypes.c_int(), ctypes.c_int()
    _check(load_library().pyro_sw_server_step(s, float(wait_ms), ctypes.byref(nq), ctypes.byref(nr)),
           "pyro_sw_server_step")
    return nq.value, nr.value


def pyro_sw_server_status(s, job_id: int) -> dict:
    st = JobStatus()
    _check(load_library().pyro_sw_server_status(s, int(job_id), ctypes.byref(st)), "pyro_sw_server_status")
    return {name: getattr(st, name) for name, _ in JobStatus._fields_ if name != "reserved"}


def pyro_sw_server_take(s, job_id: int, spin_bytes: int = 0):
    """(records, spins bytes or None) of a finished job; the job is then forgotten."""
    lib = load_library()
    n = ctypes.c_int64()
    _check(lib.pyro_sw_server_take(s, int(job_id), None, 0, ctypes.byref(n), None, 0), "pyro_sw_server_take")
    out = np.zeros(max(n.value, 1), dtype=RECORD_DTYPE)
    spins = np.zeros(spin_bytes, dtype=np.uint8) if spin_bytes else None
    _check(lib.pyro_sw_server_take(s, int(job_id), out.ctypes.data, max(n.value, 1), ctypes.byref(n),
                                   spins.ctypes.data if spins is not None else None, int(spin_bytes)),
           "pyro_sw_server_take")
    return out[:n.value], spins


def pyro_sw_server_clock(s) -> float:
    t = ctypes.c_double()
    _check(load_library().pyro_sw_server_clock(s, ctypes.byref(t)), "pyro_sw_server_clock")
    return t.value


def pyro_sw_server_destroy(s):
    if s is not None and s.value:
        _check(load_library().pyro_sw_server_destroy(s), "pyro_sw_server_destroy")


class Server:
    """A job server (continuous batching over lanes of lattice groups)."""

    def __init__(self, hbm_budget: int, max_running: int = 64, quantum_ms: float = 20.0,
                 starve_ms: float = 2000.0):
        self.s = pyro_sw_server_create(hbm_budget, max_running, quantum_ms, starve_ms)

    def submit(self, job: dict) -> int:
        return pyro_sw_server_submit(self.s, job)

    def step(self, wait_ms: float = 0.0):
        return pyro_sw_server_step(self.s, wait_ms)

    def status(self, job_id: int) -> dict:
        return pyro_sw_server_status(self.s, job_id)

    def take(self, job_id: int, spin_bytes: int = 0):
        return pyro_sw_server_take(self.s, job_id, spin_bytes)

    def clock(self) -> float:
        return pyro_sw_server_clock(self.s)

    def close(self):
        if getattr(self, "s", None) is not None:
            pyro_sw_server_destroy(self.s)
            self.s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------- graphs --


def pyro_sw_bonds(L: int):
    """Pyrochlore bond table of edge L: (bond_a, bond_b), int32 [48 L^3]."""
    n = 48 * int(L) ** 3
    a = np.zeros(n, np.int32)
    b = np.zeros(n, np.int32)
    _check(load_library().pyro_sw_bonds(int(L), a.ctypes.data_as(ctypes.c_void_p),
                                        b.ctypes.data_as(ctypes.c_void_p), n), "pyro_sw_bonds")
    return a, b


def simple_cubic_bonds(L: int):
    """Simple-cubic bond table of edge L, periodic (pyro_sw_sc_bonds): site
    (z L + y) L + x, bond 3 i + d to its +x, +y, +z neighbour (d = 0, 1, 2)."""
    n = 3 * int(L) ** 3
    a = np.zeros(n, np.int32)
    b = np.zeros(n, np.int32)
    _check(load_library().pyro_sw_sc_bonds(int(L), a.ctypes.data_as(ctypes.c_void_p),
                                           b.ctypes.data_as(ctypes.c_void_p), n), "pyro_sw_sc_bonds")
    return a, b


class Graph:
    """One lattice given by its bond table, swept by the generic graph path
    (any nearest-neighbour table; see pyro_sw_graph_init)."""

    def __init__(self, bonds, n_sites, model, T, J=1.0, seed=1, start=PYRO_START_RANDOM, device="cuda:0",
                 stream=None):
        import torch

        lib = load_library()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        a = np.ascontiguousarray(bonds[0], dtype=np.int32)
        b = np.ascontiguousarray(bonds[1], dtype=np.int32)
        if a.shape != b.shape:
            raise ValueError("bond arrays differ in length")
        self.model, self.N, self.NB = model, int(n_sites), len(a)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib.pyro_sw_graph_init(ctypes.byref(h), self.N, self.NB, a.ctypes.data_as(ctypes.c_void_p),
                                          b.ctypes.data_as(ctypes.c_void_p), int(model), float(T), float(J),
                                          int(seed), int(start), _stream_ptr(self.stream)),
                   "pyro_sw_graph_init")
        self.g = h

    def sweep(self, n=1):
        _check(load_library().pyro_sw_graph_sweep(self.g, int(n)), "pyro_sw_graph_sweep")

    def moments(self) -> np.ndarray:
        lib = load_library()
        n = ctypes.c_int64()
        _check(lib.pyro_sw_graph_moments(self.g, None, 0, ctypes.byref(n)), "pyro_sw_graph_moments")
        out = np.zeros(n.value, dtype=RECORD_DTYPE)
        if n.value:
            _check(lib.pyro_sw_graph_moments(self.g, out.ctypes.data_as(ctypes.c_void_p), n.value,
                                             ctypes.byref(n)), "pyro_sw_graph_moments")
        return out[: n.value]

    def spins(self) -> np.ndarray:
        out = np.zeros(self.N, np.int8) if self.model == PYRO_ISING else np.zeros((self.model, self.N), np.float32)
        _check(load_library().pyro_sw_graph_get_spins(self.g, out.ctypes.data_as(ctypes.c_void_p), out.nbytes),
               "pyro_sw_graph_get_spins")
        return out

    def set_spins(self, s, next_sweep):
        a = np.ascontiguousarray(s)
        _check(load_library().pyro_sw_graph_set_spins(self.g, a.ctypes.data_as(ctypes.c_void_p), a.nbytes,
                                                      int(next_sweep)), "pyro_sw_graph_set_spins")

    def labels(self) -> np.ndarray:
        out = np.zeros(self.N, np.int32)
        _check(load_library().pyro_sw_graph_get_labels(self.g, out.ctypes.data_as(ctypes.c_void_p), self.N),
               "pyro_sw_graph_get_labels")
        return out

    def set_temperature(self, T):
        _check(load_library().pyro_sw_graph_set_temperature(self.g, float(T)), "pyro_sw_graph_set_temperature")

    def close(self):
        if getattr(self, "g", None) is not None:
            pyro_sw_graph_destroy(self.g)
            self.g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pyro_sw_graph_destroy(g):
    _check(load_library().pyro_sw_graph_destroy(g), "pyro_sw_graph_destroy")
