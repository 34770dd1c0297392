"""ctypes binding of ``libmd.so`` (the C ABI declared in ``include/md.h``).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Importing this module fails loudly when the library is not built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmd.so")

MD_OK, MD_PENDING = 0, 1
MD_EINVAL, MD_ENOMEM, MD_EHIP, MD_ESTATE = -1, -2, -3, -4
MD_ECAPACITY, MD_EUNSTABLE, MD_ENOTFOUND, MD_EBUSY, MD_EWATCHDOG = -5, -6, -7, -8, -9
MD_FP64, MD_FP32_FORCE = 0, 1
OPT_ENERGY_EVERY, OPT_CLAIM_ORDER, OPT_ORDER_SEED, OPT_MIGRATION_LOG = 1, 2, 3, 4
OPT_CHUNK_CELLS, OPT_COUNT_PAIRS, OPT_WATCHDOG_MS, OPT_GRID = 5, 6, 7, 8
OPT_FAIL_AT_STEP, OPT_MAX_STEPS_PER_LAUNCH, OPT_TRACE, OPT_CELL_CAPACITY = 9, 10, 11, 12
OPT_XCD_QUEUES, OPT_WAVEFRONT_LEVELS = 13, 14
ORDER_SWEEP, ORDER_PHASED, ORDER_DESCENDING, ORDER_RANDOM, ORDER_DATAFLOW, ORDER_WAVEFRONT = 0, 1, 2, 3, 4, 5
SERVER_FAKE_EXECUTOR = 1
SERVER_MAX_QUEUED = 4096
NOALLOC_SCRATCH_BYTES = 16 << 20

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class md_stats(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("n", C.c_int64), ("slices", C.c_int32), ("ncx", C.c_int32),
        ("grid", C.c_int32 * 3), ("cell_capacity", C.c_int32), ("ncell", C.c_int64),
        ("migrations_left", C.c_int64), ("migrations_right", C.c_int64),
        ("candidates", C.c_int64), ("in_range", C.c_int64), ("counted_steps", C.c_int64),
        ("last_step_seconds", C.c_double), ("last_kernel_seconds", C.c_double),
        ("last_launches", C.c_int32), ("persistent_grid", C.c_int32),
        ("chunks_per_slice", C.c_int32), ("precision", C.c_int32), ("poisoned", C.c_int32),
        ("work_queues", C.c_int32), ("queue_first", C.c_int32 * 9),
    ]


class md_trace_rec(C.Structure):
    _fields_ = [("k", C.c_uint32), ("slice", C.c_uint32), ("chunk", C.c_uint32), ("phase", C.c_uint32),
                ("hw_id", C.c_uint32), ("launch", C.c_uint32), ("xcd", C.c_uint32), ("queue", C.c_uint32),
                ("t_claim", C.c_uint64), ("t_ready", C.c_uint64), ("t_done", C.c_uint64)]


TRACE_DTYPE = np.dtype([("k", "<u4"), ("slice", "<u4"), ("chunk", "<u4"), ("phase", "<u4"),
                        ("hw_id", "<u4"), ("launch", "<u4"), ("xcd", "<u4"), ("queue", "<u4"),
                        ("t_claim", "<u8"), ("t_ready", "<u8"), ("t_done", "<u8")])


class md_run_desc(C.Structure):
    _fields_ = [
        ("box", C.c_double * 3), ("slices", C.c_int32), ("rc", C.c_double), ("dt", C.c_double),
        ("precision", C.c_int32), ("n", C.c_int64), ("pos", C.POINTER(C.c_double)),
        ("vel", C.POINTER(C.c_double)), ("steps", C.c_int64), ("energy_every", C.c_int64),
        ("tag", C.c_uint64), ("keep_state", C.c_int32),
    ]


class md_result(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("steps_done", C.c_int64), ("tag", C.c_uint64),
        ("U0", C.c_double), ("K0", C.c_double), ("W0", C.c_double),
        ("U1", C.c_double), ("K1", C.c_double), ("W1", C.c_double),
        ("drift_per_atom_step", C.c_double),
        ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double),
    ]


_lib = None

_SIGS = {
    "md_init": ([C.POINTER(C.c_double), C.c_int, C.c_double, C.c_double, C.c_int, C.POINTER(C.c_void_p)], C.c_int),
    "md_load": ([C.c_void_p, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_double)], C.c_int),
    "md_step": ([C.c_void_p, C.c_int64], C.c_int),
    "md_step_noalloc": ([C.c_void_p, C.c_int64], C.c_int),
    "md_energy_virial": ([C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)], C.c_int),
    "md_get_state": ([C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)], C.c_int),
    "md_get_cells": ([C.c_void_p, C.POINTER(C.c_int64)], C.c_int),
    "md_get_slice_counts": ([C.c_void_p, C.POINTER(C.c_int64)], C.c_int),
    "md_get_energy_log": ([C.c_void_p, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_int64)], C.c_int),
    "md_get_migration_log": ([C.c_void_p, C.c_int64, C.POINTER(C.c_int32), C.POINTER(C.c_int64)], C.c_int),
    "md_get_stats": ([C.c_void_p, C.POINTER(md_stats)], C.c_int),
    "md_get_trace": ([C.c_void_p, C.c_int64, C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_double)], C.c_int),
    "md_set_option": ([C.c_void_p, C.c_int, C.c_int64], C.c_int),
    "md_set_thermostat": ([C.c_void_p, C.c_double], C.c_int),
    "md_set_stream": ([C.c_void_p, C.c_void_p], C.c_int),
    "md_free": ([C.c_void_p], None),
    "md_strerror": ([C.c_int], C.c_char_p),
    "md_last_error": ([], C.c_char_p),
    "md_footprint_bytes": ([C.POINTER(C.c_double), C.c_int, C.c_double, C.c_int64], C.c_int64),
    "md_claim_table": ([C.c_int, C.c_int, C.c_uint64, C.POINTER(C.c_uint16)], C.c_int),
    "md_wavefront_table": ([C.c_int, C.c_int, C.POINTER(C.c_uint32)], C.c_int),
    "md_server_create": ([C.c_size_t, C.c_int, C.POINTER(C.c_void_p)], C.c_int),
    "md_server_create_ex": ([C.c_size_t, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_void_p)], C.c_int),
    "md_submit": ([C.c_void_p, C.POINTER(md_run_desc), C.POINTER(C.c_uint64)], C.c_int),
    "md_poll": ([C.c_void_p, C.c_uint64, C.POINTER(md_result)], C.c_int),
    "md_fetch_state": ([C.c_void_p, C.c_uint64, C.POINTER(C.c_double), C.POINTER(C.c_double)], C.c_int),
    "md_server_stats": ([C.c_void_p] + [C.POINTER(C.c_int64)] * 5, C.c_int),
    "md_server_times": ([C.c_void_p] + [C.POINTER(C.c_double)] * 4, C.c_int),
    "md_server_destroy": ([C.c_void_p], C.c_int),
    "md_set_allocator": ([ALLOC_FN, FREE_FN, C.c_void_p], C.c_int),
}

EXPORTED = tuple(_SIGS)


def lib():
    """The loaded library; raises if it was not built (there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "or python -m paper_2507_11289_amd.build")
        # One HIP runtime per process: torch ships its own copy of the HIP runtime, and a
        # library loaded before torch binds to the system copy, after which torch finds no
        # GPU.  Loaded after torch, libmd binds to torch's copy (same soname), so device
        # memory and streams can pass between the two (md_set_stream, md_set_allocator).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


class MDError(RuntimeError):
    def __init__(self, code, where=""):
        msg = lib().md_last_error().decode(errors="replace")
        super().__init__(f"{where}: {lib().md_strerror(code).decode()} ({code}): {msg}")
        self.code = code


def _check(code, where):
    if code < 0:
        raise MDError(code, where)
    return code


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1, 3)
    return a


def md_strerror(code: int) -> str:
    return lib().md_strerror(code).decode()


def md_footprint_bytes(box, slices, rc, n) -> int:
    b = (C.c_double * 3)(*box)
    return lib().md_footprint_bytes(b, int(slices), float(rc), int(n))


def md_claim_table(slices: int, order: int, seed: int = 1) -> np.ndarray:
    """Per-step claim table as (phase, slice) pairs, shape (2*slices, 2)."""
    t = np.zeros(2 * slices, np.uint16)
    _check(lib().md_claim_table(int(slices), int(order), int(seed), t.ctypes.data_as(C.POINTER(C.c_uint16))),
           "md_claim_table")
    return np.stack([t >> 15, t & 0x7FFF], axis=1).astype(np.int64)


def md_wavefront_table(slices: int, levels: int) -> np.ndarray:
    """Claim table of MD_ORDER_WAVEFRONT as (step, phase, slice) rows, shape (2*slices*levels, 3)."""
    t = np.zeros(2 * slices * levels, np.uint32)
    _check(lib().md_wavefront_table(int(slices), int(levels), t.ctypes.data_as(C.POINTER(C.c_uint32))),
           "md_wavefront_table")
    return np.stack([t >> 16, (t >> 15) & 1, t & 0x7FFF], axis=1).astype(np.int64)


_allocator_refs = None


def set_allocator(alloc=None, release=None):
    """md_set_allocator with Python callables alloc(bytes) -> int address and
    release(address); None, None returns to hipMalloc / hipFree."""
    global _allocator_refs
    if alloc is None and release is None:
        _check(lib().md_set_allocator(ALLOC_FN(), FREE_FN(), None), "md_set_allocator")
        _allocator_refs = None
        return
    a = ALLOC_FN(lambda nbytes, ctx: alloc(int(nbytes)) or None)
    f = FREE_FN(lambda ptr, ctx: release(int(ptr)))
    _check(lib().md_set_allocator(a, f, None), "md_set_allocator")
    _allocator_refs = (a, f)  # the library keeps calling them: keep them alive


def use_torch_allocator():
    """Back every later device allocation of the library with torch's caching allocator
    on the current device."""
    import torch

    set_allocator(lambda n: torch.cuda.caching_allocator_alloc(n),
                  lambda p: torch.cuda.caching_allocator_delete(p))


class Sim:
    """One simulation handle (md_init ... md_free)."""

    def __init__(self, box, slices, rc=2.5, dt=0.005, precision=MD_FP64):
        self.box = tuple(float(x) for x in box)
        h = C.c_void_p()
        b = (C.c_double * 3)(*self.box)
        _check(lib().md_init(b, int(slices), float(rc), float(dt), int(precision), C.byref(h)), "md_init")
        self._h = h
        self.n = 0
        self.slices = int(slices)

    def close(self):
        if getattr(self, "_h", None):
            lib().md_free(self._h)
            self._h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # --- calls of the ABI -------------------------------------------------
    def load(self, pos, vel):
        pos = _f64(pos)
        vel = _f64(vel)
        if pos.shape != vel.shape:
            raise ValueError("pos and vel differ in shape")
        _check(lib().md_load(self._h, len(pos), _dp(pos), _dp(vel)), "md_load")
        self.n = len(pos)

    def step(self, nsteps: int) -> int:
        return _check(lib().md_step(self._h, int(nsteps)), "md_step")

    def step_noalloc(self, nsteps: int) -> int:
        """md_step_noalloc: md_step without device allocation (fixed per-GPU scratch)."""
        return _check(lib().md_step_noalloc(self._h, int(nsteps)), "md_step_noalloc")

    def step_rc(self, nsteps: int) -> int:
        """md_step returning the status code instead of raising."""
        return lib().md_step(self._h, int(nsteps))

    def energy_virial(self):
        U, K, W = C.c_double(), C.c_double(), C.c_double()
        _check(lib().md_energy_virial(self._h, C.byref(U), C.byref(K), C.byref(W)), "md_energy_virial")
        return U.value, K.value, W.value

    def state(self):
        pos = np.zeros((self.n, 3))
        vel = np.zeros((self.n, 3))
        force = np.zeros((self.n, 3))
        _check(lib().md_get_state(self._h, _dp(pos), _dp(vel), _dp(force)), "md_get_state")
        return pos, vel, force

    def cells(self):
        c = np.zeros(self.n, np.int64)
        _check(lib().md_get_cells(self._h, c.ctypes.data_as(C.POINTER(C.c_int64))), "md_get_cells")
        return c

    def slice_counts(self):
        c = np.zeros(self.slices, np.int64)
        _check(lib().md_get_slice_counts(self._h, c.ctypes.data_as(C.POINTER(C.c_int64))), "md_get_slice_counts")
        return c

    def energy_log(self):
        cnt = C.c_int64()
        _check(lib().md_get_energy_log(self._h, 0, None, C.byref(cnt)), "md_get_energy_log")
        rows = np.zeros((max(cnt.value, 1), 4))
        _check(lib().md_get_energy_log(self._h, cnt.value, _dp(rows), C.byref(cnt)), "md_get_energy_log")
        return rows[: cnt.value]

    def migration_log(self):
        steps = C.c_int64()
        _check(lib().md_get_migration_log(self._h, 0, None, C.byref(steps)), "md_get_migration_log")
        log = np.zeros((max(steps.value, 1), self.slices, 2), np.int32)
        _check(lib().md_get_migration_log(self._h, steps.value, log.ctypes.data_as(C.POINTER(C.c_int32)),
                                          C.byref(steps)), "md_get_migration_log")
        return log[: steps.value]

    def trace(self):
        """(records as a numpy structured array, device clock rate in Hz)."""
        cnt, hz = C.c_int64(), C.c_double()
        _check(lib().md_get_trace(self._h, 0, None, C.byref(cnt), C.byref(hz)), "md_get_trace")
        rec = np.zeros(cnt.value, TRACE_DTYPE)
        _check(lib().md_get_trace(self._h, cnt.value, rec.ctypes.data_as(C.c_void_p), C.byref(cnt),
                                  C.byref(hz)), "md_get_trace")
        return rec, hz.value

    def stats(self) -> md_stats:
        st = md_stats()
        _check(lib().md_get_stats(self._h, C.byref(st)), "md_get_stats")
        return st

    def set_option(self, key: int, value: int):
        _check(lib().md_set_option(self._h, int(key), int(value)), "md_set_option")

    def set_thermostat(self, temperature: float):
        """Per-slice velocity-scaling thermostat at `temperature` (0 switches it off)."""
        _check(lib().md_set_thermostat(self._h, float(temperature)), "md_set_thermostat")

    def set_stream(self, stream_handle):
        _check(lib().md_set_stream(self._h, C.c_void_p(stream_handle)), "md_set_stream")


class Server:
    """Serving engine handle (md_server_create ... md_server_destroy)."""

    def __init__(self, budget_bytes: int, max_runs: int, quantum_steps: int = 0, flags: int = 0):
        h = C.c_void_p()
        _check(lib().md_server_create_ex(int(budget_bytes), int(max_runs), int(quantum_steps), int(flags),
                                         C.byref(h)), "md_server_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().md_server_destroy(self._h)
            self._h = None

    __del__ = close

    def submit(self, box, slices, pos, vel, steps, rc=2.5, dt=0.005, precision=MD_FP32_FORCE,
               energy_every=0, tag=0, keep_state=False) -> int:
        pos = _f64(pos)
        vel = _f64(vel)
        d = md_run_desc()
        for k in range(3):
            d.box[k] = float(box[k])
        d.slices, d.rc, d.dt, d.precision = int(slices), float(rc), float(dt), int(precision)
        d.n = len(pos)
        d.pos, d.vel = _dp(pos), _dp(vel)
        d.steps, d.energy_every, d.tag, d.keep_state = int(steps), int(energy_every), int(tag), int(keep_state)
        t = C.c_uint64()
        _check(lib().md_submit(self._h, C.byref(d), C.byref(t)), "md_submit")
        return t.value

    def poll(self, ticket: int):
        """(status, md_result or None)."""
        r = md_result()
        rc = lib().md_poll(self._h, C.c_uint64(ticket), C.byref(r))
        if rc == MD_PENDING:
            return rc, None
        if rc == MD_ENOTFOUND:
            raise MDError(rc, "md_poll")
        return rc, r

    def fetch_state(self, ticket: int, n: int):
        pos = np.zeros((n, 3))
        vel = np.zeros((n, 3))
        _check(lib().md_fetch_state(self._h, C.c_uint64(ticket), _dp(pos), _dp(vel)), "md_fetch_state")
        return pos, vel

    def times(self):
        """Seconds the server thread spent admitting, launching, completing and idle."""
        v = [C.c_double() for _ in range(4)]
        _check(lib().md_server_times(self._h, *[C.byref(x) for x in v]), "md_server_times")
        return dict(zip(("admit_s", "launch_s", "finish_s", "idle_s"), [x.value for x in v]))

    def stats(self):
        v = [C.c_int64() for _ in range(5)]
        _check(lib().md_server_stats(self._h, *[C.byref(x) for x in v]), "md_server_stats")
        return dict(zip(("queued", "running", "done", "bytes_in_use", "launches"), [x.value for x in v]))
