"""ctypes binding of the C oracle (test infrastructure only).

Every function here only marshals numpy arrays into ``liboracle.so``; the
arithmetic lives in ``oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")


class Geom(C.Structure):
    _fields_ = [
        ("L", C.c_double * 3),
        ("halfL", C.c_double * 3),
        ("l", C.c_double * 3),
        ("inv_l", C.c_double * 3),
        ("rc", C.c_double),
        ("rc2", C.c_double),
        ("uc", C.c_double),
        ("S", C.c_int),
        ("ncx", C.c_int),
        ("G", C.c_int * 3),
        ("cells_per_slice", C.c_int64),
        ("ncell", C.c_int64),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int64)
        i32p = C.POINTER(C.c_int32)
        gp = C.POINTER(Geom)
        L.oracle_geometry.argtypes = [dp, C.c_int, C.c_double, gp]
        L.oracle_bin.argtypes = [gp, C.c_int64, dp, i32p, i32p, ip]
        L.oracle_bin.restype = None
        L.oracle_pair.argtypes = [gp, dp, dp, dp, dp, dp, dp, dp]
        L.oracle_forces_brute.argtypes = [gp, C.c_int64, dp, dp, dp, dp, ip]
        L.oracle_forces_cells.argtypes = [gp, C.c_int64, dp, dp, dp, dp, dp, ip, ip]
        L.oracle_forces_subset.argtypes = [gp, C.c_int64, dp, C.c_int64, ip, dp, dp, ip, ip]
        L.oracle_energy.argtypes = [gp, C.c_int64, dp, dp, dp, dp, dp]
        L.oracle_run.argtypes = [gp, C.c_int64, dp, dp, dp, C.c_double, C.c_int64, C.c_int64,
                                 dp, ip, i32p, ip]
        L.oracle_run_nvt.argtypes = [gp, C.c_int64, dp, dp, dp, C.c_double, C.c_int64, C.c_double,
                                     C.c_int64, dp, ip, i32p, ip]
        L.oracle_slice_scale.argtypes = [gp, C.c_int64, dp, dp, C.c_double, dp]
        L.oracle_set_threads.argtypes = [C.c_int]
        L.oracle_set_threads.restype = None
        L.oracle_get_threads.restype = C.c_int
        _lib = L
    return _lib


def _p(a, t=C.c_double):
    return None if a is None else a.ctypes.data_as(C.POINTER(t))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle returned {code}")
        self.code = code


def _check(rc):
    if rc != 0:
        raise OracleError(rc)


def geometry(box, slices, rc=2.5) -> Geom:
    g = Geom()
    b = _f64(box)
    _check(lib().oracle_geometry(_p(b), int(slices), float(rc), C.byref(g)))
    return g


def set_threads(n: int):
    lib().oracle_set_threads(int(n))


def get_threads() -> int:
    return lib().oracle_get_threads()


def bin_atoms(g: Geom, pos):
    pos = _f64(pos, (-1, 3))
    n = len(pos)
    gxyz = np.zeros((n, 3), np.int32)
    sl = np.zeros(n, np.int32)
    cell = np.zeros(n, np.int64)
    lib().oracle_bin(C.byref(g), n, _p(pos), _p(gxyz, C.c_int32), _p(sl, C.c_int32),
                     _p(cell, C.c_int64))
    return gxyz, sl, cell


def pair(g: Geom, ri, rj):
    ri = _f64(ri)
    rj = _f64(rj)
    f = np.zeros(3)
    u, w, s, r2 = C.c_double(), C.c_double(), C.c_double(), C.c_double()
    inr = lib().oracle_pair(C.byref(g), _p(ri), _p(rj), _p(f), C.byref(u), C.byref(w),
                            C.byref(s), C.byref(r2))
    return bool(inr), f, u.value, w.value, s.value, r2.value


def forces_brute(g: Geom, pos):
    pos = _f64(pos, (-1, 3))
    n = len(pos)
    F = np.zeros((n, 3))
    U, W, P = C.c_double(), C.c_double(), C.c_int64()
    _check(lib().oracle_forces_brute(C.byref(g), n, _p(pos), _p(F), C.byref(U), C.byref(W),
                                     C.byref(P)))
    return F, U.value, W.value, P.value


def forces_cells(g: Geom, pos):
    """Returns dict with F, u_half, w_half, scale, cand, inr (per atom)."""
    pos = _f64(pos, (-1, 3))
    n = len(pos)
    out = {"F": np.zeros((n, 3)), "u_half": np.zeros(n), "w_half": np.zeros(n),
           "scale": np.zeros(n), "cand": np.zeros(n, np.int64), "inr": np.zeros(n, np.int64)}
    _check(lib().oracle_forces_cells(C.byref(g), n, _p(pos), _p(out["F"]), _p(out["u_half"]),
                                     _p(out["w_half"]), _p(out["scale"]),
                                     _p(out["cand"], C.c_int64), _p(out["inr"], C.c_int64)))
    return out


def forces_subset(g: Geom, pos, ids):
    pos = _f64(pos, (-1, 3))
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    m = len(ids)
    out = {"F": np.zeros((m, 3)), "scale": np.zeros(m), "cand": np.zeros(m, np.int64),
           "inr": np.zeros(m, np.int64)}
    _check(lib().oracle_forces_subset(C.byref(g), len(pos), _p(pos), m, _p(ids, C.c_int64),
                                      _p(out["F"]), _p(out["scale"]),
                                      _p(out["cand"], C.c_int64), _p(out["inr"], C.c_int64)))
    return out


def energy(g: Geom, pos, vel):
    pos = _f64(pos, (-1, 3))
    vel = _f64(vel, (-1, 3))
    U, K, W = C.c_double(), C.c_double(), C.c_double()
    _check(lib().oracle_energy(C.byref(g), len(pos), _p(pos), _p(vel), C.byref(U), C.byref(K),
                               C.byref(W)))
    return U.value, K.value, W.value


def run(g: Geom, pos, vel, dt, nsteps, every=0, miglog=False, check=True, thermostat=None):
    """Trajectory from {pos, vel}.  Returns dict(pos, vel, F, elog[t,U,K,W], miglog, status).
    thermostat=T0 runs under the per-slice velocity-scaling thermostat."""
    pos = _f64(pos, (-1, 3)).copy()
    vel = _f64(vel, (-1, 3)).copy()
    n = len(pos)
    F = np.zeros((n, 3))
    cap = (nsteps // every + 1) if every > 0 else 0
    elog = np.zeros((max(cap, 1), 4))
    mig = np.zeros((max(nsteps, 1), g.S, 2), np.int32) if miglog else None
    ns, done = C.c_int64(), C.c_int64()
    if thermostat is None:
        rc = lib().oracle_run(C.byref(g), n, _p(pos), _p(vel), _p(F), float(dt), int(nsteps),
                              int(every), _p(elog), C.byref(ns), _p(mig, C.c_int32),
                              C.byref(done))
    else:
        rc = lib().oracle_run_nvt(C.byref(g), n, _p(pos), _p(vel), _p(F), float(dt), int(nsteps),
                                  float(thermostat), int(every), _p(elog), C.byref(ns),
                                  _p(mig, C.c_int32), C.byref(done))
    if check:
        _check(rc)
    return {"pos": pos, "vel": vel, "F": F, "elog": elog[: ns.value],
            "miglog": None if mig is None else mig[:nsteps], "status": rc,
            "steps_done": done.value}


def slice_scale(g: Geom, pos, vel, T0):
    """One per-slice thermostat scaling.  Returns (scaled velocities, lambda[S])."""
    pos = _f64(pos, (-1, 3))
    vel = _f64(vel, (-1, 3)).copy()
    lam = np.zeros(g.S)
    _check(lib().oracle_slice_scale(C.byref(g), len(pos), _p(pos), _p(vel), float(T0), _p(lam)))
    return vel, lam


def force_error(F_test, F_ref, scale):
    """Normalised per-atom force error e_i = |F_test - F_ref| / S_i, where S_i sums the
    magnitudes of atom i's pair-force terms; atoms without in-range pairs must have
    F_test exactly 0 (reported as inf otherwise)."""
    F_test = np.asarray(F_test, dtype=np.float64).reshape(-1, 3)
    F_ref = np.asarray(F_ref, dtype=np.float64).reshape(-1, 3)
    d = np.linalg.norm(F_test - F_ref, axis=1)
    scale = np.asarray(scale, dtype=np.float64)
    e = np.zeros_like(d)
    nz = scale > 0
    e[nz] = d[nz] / scale[nz]
    # no partner: the force must be exactly zero (compared component by component: the
    # norm of a tiny difference can underflow to 0)
    exact = (F_test[~nz] == F_ref[~nz]).all(axis=1)
    e[~nz] = np.where(exact, 0.0, np.inf)
    return e
