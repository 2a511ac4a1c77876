"""FP64 CPU oracle of the 3DPIFCM IFCM iteration -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The product library never calls it and
shares no code with it.  This module only marshals numpy arrays into the C
functions of pifcm_oracle.c (see that file for the equations and readings).
"""
from __future__ import annotations

import ctypes as ct
import os
from dataclasses import dataclass

import numpy as np

from .build import LIB, build

OR_SHELL_SQDIST = 1
OR_Q2_SQDIST = 2


class _Params(ct.Structure):
    _fields_ = [("C", ct.c_int32), ("V", ct.c_int32), ("max_iter", ct.c_int32),
                ("flags", ct.c_int32), ("m", ct.c_double), ("h", ct.c_double),
                ("eps", ct.c_double)]


@dataclass
class Params:
    C: int = 4
    m: float = 2.0
    V: int = 1
    h: float = 1.0
    eps: float = 1e-5
    max_iter: int = 50
    flags: int = 0

    def c(self):
        return _Params(self.C, self.V, self.max_iter, self.flags, self.m, self.h, self.eps)


_lib = None


def lib():
    """The oracle library: oracle/liboracle.so (built on first use), or the
    build that PIFCM_ORACLE_LIB names (the tests' mutation check loads
    deliberately broken copies this way)."""
    global _lib
    if _lib is None:
        path = os.environ.get("PIFCM_ORACLE_LIB", "") or LIB
        if path == LIB and not os.path.exists(LIB):
            build()
        _lib = ct.CDLL(path)
        d, i, f = ct.POINTER(ct.c_double), ct.c_int, ct.POINTER(ct.c_float)
        pp = ct.POINTER(_Params)
        i64 = ct.c_int64
        _lib.oracle_normalize.argtypes = [f, i64, f]
        _lib.oracle_init_memberships.argtypes = [f, i64, pp, d, d]
        _lib.oracle_step.argtypes = [f, i, i, i, pp, ct.c_double, ct.c_double, d, d, d, d, d, d, d]
        _lib.oracle_solve.argtypes = [f, i, i, i, pp, ct.c_double, ct.c_double, d, d, d, d, d,
                                      ct.POINTER(ct.c_int32), d]
        _lib.oracle_solve_slab.argtypes = [f, i, i, i, i, i, pp, ct.c_double, ct.c_double, d, d,
                                           d, d, d, ct.POINTER(ct.c_int32), d]
        _lib.oracle_fcm_init.argtypes = [f, i, i, i, pp, d, d, ct.POINTER(ct.c_int32)]
        _lib.oracle_labels.argtypes = [d, i64, i, ct.POINTER(ct.c_uint8)]
        _lib.oracle_pso.argtypes = [f, i, i, i, pp, d, d, i, i, d, d, d, d, ct.c_double,
                                    ct.c_double, ct.c_double, d, d, d, d]
        _lib.oracle_pso_interleaved.argtypes = [f, i, i, i, pp, d, d, i, i, i, d, d, d, d,
                                                ct.c_double, ct.c_double, ct.c_double, d, d, d,
                                                d, d, d]
        _lib.oracle_fd_grad.argtypes = [f, i, i, i, pp, ct.c_double, ct.c_double, d, d, i,
                                        ct.c_double, d, d]
        _lib.oracle_set_threads.argtypes = [i]
    return _lib


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _pf(a):
    return a.ctypes.data_as(ct.POINTER(ct.c_float))


def _pd(a):
    return None if a is None else a.ctypes.data_as(ct.POINTER(ct.c_double))


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with status {rc}")


def set_threads(n: int) -> int:
    return lib().oracle_set_threads(int(n))


def get_threads() -> int:
    return lib().oracle_get_threads()


def normalize(raw):
    """Algorithm 2 step 1: min-max normalisation in FP64, rounded to fp32."""
    raw = _f32(raw)
    out = np.empty_like(raw)
    _check(lib().oracle_normalize(_pf(raw), raw.size, _pf(out)), "normalize")
    return out


def init_memberships(x, c, p: Params):
    x = _f32(x)
    U = np.empty((x.size, p.C), np.float64)
    c = _f64(c)
    _check(lib().oracle_init_memberships(_pf(x), x.size, ct.byref(p.c()), _pd(c), _pd(U)),
           "init_memberships")
    return U


def step(x, U, c, p: Params, lam, xi, want_hf=False):
    """One IFCM step.  x: (Z, Y, X) float32; U: (N, C).  Returns
    (U_new, c_new, J_of_input_state[, H, F])."""
    x = _f32(x)
    nz, ny, nx = x.shape
    U = _f64(U).reshape(-1, p.C)
    c = _f64(c)
    Un = np.empty_like(U)
    cn = np.empty(p.C)
    J = ct.c_double()
    H = np.empty_like(U) if want_hf else None
    F = np.empty_like(U) if want_hf else None
    _check(lib().oracle_step(_pf(x), nx, ny, nz, ct.byref(p.c()), float(lam), float(xi),
                             _pd(U), _pd(c), _pd(Un), _pd(cn), ct.byref(J), _pd(H), _pd(F)),
           "step")
    if want_hf:
        return Un, cn, J.value, H, F
    return Un, cn, J.value


def solve(x, c0, p: Params, lam, xi, U0=None, want_hist=False):
    """IFCM solve.  Returns dict(U, c, J, iters[, J_hist])."""
    x = _f32(x)
    nz, ny, nx = x.shape
    c0 = _f64(c0)
    U0a = None if U0 is None else _f64(U0).reshape(-1, p.C)
    U = np.empty((x.size, p.C))
    c = np.empty(p.C)
    J = ct.c_double()
    it = ct.c_int32()
    hist = np.zeros(max(p.max_iter, 1)) if want_hist else None
    _check(lib().oracle_solve(_pf(x), nx, ny, nz, ct.byref(p.c()), float(lam), float(xi),
                              _pd(c0), _pd(U0a), _pd(U), _pd(c), ct.byref(J), ct.byref(it),
                              _pd(hist)), "solve")
    out = dict(U=U, c=c, J=J.value, iters=it.value)
    if want_hist:
        out["J_hist"] = hist[: it.value]
    return out


def solve_slab(x, c0, p: Params, lam, xi, U0, zbeg, zend, want_hist=False):
    """IFCM solve of the planes [zbeg, zend) only, the other planes' memberships
    held at U0 (context).  Returns dict(U, c, J, iters[, J_hist])."""
    x = _f32(x)
    nz, ny, nx = x.shape
    U0 = _f64(U0).reshape(-1, p.C)
    U = np.empty_like(U0)
    c = np.empty(p.C)
    J = ct.c_double()
    it = ct.c_int32()
    hist = np.empty(max(1, p.max_iter)) if want_hist else None
    _check(lib().oracle_solve_slab(_pf(x), nx, ny, nz, int(zbeg), int(zend), ct.byref(p.c()),
                                   float(lam), float(xi), _pd(_f64(c0)), _pd(U0), _pd(U), _pd(c),
                                   ct.byref(J), ct.byref(it), _pd(hist)), "solve_slab")
    out = dict(U=U, c=c, J=J.value, iters=it.value)
    if want_hist:
        out["J_hist"] = hist[: it.value].copy()
    return out


def fcm_init(x, p: Params):
    """Initial (c0, U0): FCM from evenly spaced centres, sorted."""
    x = _f32(x)
    nz, ny, nx = x.shape
    U = np.empty((x.size, p.C))
    c = np.empty(p.C)
    it = ct.c_int32()
    _check(lib().oracle_fcm_init(_pf(x), nx, ny, nz, ct.byref(p.c()), _pd(U), _pd(c),
                                 ct.byref(it)), "fcm_init")
    return c, U, it.value


def labels(U, C):
    U = _f64(U).reshape(-1, C)
    out = np.empty(U.shape[0], np.uint8)
    _check(lib().oracle_labels(_pd(U), U.shape[0], C,
                               out.ctypes.data_as(ct.POINTER(ct.c_uint8))), "labels")
    return out


def pso(x, c0, U0, p: Params, streams, w=0.7, c1=1.5, c2=1.5):
    """Global-best PSO over (lambda, xi).  streams: dict(x0, v0, r1, r2) as
    drawn by synth.pso_streams.  Returns dict(best_pos, best_fit, fit_hist,
    pos_hist)."""
    x = _f32(x)
    nz, ny, nx = x.shape
    x0, v0 = _f64(streams["x0"]), _f64(streams["v0"])
    r1, r2 = _f64(streams["r1"]), _f64(streams["r2"])
    G, P = r1.shape[0], r1.shape[1]
    bp = np.empty(2)
    bf = ct.c_double()
    fh = np.empty((G, P))
    ph = np.empty((G, P, 2))
    _check(lib().oracle_pso(_pf(x), nx, ny, nz, ct.byref(p.c()), _pd(_f64(c0)),
                            _pd(_f64(U0).reshape(-1, p.C)), P, G, _pd(x0), _pd(v0), _pd(r1),
                            _pd(r2), w, c1, c2, _pd(bp), ct.byref(bf), _pd(fh), _pd(ph)), "pso")
    return dict(best_pos=bp, best_fit=bf.value, fit_hist=fh, pos_hist=ph)


def pso_interleaved(x, c0, U0, p: Params, streams, steps=1, w=0.7, c1=1.5, c2=1.5):
    """Swarm whose particles carry their own IFCM state (`steps` iterations
    per generation).  Returns dict(best_pos, best_fit, fit_hist, pos_hist,
    U_best, c_best)."""
    x = _f32(x)
    nz, ny, nx = x.shape
    x0, v0 = _f64(streams["x0"]), _f64(streams["v0"])
    r1, r2 = _f64(streams["r1"]), _f64(streams["r2"])
    G, P = r1.shape[0], r1.shape[1]
    bp = np.empty(2)
    bf = ct.c_double()
    fh = np.empty((G, P))
    ph = np.empty((G, P, 2))
    Ub = np.empty((x.size, p.C))
    cb = np.empty(p.C)
    _check(lib().oracle_pso_interleaved(_pf(x), nx, ny, nz, ct.byref(p.c()), _pd(_f64(c0)),
                                        _pd(_f64(U0).reshape(-1, p.C)), P, G, int(steps), _pd(x0),
                                        _pd(v0), _pd(r1), _pd(r2), w, c1, c2, _pd(bp),
                                        ct.byref(bf), _pd(fh), _pd(ph), _pd(Ub), _pd(cb)),
           "pso_interleaved")
    return dict(best_pos=bp, best_fit=bf.value, fit_hist=fh, pos_hist=ph, U_best=Ub, c_best=cb)


def fd_grad(x, c0, U0, p: Params, lam, xi, K, step=1e-4):
    """Central differences of J_K.  Returns (J, grad[2 + C])."""
    x = _f32(x)
    nz, ny, nx = x.shape
    g = np.empty(2 + p.C)
    J = ct.c_double()
    _check(lib().oracle_fd_grad(_pf(x), nx, ny, nz, ct.byref(p.c()), float(lam), float(xi),
                                _pd(_f64(c0)), _pd(_f64(U0).reshape(-1, p.C)), int(K),
                                float(step), ct.byref(J), _pd(g)), "fd_grad")
    return J.value, g
