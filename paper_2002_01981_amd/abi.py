"""ctypes binding of libpifcm (include/pifcm.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libpifcm.so.  PyTorch provides device memory (tensors' data
pointers) and the current HIP stream.  If the shared library is missing this
module raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as ct
import os
import re
from dataclasses import dataclass

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
# PIFCM_LIB selects another build of the library (kernel variants).
LIB_PATH = os.environ.get("PIFCM_LIB") or os.path.join(PKG, "libpifcm.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "pifcm.h")

PIFCM_OK = 0
PIFCM_E_INVALID = -1
PIFCM_E_NONFINITE = -2
PIFCM_E_OOM = -3
PIFCM_E_HIP = -4
PIFCM_E_UNSUPPORTED = -5
PIFCM_SHELL_SQDIST = 1
PIFCM_Q2_SQDIST = 2
PIFCM_SWARM_BATCHED = 0
PIFCM_SWARM_PLAIN = 1

_STATUS = {0: "OK", -1: "INVALID", -2: "NONFINITE", -3: "OOM", -4: "HIP", -5: "UNSUPPORTED"}


class PifcmError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"libpifcm {_STATUS.get(status, status)}: {message}")
        self.status = status


class _Params(ct.Structure):
    _fields_ = [("C", ct.c_int32), ("m", ct.c_float), ("V", ct.c_int32), ("h", ct.c_float),
                ("eps", ct.c_float), ("max_iter", ct.c_int32), ("flags", ct.c_int32)]


class _Volume(ct.Structure):
    _fields_ = [("nx", ct.c_int32), ("ny", ct.c_int32), ("nz", ct.c_int32), ("x", ct.c_void_p)]


@dataclass
class Params:
    """pifcm_params: C clusters, fuzziness m, depth V, decay h, stop eps,
    iteration cap, reading flags."""
    C: int = 4
    m: float = 2.0
    V: int = 1
    h: float = 1.0
    eps: float = 1e-5
    max_iter: int = 50
    flags: int = 0

    def c(self):
        return _Params(self.C, self.m, self.V, self.h, self.eps, self.max_iter, self.flags)


def header_symbols(path=HEADER):
    """Names of the functions declared in include/pifcm.h."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:pifcm_status|void|const char\*)\s+(\w+)\s*\(", text, re.M)))


_lib = None


def load_library(path=LIB_PATH):
    """Load libpifcm.so and declare its functions.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run `python paper_2002_01981_amd/build.py`")
    lib = ct.CDLL(path)
    P, vp, i32, i64 = ct.POINTER, ct.c_void_p, ct.c_int32, ct.c_int64
    f32, f64 = ct.c_float, ct.c_double
    st = ct.c_int
    lib.pifcm_create.argtypes = [ct.c_int, vp, P(vp)]
    lib.pifcm_create.restype = st
    lib.pifcm_destroy.argtypes = [vp]
    lib.pifcm_destroy.restype = None
    lib.pifcm_set_stream.argtypes = [vp, vp]
    lib.pifcm_set_stream.restype = st
    lib.pifcm_last_error.argtypes = [vp]
    lib.pifcm_last_error.restype = ct.c_char_p
    lib.pifcm_normalize.argtypes = [vp, vp, i64, vp]
    lib.pifcm_normalize.restype = st
    lib.ifcm_solve.argtypes = [vp, P(_Volume), P(_Params), f32, f32, P(f32), vp, vp, P(f32), vp,
                               P(f64), P(i32), P(f64)]
    lib.ifcm_solve.restype = st
    lib.ifcm_solve_noalloc.argtypes = lib.ifcm_solve.argtypes
    lib.ifcm_solve_noalloc.restype = st
    lib.ifcm_solve_slab.argtypes = [vp, P(_Volume), i32, i32, P(_Params), f32, f32, P(f32), vp, vp,
                                    P(f32), vp, P(f64), P(i32), P(f64)]
    lib.ifcm_solve_slab.restype = st
    lib.pifcm_fcm_init.argtypes = [vp, P(_Volume), P(_Params), vp, P(f32), P(i32)]
    lib.pifcm_fcm_init.restype = st
    lib.swarm_evaluate.argtypes = [vp, P(_Volume), i32, P(_Params), P(f32), i32, P(f32), P(vp),
                                   P(f64), P(f32), P(i32), i32]
    lib.swarm_evaluate.restype = st
    lib.ifcm_backward.argtypes = [vp, P(_Volume), P(_Params), f32, f32, P(f32), vp, i32, i32,
                                  P(f64), P(f64), P(f64), P(f64)]
    lib.ifcm_backward.restype = st
    lib.pifcm_tune.argtypes = [vp, P(_Volume), i32, P(_Params), i32, ct.c_char_p, i32]
    lib.pifcm_tune.restype = st
    lib.pifcm_set_decomposition.argtypes = [vp, P(_Volume), i32, P(_Params), i32, i32, i32]
    lib.pifcm_set_decomposition.restype = st
    lib.pifcm_pso.argtypes = [vp, P(_Volume), i32, P(_Params), i32, i32, P(f64), P(f64), P(f64),
                              P(f64), f64, f64, f64, P(f32), P(vp), i32, P(f64), P(f64), P(f64),
                              P(f64), P(i32)]
    lib.pifcm_pso.restype = st
    lib.pifcm_pso_interleaved.argtypes = [vp, P(_Volume), i32, P(_Params), i32, i32, i32, P(f64),
                                          P(f64), P(f64), P(f64), f64, f64, f64, P(f32), P(vp),
                                          i32, P(f64), P(f64), P(f64), P(f64), P(vp), P(f32)]
    lib.pifcm_pso_interleaved.restype = st
    lib.pifcm_confusion.argtypes = [vp, vp, vp, i64, i32, i32, P(i64)]
    lib.pifcm_confusion.restype = st
    lib.pifcm_workspace_bytes.argtypes = [vp, P(i64), P(i64)]
    lib.pifcm_workspace_bytes.restype = st
    lib.pifcm_set_timing.argtypes = [vp, i32]
    lib.pifcm_set_timing.restype = st
    lib.pifcm_get_timing.argtypes = [vp, P(f64), P(i64), i32]
    lib.pifcm_get_timing.restype = st
    _lib = lib
    return lib


def _fp(a):
    return a.ctypes.data_as(ct.POINTER(ct.c_float))


def _dp(a):
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def _ip(a):
    return a.ctypes.data_as(ct.POINTER(ct.c_int32))


def _is_device(t):
    return t.is_cuda


def _dev(t, dtype=None, numel=None, what="tensor"):
    """A contiguous device tensor of the given dtype and element count.  The
    C ABI receives bare pointers and cannot know buffer sizes, so every
    device buffer is checked here before the library is called."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what}: expected a torch tensor, got {type(t).__name__}")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{what}: expected {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{what}: {t.numel()} elements, expected {numel}")
    if not t.is_contiguous():
        raise ValueError(f"{what}: expected a contiguous tensor")
    if not _is_device(t):
        raise TypeError(f"{what}: expected a device tensor")
    return t


def _memberships(u, x, C, what):
    """Memberships (N, C) float32 of volume x, on x's device."""
    import torch
    _dev(u, torch.float32, x.numel() * C, what)
    if u.device != x.device:
        raise ValueError(f"{what} is on {u.device}, the volume on {x.device}")
    return u


def _host_vec(a, n, dtype, what):
    v = np.ascontiguousarray(a, dtype)
    if v.size != n:
        raise ValueError(f"{what}: {v.size} values, expected {n}")
    return v


def _volume(x):
    import torch
    _dev(x, torch.float32, what="volume")
    if x.dim() != 3:
        raise ValueError("volume must be (Z, Y, X)")
    nz, ny, nx = x.shape
    return _Volume(nx, ny, nz, x.data_ptr())


def _volumes(xs, U0s, C):
    """Volume table of a batch and its B initial-membership pointers."""
    B = len(xs)
    if B < 1:
        raise ValueError("need at least one volume")
    if len(U0s) != B:
        raise ValueError(f"{len(U0s)} initial memberships for {B} volumes")
    vols = (_Volume * B)(*[_volume(x) for x in xs])
    ptrs = (ct.c_void_p * B)(*[_memberships(u, x, C, f"U0s[{b}]").data_ptr()
                               for b, (x, u) in enumerate(zip(xs, U0s))])
    return vols, ptrs


def _streams(streams):
    x0 = np.ascontiguousarray(streams["x0"], np.float64)
    v0 = np.ascontiguousarray(streams["v0"], np.float64)
    r1 = np.ascontiguousarray(streams["r1"], np.float64)
    r2 = np.ascontiguousarray(streams["r2"], np.float64)
    if r1.ndim != 3 or r1.shape[2] != 2:
        raise ValueError("r1 must be (G, P, 2)")
    G, P = r1.shape[0], r1.shape[1]
    if x0.shape != (P, 2) or v0.shape != (P, 2) or r2.shape != (G, P, 2):
        raise ValueError("stream shapes do not agree")
    return x0, v0, r1, r2, G, P


class Context:
    """A libpifcm context on one GPU, ordered on torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.lib = load_library()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        h = ct.c_void_p()
        rc = self.lib.pifcm_create(device, ct.c_void_p(stream.cuda_stream), ct.byref(h))
        if rc != PIFCM_OK:
            raise PifcmError(rc, f"pifcm_create(device={device}) failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.pifcm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != PIFCM_OK:
            msg = self.lib.pifcm_last_error(self.h)
            raise PifcmError(rc, msg.decode() if msg else "")

    def set_stream(self, stream):
        self._check(self.lib.pifcm_set_stream(self.h, ct.c_void_p(stream.cuda_stream)))

    # ------------------------------------------------------------ entry points
    def pifcm_normalize(self, raw, out=None):
        import torch
        _dev(raw, torch.float32, what="raw")
        if out is None:
            out = torch.empty_like(raw)
        _dev(out, torch.float32, raw.numel(), "out")
        self._check(self.lib.pifcm_normalize(self.h, raw.data_ptr(), raw.numel(), out.data_ptr()))
        return out

    def pifcm_fcm_init(self, x, p: Params):
        import torch
        vol = _volume(x)
        U0 = torch.empty((x.numel(), p.C), dtype=torch.float32, device=x.device)
        c = np.empty(p.C, np.float32)
        it = np.zeros(1, np.int32)
        self._check(self.lib.pifcm_fcm_init(self.h, ct.byref(vol), ct.byref(p.c()), U0.data_ptr(),
                                            _fp(c), _ip(it)))
        return c, U0, int(it[0])

    def ifcm_solve(self, x, p: Params, lam, xi, centres, U_in=None, labels=False,
                   want_hist=False, U_out=None):
        return self._solve("ifcm_solve", x, p, lam, xi, centres, U_in, labels, want_hist, U_out)

    def ifcm_solve_noalloc(self, x, p: Params, lam, xi, centres, U_in=None, labels=False,
                           want_hist=False, U_out=None):
        """ifcm_solve in the library's per-device scratch (no device
        allocation by the library; U_out and labels are allocated here unless
        given)."""
        return self._solve("ifcm_solve_noalloc", x, p, lam, xi, centres, U_in, labels,
                           want_hist, U_out)

    def _solve(self, name, x, p: Params, lam, xi, centres, U_in, labels, want_hist, U_out):
        import torch
        vol = _volume(x)
        c = _host_vec(centres, p.C, np.float32, "centres")
        if U_in is not None:
            _memberships(U_in, x, p.C, "U_in")
        if U_out is None:
            U_out = torch.empty((x.numel(), p.C), dtype=torch.float32, device=x.device)
        _memberships(U_out, x, p.C, "U_out")
        lab = torch.empty(x.numel(), dtype=torch.uint8, device=x.device) if labels else None
        cout = np.empty(p.C, np.float32)
        J = np.zeros(1, np.float64)
        it = np.zeros(1, np.int32)
        hist = np.zeros(max(1, p.max_iter), np.float64)
        self._check(getattr(self.lib, name)(
            self.h, ct.byref(vol), ct.byref(p.c()), float(lam), float(xi), _fp(c),
            None if U_in is None else U_in.data_ptr(), U_out.data_ptr(), _fp(cout),
            None if lab is None else lab.data_ptr(), _dp(J), _ip(it),
            _dp(hist) if want_hist else None))
        out = dict(U=U_out, c=cout, J=float(J[0]), iters=int(it[0]))
        if labels:
            out["labels"] = lab
        if want_hist:
            out["J_hist"] = hist[: out["iters"]].copy()
        return out

    def ifcm_solve_slab(self, x, zbeg, zend, p: Params, lam, xi, centres, U_in, labels=False,
                        want_hist=False):
        """ifcm_solve on the planes [zbeg, zend) only, the rest of U_in held
        fixed as context."""
        import torch
        vol = _volume(x)
        c = _host_vec(centres, p.C, np.float32, "centres")
        _memberships(U_in, x, p.C, "U_in")
        U_out = torch.empty((x.numel(), p.C), dtype=torch.float32, device=x.device)
        lab = torch.empty(x.numel(), dtype=torch.uint8, device=x.device) if labels else None
        cout = np.empty(p.C, np.float32)
        J = np.zeros(1, np.float64)
        it = np.zeros(1, np.int32)
        hist = np.zeros(max(1, p.max_iter), np.float64)
        self._check(self.lib.ifcm_solve_slab(
            self.h, ct.byref(vol), int(zbeg), int(zend), ct.byref(p.c()), float(lam), float(xi),
            _fp(c), U_in.data_ptr(), U_out.data_ptr(), _fp(cout),
            None if lab is None else lab.data_ptr(), _dp(J), _ip(it),
            _dp(hist) if want_hist else None))
        out = dict(U=U_out, c=cout, J=float(J[0]), iters=int(it[0]))
        if labels:
            out["labels"] = lab
        if want_hist:
            out["J_hist"] = hist[: out["iters"]].copy()
        return out

    def swarm_evaluate(self, xs, p: Params, particles, centres0, U0s, mode=PIFCM_SWARM_BATCHED):
        """xs: list of B (Z, Y, X) tensors; particles: (B, P, 2); centres0:
        (B, C); U0s: list of B (N_b, C) tensors."""
        B = len(xs)
        vols, ptrs = _volumes(xs, U0s, p.C)
        part = np.ascontiguousarray(particles, np.float32)
        if part.ndim == 2:
            part = np.ascontiguousarray(np.broadcast_to(part, (B,) + part.shape))
        if part.ndim != 3 or part.shape[0] != B or part.shape[2] != 2 or part.shape[1] < 1:
            raise ValueError(f"particles must be (P, 2) or (B={B}, P, 2), got {part.shape}")
        P = part.shape[1]
        c0 = _host_vec(centres0, B * p.C, np.float32, "centres0").reshape(B, p.C)
        fit = np.empty((B, P), np.float64)
        cout = np.empty((B, P, p.C), np.float32)
        it = np.empty((B, P), np.int32)
        self._check(self.lib.swarm_evaluate(self.h, vols, B, ct.byref(p.c()), _fp(part), P, _fp(c0),
                                            ptrs, _dp(fit), _fp(cout), _ip(it), int(mode)))
        return dict(fitness=fit, centres=cout, iters=it)

    def ifcm_backward(self, x, p: Params, lam, xi, centres0, U0, K, ckpt_every):
        vol = _volume(x)
        c = _host_vec(centres0, p.C, np.float32, "centres0")
        _memberships(U0, x, p.C, "U0")
        J = np.zeros(1)
        dl = np.zeros(1)
        dx = np.zeros(1)
        dc = np.zeros(p.C)
        self._check(self.lib.ifcm_backward(self.h, ct.byref(vol), ct.byref(p.c()), float(lam),
                                           float(xi), _fp(c), U0.data_ptr(), int(K),
                                           int(ckpt_every), _dp(J), _dp(dl), _dp(dx), _dp(dc)))
        return dict(J=float(J[0]), dlam=float(dl[0]), dxi=float(dx[0]), dc=dc)

    def pifcm_confusion(self, labels, truth, C, K):
        """Confusion counts (C, K) of device uint8 labels against device uint8
        reference classes."""
        import torch
        lab = _dev(labels, torch.uint8)
        tru = _dev(truth, torch.uint8)
        if lab.numel() != tru.numel():
            raise ValueError("labels and truth differ in size")
        out = np.empty((C, K), np.int64)
        self._check(self.lib.pifcm_confusion(self.h, lab.data_ptr(), tru.data_ptr(), lab.numel(),
                                             int(C), int(K),
                                             out.ctypes.data_as(ct.POINTER(ct.c_int64))))
        return out

    def workspace_bytes(self):
        """Device bytes of workspace the context holds (its peak so far)."""
        d, h = ct.c_int64(), ct.c_int64()
        self._check(self.lib.pifcm_workspace_bytes(self.h, ct.byref(d), ct.byref(h)))
        return int(d.value)

    def pifcm_set_timing(self, enable=True):
        self._check(self.lib.pifcm_set_timing(self.h, 1 if enable else 0))

    def pifcm_get_timing(self, reset=False):
        ms = ct.c_double()
        n = ct.c_int64()
        self._check(self.lib.pifcm_get_timing(self.h, ct.byref(ms), ct.byref(n), 1 if reset else 0))
        return ms.value, n.value

    def pifcm_set_decomposition(self, xs, p: Params, waves_per_group=4, planes_per_tile=32,
                                particles_per_item=1):
        B = len(xs)
        vols = (_Volume * B)(*[_volume(x) for x in xs])
        self._check(self.lib.pifcm_set_decomposition(self.h, vols, B, ct.byref(p.c()), int(waves_per_group),
                                                     int(planes_per_tile), int(particles_per_item)))

    def pifcm_tune(self, xs, p: Params, P):
        B = len(xs)
        vols = (_Volume * B)(*[_volume(x) for x in xs])
        buf = ct.create_string_buffer(1024)
        self._check(self.lib.pifcm_tune(self.h, vols, B, ct.byref(p.c()), int(P), buf, 1024))
        return buf.value.decode()

    def pifcm_pso(self, xs, p: Params, streams, centres0, U0s, w=0.7, c1=1.5, c2=1.5,
                  mode=PIFCM_SWARM_BATCHED):
        """Global-best PSO on B volumes.  streams: dict(x0, v0 (P, 2), r1, r2
        (G, P, 2)); centres0 (B, C); U0s: list of B (N_b, C) tensors.
        Returns dict(best_pos (B, 2), best_fit (B,), fit_hist (B, G, P),
        pos_hist (B, G, P, 2), iters_hist (B, G, P) iterations per evaluation)."""
        B = len(xs)
        vols, ptrs = _volumes(xs, U0s, p.C)
        x0, v0, r1, r2, G, P = _streams(streams)
        c0 = _host_vec(centres0, B * p.C, np.float32, "centres0").reshape(B, p.C)
        bp = np.empty((B, 2))
        bf = np.empty(B)
        fh = np.empty((B, G, P))
        ph = np.empty((B, G, P, 2))
        ih = np.empty((B, G, P), np.int32)
        self._check(self.lib.pifcm_pso(self.h, vols, B, ct.byref(p.c()), P, G, _dp(x0), _dp(v0),
                                       _dp(r1), _dp(r2), float(w), float(c1), float(c2), _fp(c0),
                                       ptrs, int(mode), _dp(bp), _dp(bf), _dp(fh), _dp(ph), _ip(ih)))
        return dict(best_pos=bp, best_fit=bf, fit_hist=fh, pos_hist=ph, iters_hist=ih)

    def pifcm_pso_interleaved(self, xs, p: Params, streams, centres0, U0s, steps=1, w=0.7, c1=1.5,
                              c2=1.5, mode=PIFCM_SWARM_BATCHED):
        """Swarm whose particles carry their own IFCM state, `steps`
        iterations per generation.  Returns the outputs of pifcm_pso plus
        U_best (list of B device (N_b, C) tensors) and centres_best (B, C)."""
        import torch
        B = len(xs)
        vols, ptrs = _volumes(xs, U0s, p.C)
        x0, v0, r1, r2, G, P = _streams(streams)
        c0 = _host_vec(centres0, B * p.C, np.float32, "centres0").reshape(B, p.C)
        ub = [torch.empty((x.numel(), p.C), dtype=torch.float32, device=x.device) for x in xs]
        uptr = (ct.c_void_p * B)(*[u.data_ptr() for u in ub])
        cb = np.empty((B, p.C), np.float32)
        bp = np.empty((B, 2))
        bf = np.empty(B)
        fh = np.empty((B, G, P))
        ph = np.empty((B, G, P, 2))
        self._check(self.lib.pifcm_pso_interleaved(
            self.h, vols, B, ct.byref(p.c()), P, G, int(steps), _dp(x0), _dp(v0), _dp(r1), _dp(r2),
            float(w), float(c1), float(c2), _fp(c0), ptrs, int(mode), _dp(bp), _dp(bf), _dp(fh),
            _dp(ph), uptr, _fp(cb)))
        return dict(best_pos=bp, best_fit=bf, fit_hist=fh, pos_hist=ph, U_best=ub, centres_best=cb)
