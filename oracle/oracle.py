"""Python access to the CPU oracle (``ss_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use this module to obtain an independent, plain
double-double evaluation of the stealthy-hyperuniform energy, its gradient, the
collective density n~(k), the wavevector set and the L-BFGS minimiser.  The
product library never imports it and has no CPU fallback to it.

Arrays of double-double values use a leading axis of length 2 (hi plane, lo
plane), e.g. positions are ``float64[2, d, N]`` of fractional coordinates
u = r / L; n~(k) is ``float64[4, M]`` = (C.hi, C.lo, S.hi, S.lo) with
n~(k) = C - i S (Eq. ntilde of the paper).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ss_oracle.c")
_SO = os.path.join(_HERE, "libss_oracle.so")
_LIB = None

_CFLAGS = ["-O2", "-mfma", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-std=c11", "-Wall", "-Wno-unused-function"]


def build(force: bool = True) -> str:
    """Compile the oracle shared library with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", *_CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_P = ctypes.POINTER
_D = _P(ctypes.c_double)
_I32 = _P(ctypes.c_int32)
_I64 = _P(ctypes.c_int64)


class LbfgsOpts(ctypes.Structure):
    _fields_ = [("history", ctypes.c_int), ("max_iter", ctypes.c_int64),
                ("s_floor", ctypes.c_double), ("stall_window", ctypes.c_int),
                ("stall_ratio", ctypes.c_double), ("c1", ctypes.c_double),
                ("step_cap", ctypes.c_double), ("max_halvings", ctypes.c_int),
                ("max_ls_fail", ctypes.c_int), ("method", ctypes.c_int)]


class LbfgsResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int64), ("evals", ctypes.c_int64),
                ("grad_evals", ctypes.c_int64), ("phi", ctypes.c_double * 2),
                ("smax", ctypes.c_double * 2)]


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_SO)
        L.or_cutoff.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, _I64, _I64]
        L.or_count.argtypes = [ctypes.c_int, ctypes.c_int64]
        L.or_count.restype = ctypes.c_int64
        L.or_wavevectors.argtypes = [ctypes.c_int, ctypes.c_int64, _I32, ctypes.c_int64, _I64]
        L.or_weights.argtypes = [ctypes.c_int, ctypes.c_int64, _I32, ctypes.c_int64, ctypes.c_int, _D]
        L.or_phase.argtypes = [ctypes.c_int, _I32, _D, _D, _D]
        L.or_sincos2pi.argtypes = [_D, _D, _D]
        L.or_two_pi.argtypes = [_D]
        for nm in ("or_dd_add", "or_dd_mul", "or_dd_div"):
            getattr(L, nm).argtypes = [_D, _D, _D]
        L.or_dd_sqrt.argtypes = [_D, _D]
        L.or_nk.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, _I32, _D, _D,
                            ctypes.c_int64, ctypes.c_int64]
        L.or_energy_from_nk.argtypes = [ctypes.c_int64, ctypes.c_int64, _D, _D, _D, _D, _I64, _D]
        L.or_grad.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_double, _I32,
                              _D, _D, _D, _I64, ctypes.c_int64, _D]
        L.or_energy_grad.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                                     _I32, _D, _D, _D, _D, _D, _D]
        L.or_minimize.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                                  _I32, _D, _D, _P(LbfgsOpts), _P(LbfgsResult), _D, ctypes.c_int64]
        L.or_minimize_quadratic.argtypes = [ctypes.c_int64, _D, _D, _D, _P(LbfgsOpts),
                                            _P(LbfgsResult), _D, ctypes.c_int64]
        L.or_num_threads.restype = ctypes.c_int
        L.or_set_num_threads.argtypes = [ctypes.c_int]
        _LIB = L
    return _LIB


def _dptr(a):
    return a.ctypes.data_as(_D) if a is not None else None


def _cd(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return lib().or_num_threads()


def set_num_threads(n: int) -> None:
    lib().or_set_num_threads(int(n))


# --- primitives -------------------------------------------------------------

def dd_add(a, b):
    r = np.zeros(2)
    lib().or_dd_add(_dptr(_cd(a)), _dptr(_cd(b)), _dptr(r))
    return r


def dd_mul(a, b):
    r = np.zeros(2)
    lib().or_dd_mul(_dptr(_cd(a)), _dptr(_cd(b)), _dptr(r))
    return r


def dd_div(a, b):
    r = np.zeros(2)
    lib().or_dd_div(_dptr(_cd(a)), _dptr(_cd(b)), _dptr(r))
    return r


def dd_sqrt(a):
    r = np.zeros(2)
    lib().or_dd_sqrt(_dptr(_cd(a)), _dptr(r))
    return r


def two_pi():
    r = np.zeros(2)
    lib().or_two_pi(_dptr(r))
    return r


def phase(n, uhi, ulo):
    """frac(n . u) in [-1/2, 1/2] as (hi, lo), integer part removed exactly."""
    n = np.ascontiguousarray(n, dtype=np.int32)
    t = np.zeros(2)
    lib().or_phase(len(n), n.ctypes.data_as(_I32), _dptr(_cd(uhi)), _dptr(_cd(ulo)), _dptr(t))
    return t


def sincos2pi(t):
    """(cos 2 pi t, sin 2 pi t) as two (hi, lo) pairs."""
    c = np.zeros(2)
    s = np.zeros(2)
    lib().or_sincos2pi(_dptr(_cd(t)), _dptr(c), _dptr(s))
    return c, s


# --- wavevectors --------------------------------------------------------------

def cutoff(d: int, N: int, chi: float):
    R2 = ctypes.c_int64()
    M = ctypes.c_int64()
    rc = lib().or_cutoff(d, N, chi, ctypes.byref(R2), ctypes.byref(M))
    if rc != 0:
        raise ValueError(f"invalid cutoff request d={d} N={N} chi={chi}")
    return R2.value, M.value


def count(d: int, R2: int) -> int:
    return int(lib().or_count(d, R2))


def wavevectors(d: int, R2: int) -> np.ndarray:
    M = ctypes.c_int64()
    lib().or_wavevectors(d, R2, None, 0, ctypes.byref(M))
    out = np.zeros((M.value, d), dtype=np.int32)
    lib().or_wavevectors(d, R2, out.ctypes.data_as(_I32), M.value, ctypes.byref(M))
    return out


def weights(n: np.ndarray, R2: int, vkind: int) -> np.ndarray:
    n = np.ascontiguousarray(n, dtype=np.int32)
    M, d = n.shape
    v = np.zeros((2, M))
    rc = lib().or_weights(d, M, n.ctypes.data_as(_I32), R2, vkind, _dptr(v))
    if rc != 0:
        raise ValueError("unknown weight kind")
    return v


# --- energy ------------------------------------------------------------------

def nk(n: np.ndarray, pos: np.ndarray, k0: int = 0, k1: int | None = None) -> np.ndarray:
    n = np.ascontiguousarray(n, dtype=np.int32)
    pos = _cd(pos)
    M, d = n.shape
    N = pos.shape[2]
    k1 = M if k1 is None else k1
    out = np.zeros((4, M))
    lib().or_nk(d, N, M, n.ctypes.data_as(_I32), _dptr(pos), _dptr(out), k0, k1)
    return out


@dataclass
class Energy:
    phi: np.ndarray      # (hi, lo)
    smax: np.ndarray     # (hi, lo)
    kmax: int
    sk: np.ndarray       # [2, M]


def energy_from_nk(N: int, v, nkv: np.ndarray) -> Energy:
    nkv = _cd(nkv)
    M = nkv.shape[1]
    phi = np.zeros(2)
    smax = np.zeros(2)
    kmax = ctypes.c_int64()
    sk = np.zeros((2, M))
    lib().or_energy_from_nk(N, M, _dptr(_cd(v)) if v is not None else None, _dptr(nkv),
                            _dptr(phi), _dptr(smax), ctypes.byref(kmax), _dptr(sk))
    return Energy(phi, smax, kmax.value, sk)


def grad(n, v, pos, nkv, L: float = 1.0, js=None) -> np.ndarray:
    """dPhi/dr for the listed particles (all when js is None): float64[nj, d, 2]."""
    n = np.ascontiguousarray(n, dtype=np.int32)
    pos = _cd(pos)
    M, d = n.shape
    N = pos.shape[2]
    if js is None:
        nj = N
        jp = None
    else:
        js = np.ascontiguousarray(js, dtype=np.int64)
        nj = len(js)
        jp = js.ctypes.data_as(_I64)
    g = np.zeros((nj, d, 2))
    lib().or_grad(d, N, M, L, n.ctypes.data_as(_I32), _dptr(_cd(v)) if v is not None else None,
                  _dptr(pos), _dptr(_cd(nkv)), jp, nj, _dptr(g))
    return g


def energy_grad(n, v, pos, L: float = 1.0, want_grad: bool = True):
    """Full evaluation; returns dict(phi, smax, grad[2,d,N] or None, nk[4,M])."""
    n = np.ascontiguousarray(n, dtype=np.int32)
    pos = _cd(pos)
    M, d = n.shape
    N = pos.shape[2]
    phi = np.zeros(2)
    smax = np.zeros(2)
    g = np.zeros((2, d, N)) if want_grad else None
    nkv = np.zeros((4, M))
    lib().or_energy_grad(d, N, M, L, n.ctypes.data_as(_I32),
                         _dptr(_cd(v)) if v is not None else None, _dptr(pos),
                         _dptr(phi), _dptr(smax), _dptr(g), _dptr(nkv))
    return dict(phi=phi, smax=smax, grad=g, nk=nkv)


# --- minimiser ----------------------------------------------------------------

DEFAULT_OPTS = dict(history=8, max_iter=100000, s_floor=1e-40, stall_window=50,
                    stall_ratio=0.99, c1=1e-4, step_cap=1e-2, max_halvings=40, max_ls_fail=3, method=0)
METHODS = {"lbfgs": 0, "fire": 1}

STATUS = {0: "converged", 1: "stalled", 2: "max_iter", 3: "numeric"}


def _opts(**kw) -> LbfgsOpts:
    o = dict(DEFAULT_OPTS)
    o.update(kw)
    if isinstance(o["method"], str):
        o["method"] = METHODS[o["method"]]
    return LbfgsOpts(**o)


def minimize(n, v, pos, L: float = 1.0, trace_cap: int = 0, **kw):
    """L-BFGS (method="lbfgs") or FIRE (method="fire") on the stealthy energy;
    returns (pos_out, result dict, phi trace [k,2])."""
    n = np.ascontiguousarray(n, dtype=np.int32)
    x = np.array(pos, dtype=np.float64, copy=True, order="C")
    M, d = n.shape
    N = x.shape[2]
    op = _opts(**kw)
    res = LbfgsResult()
    tr = np.zeros((max(trace_cap, 1), 2))
    rc = lib().or_minimize(d, N, M, L, n.ctypes.data_as(_I32),
                           _dptr(_cd(v)) if v is not None else None, _dptr(x),
                           ctypes.byref(op), ctypes.byref(res), _dptr(tr), trace_cap)
    if rc != 0:
        raise MemoryError("oracle minimiser allocation failed")
    out = dict(status=STATUS[res.status], iters=res.iters, evals=res.evals,
               grad_evals=res.grad_evals, phi=np.array(res.phi[:]), smax=np.array(res.smax[:]))
    return x, out, tr[:min(trace_cap, res.iters + 1)]


def minimize_quadratic(w, c, x0, trace_cap: int = 0, **kw):
    """Same minimiser on f(x) = 1/2 sum w_i (x_i - c_i)^2; arrays are dd [2, n]."""
    w = _cd(w)
    c = _cd(c)
    x = np.array(x0, dtype=np.float64, copy=True, order="C")
    nv = x.shape[1]
    op = _opts(**kw)
    res = LbfgsResult()
    tr = np.zeros((max(trace_cap, 1), 2))
    rc = lib().or_minimize_quadratic(nv, _dptr(w), _dptr(c), _dptr(x), ctypes.byref(op),
                                     ctypes.byref(res), _dptr(tr), trace_cap)
    if rc != 0:
        raise MemoryError("oracle minimiser allocation failed")
    out = dict(status=STATUS[res.status], iters=res.iters, evals=res.evals,
               grad_evals=res.grad_evals, phi=np.array(res.phi[:]), smax=np.array(res.smax[:]))
    return x, out, tr[:min(trace_cap, res.iters + 1)]
