"""ctypes binding of libss.so (the C interface declared in include/ss.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libss.so.  PyTorch provides device memory (tensors) and streams.
There is no fallback: if libss.so is missing or no HIP device is present the
calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libss.so")
_LIB = None

SS_OK, SS_PENDING = 0, 1
SS_EINVAL, SS_ENOMEM, SS_EHIP, SS_ENOTFOUND, SS_ESTATE, SS_ENUMERIC = -1, -2, -3, -4, -5, -6


class SSError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what} (code {code})")
        self.code = code


class Problem(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("N", ctypes.c_int64), ("R2", ctypes.c_int64),
                ("M", ctypes.c_int64), ("L", ctypes.c_double), ("vkind", ctypes.c_int32)]


class MinOpts(ctypes.Structure):
    _fields_ = [("history", ctypes.c_int32), ("max_iter", ctypes.c_int64), ("s_floor", ctypes.c_double),
                ("stall_window", ctypes.c_int32), ("stall_ratio", ctypes.c_double), ("c1", ctypes.c_double),
                ("step_cap", ctypes.c_double), ("max_halvings", ctypes.c_int32),
                ("max_ls_fail", ctypes.c_int32)]


class MinResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int64), ("evals", ctypes.c_int64),
                ("grad_evals", ctypes.c_int64), ("phi", ctypes.c_double * 2), ("smax", ctypes.c_double * 2),
                ("seconds", ctypes.c_double)]


_V = ctypes.c_void_p
_I64P = ctypes.POINTER(ctypes.c_int64)
_SZP = ctypes.POINTER(ctypes.c_size_t)

# name -> (restype, argtypes); every symbol declared in include/ss.h
SIGNATURES = {
    "ss_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_V)]),
    "ss_destroy": (ctypes.c_int, [_V]),
    "ss_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "ss_last_error": (ctypes.c_char_p, [_V]),
    "ss_count": (ctypes.c_int, [ctypes.c_int, ctypes.c_int64, _I64P]),
    "ss_cutoff": (ctypes.c_int, [ctypes.c_int, ctypes.c_int64, ctypes.c_double, _I64P, _I64P]),
    "ss_wavevectors": (ctypes.c_int, [_V, ctypes.c_int, ctypes.c_int64, _V, ctypes.c_int64, _I64P, _V]),
    "ss_weights": (ctypes.c_int, [_V, ctypes.POINTER(Problem), _V, _V, _V]),
    "ss_workspace_size": (ctypes.c_int, [_V, ctypes.POINTER(Problem), ctypes.c_int, _SZP]),
    "ss_energy_grad": (ctypes.c_int, [_V, ctypes.POINTER(Problem), _V, _V, _V, _V, _V, _V, _V, _V,
                                      ctypes.c_size_t, _V]),
    "ss_profile_enable": (ctypes.c_int, [_V, ctypes.c_int]),
    "ss_profile_read": (ctypes.c_int, [_V, ctypes.c_int, ctypes.c_int, _I64P, ctypes.POINTER(ctypes.c_double)]),
    "ss_minimize": (ctypes.c_int, [_V, ctypes.POINTER(Problem), _V, _V, _V, ctypes.POINTER(MinOpts),
                                   ctypes.POINTER(MinResult), _V, ctypes.c_size_t, _V]),
}


def lib():
    """Load libss.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2304_09139_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            if hasattr(L, name):
                fn = getattr(L, name)
                fn.restype = res
                fn.argtypes = args
        _LIB = L
    return _LIB


def strerror(code: int) -> str:
    return lib().ss_strerror(code).decode()


def _check(rc: int, ctx=None, what: str = "") -> int:
    if rc < 0:
        detail = lib().ss_last_error(ctx).decode() if ctx else ""
        raise SSError(rc, f"{what}: {strerror(rc)}" + (f" [{detail}]" if detail else ""))
    return rc


def count(d: int, R2: int) -> int:
    M = ctypes.c_int64()
    _check(lib().ss_count(d, R2, ctypes.byref(M)), what="ss_count")
    return M.value


def cutoff(d: int, N: int, chi: float) -> tuple[int, int]:
    R2 = ctypes.c_int64()
    M = ctypes.c_int64()
    _check(lib().ss_cutoff(d, N, chi, ctypes.byref(R2), ctypes.byref(M)), what="ss_cutoff")
    return R2.value, M.value


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


STATUS = {0: "converged", 1: "stalled", 2: "max_iter", 3: "numeric"}


@dataclass
class Workload:
    d: int
    N: int
    R2: int
    M: int
    L: float = 1.0
    vkind: int = 0

    def problem(self) -> Problem:
        return Problem(self.d, self.N, self.R2, self.M, self.L, self.vkind)

    @classmethod
    def from_chi(cls, d: int, N: int, chi: float, L: float = 1.0, vkind: int = 0) -> "Workload":
        R2, M = cutoff(d, N, chi)
        return cls(d, N, R2, M, L, vkind)


class Context:
    """A libss context on one HIP device."""

    def __init__(self, device: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("libss needs a HIP device; none is visible")
        self.device = torch.device("cuda", device)
        self._h = ctypes.c_void_p()
        _check(lib().ss_create(device, ctypes.byref(self._h)), what="ss_create")
        self._ws = None

    def close(self):
        if self._h:
            lib().ss_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc, what):
        return _check(rc, self._h, what)

    KERNELS = {"nk": 0, "grad": 1, "table": 2}

    def profile(self, enable: bool = True, kernels=("nk", "grad", "table")) -> None:
        """Turn per-launch event timing of the named kernels on (or all timing off)."""
        mask = sum(1 << self.KERNELS[k] for k in kernels) if enable else 0
        self._chk(lib().ss_profile_enable(self._h, mask), "ss_profile_enable")

    def profile_read(self, kernel: str, reset: bool = True) -> tuple[int, float]:
        """(launches, total milliseconds) of one kernel since the last reset."""
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        self._chk(lib().ss_profile_read(self._h, self.KERNELS[kernel], 1 if reset else 0, ctypes.byref(n),
                                        ctypes.byref(ms)), "ss_profile_read")
        return n.value, ms.value

    def wavevectors(self, d: int, R2: int) -> torch.Tensor:
        M = ctypes.c_int64()
        self._chk(lib().ss_wavevectors(self._h, d, R2, None, 0, ctypes.byref(M), None), "ss_wavevectors")
        n = torch.empty((M.value, d), dtype=torch.int32, device=self.device)
        self._chk(lib().ss_wavevectors(self._h, d, R2, _ptr(n), M.value, ctypes.byref(M),
                                       _stream(self.device)), "ss_wavevectors")
        return n

    def weights(self, w: Workload, n: torch.Tensor) -> torch.Tensor:
        v = torch.empty((2, w.M), dtype=torch.float64, device=self.device)
        p = w.problem()
        self._chk(lib().ss_weights(self._h, ctypes.byref(p), _ptr(n), _ptr(v), _stream(self.device)),
                  "ss_weights")
        return v

    def workspace_size(self, w: Workload, op: int = 0) -> int:
        b = ctypes.c_size_t()
        p = w.problem()
        self._chk(lib().ss_workspace_size(self._h, ctypes.byref(p), op, ctypes.byref(b)), "ss_workspace_size")
        return b.value

    def workspace(self, w: Workload, op: int = 0) -> torch.Tensor:
        nbytes = self.workspace_size(w, op)
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        return self._ws

    def energy_grad(self, w: Workload, n: torch.Tensor, v: torch.Tensor | None, pos: torch.Tensor,
                    grad: bool = True, nk: bool = False, out: dict | None = None) -> dict:
        """Phi, S_max, optionally the gradient [2, d, N] and n~ [4, M] (device tensors)."""
        dev = self.device
        o = out if out is not None else {}
        if "phi" not in o:
            o["phi"] = torch.empty(2, dtype=torch.float64, device=dev)
            o["smax"] = torch.empty(2, dtype=torch.float64, device=dev)
        if grad and "grad" not in o:
            o["grad"] = torch.empty((2, w.d, w.N), dtype=torch.float64, device=dev)
        if nk and "nk" not in o:
            o["nk"] = torch.empty((4, w.M), dtype=torch.float64, device=dev)
        ws = self.workspace(w, 0)
        p = w.problem()
        self._chk(lib().ss_energy_grad(self._h, ctypes.byref(p), _ptr(n), _ptr(v), _ptr(pos), _ptr(o["phi"]),
                                       _ptr(o["smax"]), _ptr(o.get("grad") if grad else None),
                                       _ptr(o.get("nk") if nk else None), _ptr(ws), ws.numel(),
                                       _stream(dev)), "ss_energy_grad")
        return o

    def minimize(self, w: Workload, n: torch.Tensor, v: torch.Tensor | None, pos: torch.Tensor,
                 **opts) -> dict:
        """L-BFGS quench of pos (updated in place, [2, d, N]) on the device."""
        base = dict(history=8, max_iter=100000, s_floor=1e-40, stall_window=50, stall_ratio=0.99, c1=1e-4,
                    step_cap=1e-2, max_halvings=40, max_ls_fail=3)
        base.update(opts)
        mo = MinOpts(**base)
        res = MinResult()
        ws = self.workspace(w, 1)
        p = w.problem()
        self._chk(lib().ss_minimize(self._h, ctypes.byref(p), _ptr(n), _ptr(v), _ptr(pos), ctypes.byref(mo),
                                    ctypes.byref(res), _ptr(ws), ws.numel(), _stream(self.device)),
                  "ss_minimize")
        return dict(status=STATUS.get(res.status, str(res.status)), iters=res.iters, evals=res.evals,
                    grad_evals=res.grad_evals, phi=(res.phi[0], res.phi[1]), smax=(res.smax[0], res.smax[1]),
                    seconds=res.seconds)
