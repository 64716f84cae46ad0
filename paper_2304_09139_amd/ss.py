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
                ("max_ls_fail", ctypes.c_int32), ("precision", ctypes.c_int32), ("fp64_floor", ctypes.c_double),
                ("method", ctypes.c_int32), ("fault_iter", ctypes.c_int64)]


class MinResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int64), ("evals", ctypes.c_int64),
                ("grad_evals", ctypes.c_int64), ("phi", ctypes.c_double * 2), ("smax", ctypes.c_double * 2),
                ("seconds", ctypes.c_double), ("iters_fp64", ctypes.c_int64), ("evals_fp64", ctypes.c_int64)]


class Tile(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("max_N", ctypes.c_int64), ("max_M", ctypes.c_int64),
                ("nk_chunk", ctypes.c_int64), ("grad_k", ctypes.c_int64)]


class Request(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("N", ctypes.c_int64), ("R2", ctypes.c_int64), ("L", ctypes.c_double),
                ("vkind", ctypes.c_int32), ("pos_host", ctypes.c_void_p), ("seed", ctypes.c_uint64),
                ("opts", MinOpts)]


class ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("submitted", "admitted", "completed", "queued", "running",
                                               "max_running", "steps", "overtaking")]


_V = ctypes.c_void_p
_I64P = ctypes.POINTER(ctypes.c_int64)
_SZP = ctypes.POINTER(ctypes.c_size_t)

# name -> (restype, argtypes); every symbol declared in include/ss.h
SIGNATURES = {
    "ss_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_V)]),
    "ss_destroy": (ctypes.c_int, [_V]),
    "ss_build_id": (ctypes.c_char_p, []),
    "ss_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "ss_last_error": (ctypes.c_char_p, [_V]),
    "ss_count": (ctypes.c_int, [ctypes.c_int, ctypes.c_int64, _I64P]),
    "ss_uniform_positions": (ctypes.c_int, [ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, _V]),
    "ss_cutoff": (ctypes.c_int, [ctypes.c_int, ctypes.c_int64, ctypes.c_double, _I64P, _I64P]),
    "ss_wavevectors": (ctypes.c_int, [_V, ctypes.c_int, ctypes.c_int64, _V, ctypes.c_int64, _I64P, _V]),
    "ss_weights": (ctypes.c_int, [_V, ctypes.POINTER(Problem), _V, _V, _V]),
    "ss_workspace_size": (ctypes.c_int, [_V, ctypes.POINTER(Problem), ctypes.c_int, _SZP]),
    "ss_energy_grad": (ctypes.c_int, [_V, ctypes.POINTER(Problem), _V, _V, _V, _V, _V, _V, _V, _V,
                                      ctypes.c_size_t, _V]),
    "ss_energy_grad_fp64": (ctypes.c_int, [_V, ctypes.POINTER(Problem), _V, _V, _V, _V, _V, _V, _V, _V,
                                           ctypes.c_size_t, _V]),
    "ss_energy_grad_static": (ctypes.c_int, [_V, ctypes.POINTER(Problem), _V, _V, _V, _V, _V, _V, _V, _V]),
    "ss_static_scratch_bytes": (ctypes.c_size_t, []),
    "ss_set_progress": (ctypes.c_int, [_V, ctypes.c_double]),
    "ss_profile_enable": (ctypes.c_int, [_V, ctypes.c_int]),
    "ss_profile_read": (ctypes.c_int, [_V, ctypes.c_int, ctypes.c_int, _I64P, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double)]),
    "ss_minimize": (ctypes.c_int, [_V, ctypes.POINTER(Problem), _V, _V, _V, ctypes.POINTER(MinOpts),
                                   ctypes.POINTER(MinResult), _V, ctypes.c_size_t, _V]),
    "ss_set_tiles": (ctypes.c_int, [_V, ctypes.POINTER(Tile), ctypes.c_int]),
    "ss_get_tile": (ctypes.c_int, [_V, ctypes.POINTER(Problem), ctypes.POINTER(Tile)]),
    "ss_batch_workspace_size": (ctypes.c_int, [_V, ctypes.c_int, ctypes.POINTER(Problem), ctypes.POINTER(MinOpts),
                                               _SZP]),
    "ss_minimize_batch": (ctypes.c_int, [_V, ctypes.c_int, ctypes.POINTER(Problem), ctypes.POINTER(_V),
                                         ctypes.POINTER(_V), ctypes.POINTER(MinOpts), ctypes.POINTER(MinResult),
                                         _V, ctypes.c_size_t, _V]),
    "ss_server_start": (ctypes.c_int, [_V, _V, ctypes.c_size_t, ctypes.c_int]),
    "ss_submit": (ctypes.c_int, [_V, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]),
    "ss_poll": (ctypes.c_int, [_V, ctypes.c_uint64, ctypes.POINTER(MinResult), _V]),
    "ss_server_stop": (ctypes.c_int, [_V]),
    "ss_server_stats": (ctypes.c_int, [_V, ctypes.c_void_p]),
}

DEFAULT_MIN_OPTS = dict(history=8, max_iter=100000, s_floor=1e-40, stall_window=50, stall_ratio=0.99, c1=1e-4,
                        step_cap=1e-2, max_halvings=40, max_ls_fail=3, precision=0, fp64_floor=1e-24, method=0,
                        fault_iter=0)
PRECISION = {"dd": 0, "fp64": 1, "staged": 2}
METHOD = {"lbfgs": 0, "fire": 1}


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


def build_id() -> str:
    """The source hash libss.so was compiled from (ss_build_id)."""
    return lib().ss_build_id().decode()


def check_build() -> None:
    """Raise if libss.so was not built from the sources next to it (a stale
    binary would silently run other kernels than the tree holds)."""
    from .build import source_hash

    have, want = build_id(), source_hash()
    if have != want:
        raise RuntimeError(f"{LIB_PATH} was built from sources {have}, the tree holds {want}: rebuild it with "
                           f"paper_2304_09139_amd.build.build()")


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


def uniform_positions(d: int, N: int, seed: int):
    """The library's seeded uniform start (ss_uniform_positions) as float64[2, d, N]."""
    import numpy as np

    out = np.empty((2, d, N), dtype=np.float64)
    _check(lib().ss_uniform_positions(d, N, seed & 0xFFFFFFFFFFFFFFFF, out.ctypes.data_as(ctypes.c_void_p)),
           what="ss_uniform_positions")
    return out


def cutoff(d: int, N: int, chi: float) -> tuple[int, int]:
    R2 = ctypes.c_int64()
    M = ctypes.c_int64()
    _check(lib().ss_cutoff(d, N, chi, ctypes.byref(R2), ctypes.byref(M)), what="ss_cutoff")
    return R2.value, M.value


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _need(t, device, dtype, shape, name: str):
    """Check a tensor handed to the library as a raw device pointer: on the
    context's device, of the expected dtype and shape, and contiguous (a host
    pointer would fault the GPU; another dtype or layout would be misread)."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, the context is on {device}")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _need_problem(ctx, w, n, v, pos):
    dev = ctx.device
    _need(n, dev, torch.int32, (w.M, w.d), "wavevectors n")
    if v is not None:
        _need(v, dev, torch.float64, (2, w.M), "weights v")
    _need(pos, dev, torch.float64, (2, w.d, w.N), "positions")


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


STATUS = {0: "converged", 1: "stalled", 2: "max_iter", 3: "numeric"}


def _min_opts(opts: dict) -> MinOpts:
    """MinOpts from the defaults updated by opts (precision and method by name or number)."""
    o = dict(DEFAULT_MIN_OPTS)
    o.update(opts)
    if isinstance(o["precision"], str):
        o["precision"] = PRECISION[o["precision"]]
    if isinstance(o["method"], str):
        o["method"] = METHOD[o["method"]]
    return MinOpts(**o)


def _result(r) -> dict:
    return dict(status=STATUS.get(r.status, str(r.status)), iters=r.iters, evals=r.evals, grad_evals=r.grad_evals,
                phi=(r.phi[0], r.phi[1]), smax=(r.smax[0], r.smax[1]), seconds=r.seconds,
                iters_fp64=r.iters_fp64, evals_fp64=r.evals_fp64)


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

    def __init__(self, device: int = 0, tiles: str | list | None = None):
        """tiles: None (built-in batched tile shapes), "tuned" (the measured table
        in tiles.json next to this module, if present) or a list of entries."""
        if not torch.cuda.is_available():
            raise RuntimeError("libss needs a HIP device; none is visible")
        check_build()
        self.device = torch.device("cuda", device)
        self._h = ctypes.c_void_p()
        _check(lib().ss_create(device, ctypes.byref(self._h)), what="ss_create")
        self._ws = None
        if tiles == "tuned":
            from .tune import load_tiles
            tiles = load_tiles()
        if tiles:
            self.set_tiles(tiles)

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

    def progress(self, seconds: float) -> None:
        """Print progress lines of long quenches to stderr at most every `seconds` (0: off)."""
        self._chk(lib().ss_set_progress(self._h, seconds), "ss_set_progress")

    KERNELS = {"nk": 0, "grad": 1, "table": 2}

    def profile(self, enable: bool = True, kernels=("nk", "grad", "table")) -> None:
        """Turn per-launch event timing of the named kernels on (or all timing off)."""
        mask = sum(1 << self.KERNELS[k] for k in kernels) if enable else 0
        self._chk(lib().ss_profile_enable(self._h, mask), "ss_profile_enable")

    def profile_read(self, kernel: str, reset: bool = True, work: bool = False):
        """(launches, total milliseconds[, work]) of one kernel since the last reset;
        work = pairs covered (passes) or table entries (table)."""
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        wk = ctypes.c_double()
        self._chk(lib().ss_profile_read(self._h, self.KERNELS[kernel], 1 if reset else 0, ctypes.byref(n),
                                        ctypes.byref(ms), ctypes.byref(wk)), "ss_profile_read")
        return (n.value, ms.value, wk.value) if work else (n.value, ms.value)

    def wavevectors(self, d: int, R2: int) -> torch.Tensor:
        M = ctypes.c_int64()
        self._chk(lib().ss_wavevectors(self._h, d, R2, None, 0, ctypes.byref(M), None), "ss_wavevectors")
        n = torch.empty((M.value, d), dtype=torch.int32, device=self.device)
        self._chk(lib().ss_wavevectors(self._h, d, R2, _ptr(n), M.value, ctypes.byref(M),
                                       _stream(self.device)), "ss_wavevectors")
        return n

    def weights(self, w: Workload, n: torch.Tensor) -> torch.Tensor:
        _need(n, self.device, torch.int32, (w.M, w.d), "wavevectors n")
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
                    grad: bool = True, nk: bool = False, out: dict | None = None, fp64: bool = False) -> dict:
        """Phi, S_max, optionally the gradient [2, d, N] and n~ [4, M] (device tensors);
        fp64=True runs the FP64 passes (results in the dd layout, zero low words)."""
        dev = self.device
        o = out if out is not None else {}
        if "phi" not in o:
            o["phi"] = torch.empty(2, dtype=torch.float64, device=dev)
            o["smax"] = torch.empty(2, dtype=torch.float64, device=dev)
        if grad and "grad" not in o:
            o["grad"] = torch.empty((2, w.d, w.N), dtype=torch.float64, device=dev)
        if nk and "nk" not in o:
            o["nk"] = torch.empty((4, w.M), dtype=torch.float64, device=dev)
        _need_problem(self, w, n, v, pos)
        for k, shape in (("phi", (2,)), ("smax", (2,)), ("grad", (2, w.d, w.N)), ("nk", (4, w.M))):
            if k in o and o[k] is not None:
                _need(o[k], dev, torch.float64, shape, f"output {k}")
        ws = self.workspace(w, 0)
        p = w.problem()
        fn = lib().ss_energy_grad_fp64 if fp64 else lib().ss_energy_grad
        self._chk(fn(self._h, ctypes.byref(p), _ptr(n), _ptr(v), _ptr(pos), _ptr(o["phi"]),
                     _ptr(o["smax"]), _ptr(o.get("grad") if grad else None),
                     _ptr(o.get("nk") if nk else None), _ptr(ws), ws.numel(),
                     _stream(dev)), "ss_energy_grad")
        return o

    def energy_grad_static(self, w: Workload, n: torch.Tensor, v: torch.Tensor | None, pos: torch.Tensor,
                           out: dict, grad: bool = True, nk: bool = False) -> dict:
        """ss_energy_grad_static: the evaluation of energy_grad in the library's
        static scratch (no allocation by the library).  The caller passes the
        outputs in `out` ("phi", "smax"[, "grad"][, "nk"], device float64) and
        has prepared the problem with workspace_size(w)."""
        dev = self.device
        _need_problem(self, w, n, v, pos)
        for k, shape in (("phi", (2,)), ("smax", (2,)), ("grad", (2, w.d, w.N)), ("nk", (4, w.M))):
            if k in ("phi", "smax") or (k == "grad" and grad) or (k == "nk" and nk):
                _need(out.get(k), dev, torch.float64, shape, f"output {k}")
        p = w.problem()
        self._chk(lib().ss_energy_grad_static(self._h, ctypes.byref(p), _ptr(n), _ptr(v), _ptr(pos),
                                              _ptr(out["phi"]), _ptr(out["smax"]),
                                              _ptr(out["grad"]) if grad else None,
                                              _ptr(out["nk"]) if nk else None, _stream(dev)),
                  "ss_energy_grad_static")
        return out

    def minimize(self, w: Workload, n: torch.Tensor, v: torch.Tensor | None, pos: torch.Tensor,
                 **opts) -> dict:
        """L-BFGS quench of pos (updated in place, [2, d, N]) on the device."""
        _need_problem(self, w, n, v, pos)
        mo = _min_opts(opts)
        res = MinResult()
        ws = self.workspace(w, 1)
        p = w.problem()
        self._chk(lib().ss_minimize(self._h, ctypes.byref(p), _ptr(n), _ptr(v), _ptr(pos), ctypes.byref(mo),
                                    ctypes.byref(res), _ptr(ws), ws.numel(), _stream(self.device)),
                  "ss_minimize")
        return _result(res)

    # ---- batches ---------------------------------------------------------------
    def set_tiles(self, tiles: list[dict]) -> None:
        """Replace the batched tile table: dicts with d, max_N, max_M, nk_chunk, grad_k."""
        arr = (Tile * max(len(tiles), 1))(*[Tile(t.get("d", 0), t["max_N"], t["max_M"], t["nk_chunk"],
                                                  t["grad_k"]) for t in tiles])
        self._chk(lib().ss_set_tiles(self._h, arr, len(tiles)), "ss_set_tiles")

    def get_tile(self, w: Workload) -> dict:
        t = Tile()
        p = w.problem()
        self._chk(lib().ss_get_tile(self._h, ctypes.byref(p), ctypes.byref(t)), "ss_get_tile")
        return dict(nk_chunk=t.nk_chunk, grad_k=t.grad_k)

    @staticmethod
    def _batch_args(works, opts_list):
        n = len(works)
        probs = (Problem * n)(*[w.problem() for w in works])
        mos = (MinOpts * n)(*[_min_opts(o) for o in opts_list])
        return probs, mos

    def batch_workspace_size(self, works: list[Workload], opts_list: list[dict]) -> int:
        probs, mos = self._batch_args(works, opts_list)
        b = ctypes.c_size_t()
        self._chk(lib().ss_batch_workspace_size(self._h, len(works), probs, mos, ctypes.byref(b)),
                  "ss_batch_workspace_size")
        return b.value

    def minimize_batch(self, works: list[Workload], positions: list[torch.Tensor],
                       weights: list[torch.Tensor | None] | None = None, opts: list[dict] | dict | None = None,
                       ws: torch.Tensor | None = None) -> list[dict]:
        """Quench many configurations together (positions updated in place)."""
        n = len(works)
        if len(positions) != n:
            raise ValueError("one position tensor per workload")
        if weights is not None and len(weights) != n:
            raise ValueError("one weight entry (tensor or None) per workload")
        for i, (w, x) in enumerate(zip(works, positions)):
            _need(x, self.device, torch.float64, (2, w.d, w.N), f"positions[{i}]")
            wt = None if weights is None else weights[i]
            if wt is not None:
                _need(wt, self.device, torch.float64, (2, w.M), f"weights[{i}]")
        if opts is None or isinstance(opts, dict):
            o = dict(DEFAULT_MIN_OPTS)
            o.update(opts or {})
            opts_list = [o] * n
        else:
            opts_list = []
            for x in opts:
                o = dict(DEFAULT_MIN_OPTS)
                o.update(x)
                opts_list.append(o)
        probs, mos = self._batch_args(works, opts_list)
        need = self.batch_workspace_size(works, opts_list)
        if ws is None:
            ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
        elif ws.device != self.device or not ws.is_contiguous():
            raise ValueError(f"the batch workspace must be a contiguous tensor on {self.device}")
        pos_arr = (_V * n)(*[p.data_ptr() for p in positions])
        v_arr = None
        if weights is not None:
            v_arr = (_V * n)(*[(v.data_ptr() if v is not None else None) for v in weights])
        res = (MinResult * n)()
        self._chk(lib().ss_minimize_batch(self._h, n, probs, v_arr, pos_arr, mos, res, _ptr(ws),
                                          ws.numel() * ws.element_size(), _stream(self.device)),
                  "ss_minimize_batch")
        return [_result(r) for r in res]

    # ---- serving -----------------------------------------------------------------
    def server_start(self, arena_bytes: int, max_slots: int = 256) -> None:
        """Start the continuous-batching server with a device arena of arena_bytes."""
        self._arena = torch.empty(arena_bytes, dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize()
        self._chk(lib().ss_server_start(self._h, _ptr(self._arena), arena_bytes, max_slots), "ss_server_start")

    def submit(self, w: Workload, pos=None, seed: int = 0, **opts) -> int:
        """Queue a quench of host positions pos (float64 [2, d, N]), or with pos
        None of the library's uniform start drawn from seed; returns its ticket."""
        import numpy as np

        if pos is None:
            p = None
            req = Request(w.d, w.N, w.R2, w.L, w.vkind, None, seed & 0xFFFFFFFFFFFFFFFF, _min_opts(opts))
        else:
            p = np.ascontiguousarray(pos, dtype=np.float64)
            if p.shape != (2, w.d, w.N):
                raise ValueError("positions must be [2, d, N]")
            req = Request(w.d, w.N, w.R2, w.L, w.vkind, p.ctypes.data, 0, _min_opts(opts))
        t = ctypes.c_uint64()
        self._chk(lib().ss_submit(self._h, ctypes.byref(req), ctypes.byref(t)), "ss_submit")
        self._served = getattr(self, "_served", {})
        self._served[t.value] = (w.d, w.N)
        return t.value

    def poll(self, ticket: int):
        """None while pending, else (result dict, final positions [2, d, N])."""
        import numpy as np

        d, N = self._served[ticket]
        out = np.empty((2, d, N), dtype=np.float64)
        res = MinResult()
        rc = lib().ss_poll(self._h, ticket, ctypes.byref(res), out.ctypes.data_as(ctypes.c_void_p))
        if rc == SS_PENDING:
            return None
        self._chk(rc, "ss_poll")
        del self._served[ticket]
        return _result(res), out

    def server_stats(self) -> dict:
        """Counters of the running server (ss_server_stats)."""
        st = ServerStats()
        self._chk(lib().ss_server_stats(self._h, ctypes.byref(st)), "ss_server_stats")
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def server_stop(self) -> None:
        rc = lib().ss_server_stop(self._h)
        self._arena = None
        self._chk(rc, "ss_server_stop")
