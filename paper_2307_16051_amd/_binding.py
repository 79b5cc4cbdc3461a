"""ctypes binding of libn3p (argument marshalling only).

Names follow the C ABI in include/n3p.h.  Tensors must be CUDA (HIP) tensors
on the current device; the binding passes their data pointers and the
current torch stream.  Workspaces are allocated with torch (the library never
allocates device memory).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import List, Optional

import torch

FP16, BF16, FP32, FP64 = 0, 1, 2, 3
IR, GMRES_IR, DIRECT = 0, 1, 2
SCALE_AUTO, SCALE_NONE = 0, 1
MAX_HIST = 64

_HERE = os.path.dirname(os.path.abspath(__file__))
# N3P_LIB: another build of the same sources (the sanitizer test loads a
# host-side AddressSanitizer build this way); there is no fallback
lib_path = os.environ.get("N3P_LIB") or os.path.join(_HERE, "libn3p.so")

if not os.path.exists(lib_path):
    raise ImportError(
        "the n3p library is not built (%s); run `python -c \"import __graft_entry__ as g; g.build()\"`"
        % lib_path)

lib = ctypes.CDLL(lib_path)

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_f64 = ctypes.c_double
_int = ctypes.c_int
_ip = ctypes.POINTER(ctypes.c_int)
_dp = ctypes.POINTER(ctypes.c_double)


class Options(ctypes.Structure):
    _fields_ = [("tau_r", _f64), ("tau_a", _f64), ("tau_abs_override", _f64), ("eta", _f64),
                ("maxit", _int), ("max_ir_sweeps", _int), ("gmres_restart", _int),
                ("gmres_tol", _f64), ("gmres_max_restarts", _int), ("scale_mode", _int),
                ("timing", _int), ("fft_residual", _int), ("matrix_free", _int),
                ("ir_scaled_half", _int)]

    @classmethod
    def default(cls, **kw) -> "Options":
        o = cls()
        lib.n3p_default_options(ctypes.byref(o))
        for k, v in kw.items():
            if not hasattr(o, k):
                raise AttributeError(k)
            setattr(o, k, v)
        return o


class _Report(ctypes.Structure):
    _fields_ = [("status", _int), ("its", _int), ("f0", _f64), ("fnorm", _f64),
                ("resid_rel", _f64 * MAX_HIST), ("lin_its", _int * MAX_HIST),
                ("lin_outer", _int * MAX_HIST), ("lin_fail", ctypes.c_uint8 * MAX_HIST),
                ("pivoted", ctypes.c_uint8 * MAX_HIST), ("lin_rel", _f64 * MAX_HIST),
                ("ms_jac", ctypes.c_float), ("ms_getrf", ctypes.c_float),
                ("ms_solve", ctypes.c_float), ("ms_resid", ctypes.c_float),
                ("ms_total", ctypes.c_float)]


RESID_FN = ctypes.CFUNCTYPE(_int, _vp, _vp, _vp, _i64, _vp)
JAC_FN = ctypes.CFUNCTYPE(_int, _vp, _vp, _vp, _i64, _i64, _vp)


class _Problem(ctypes.Structure):
    _fields_ = [("kind", _int), ("n", _i64), ("c", _f64), ("A", _vp), ("b", _vp), ("lda", _i64),
                ("residual", RESID_FN), ("jacobian", JAC_FN), ("ctx", _vp)]


@dataclasses.dataclass
class Report:
    status: int
    its: int
    f0: float
    fnorm: float
    resid_rel: List[float]
    lin_its: List[int]
    lin_outer: List[int]
    lin_fail: List[bool]
    pivoted: List[bool]
    lin_rel: List[float]
    ms_jac: float
    ms_getrf: float
    ms_solve: float
    ms_resid: float
    ms_total: float

    @classmethod
    def from_c(cls, r: _Report) -> "Report":
        k = r.its
        return cls(status=r.status, its=k, f0=r.f0, fnorm=r.fnorm,
                   resid_rel=list(r.resid_rel[: k + 1]), lin_its=list(r.lin_its[:k]),
                   lin_outer=list(r.lin_outer[:k]), lin_fail=[bool(v) for v in r.lin_fail[:k]],
                   pivoted=[bool(v) for v in r.pivoted[:k]], lin_rel=list(r.lin_rel[:k]),
                   ms_jac=r.ms_jac, ms_getrf=r.ms_getrf, ms_solve=r.ms_solve,
                   ms_resid=r.ms_resid, ms_total=r.ms_total)


class N3PError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__("%s: %s (%d)" % (where, status_str(status), status))
        self.status = status


def _setup():
    L = lib
    L.n3p_status_str.restype = ctypes.c_char_p
    L.n3p_status_str.argtypes = [_int]
    L.n3p_version.restype = ctypes.c_char_p
    L.n3p_default_options.argtypes = [ctypes.POINTER(Options)]
    L.n3p_default_options.restype = None
    L.n3p_problem_heq.argtypes = [ctypes.POINTER(_Problem), _i64, _f64]
    L.n3p_problem_dense_tanh.argtypes = [ctypes.POINTER(_Problem), _i64, _vp, _i64, _vp]
    L.n3p_problem_callbacks.argtypes = [ctypes.POINTER(_Problem), _i64, RESID_FN, JAC_FN, _vp]
    L.n3p_workspace_size.argtypes = [_i64, _int, _int, ctypes.POINTER(Options)]
    L.n3p_workspace_size.restype = ctypes.c_size_t
    L.n3p_solve.argtypes = [ctypes.POINTER(_Problem), _vp, _int, _int, ctypes.POINTER(Options),
                            _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_Report)]
    L.n3p_getrf_workspace_size.argtypes = [_i64, _int]
    L.n3p_getrf_workspace_size.restype = ctypes.c_size_t
    L.n3p_getrf.argtypes = [_int, _i64, _vp, _i64, _vp, _ip, _vp, ctypes.c_size_t, _vp]
    L.n3p_getrs.argtypes = [_int, _i64, _vp, _i64, _vp, _vp, _vp, ctypes.c_size_t, _vp]
    L.n3p_gemv_resid_f32.argtypes = [_i64, _vp, _i64, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
    L.n3p_heq_residual.argtypes = [_i64, _f64, _vp, _vp, _vp, _vp]
    L.n3p_heq_jacobian.argtypes = [_i64, _f64, _vp, _vp, _i64, _vp]
    L.n3p_linsolve_workspace_size.argtypes = [_i64, _int]
    L.n3p_linsolve_workspace_size.restype = ctypes.c_size_t
    L.n3p_ir.argtypes = [_int, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _vp, _vp, _f64, _int, _ip, _ip,
                         _dp, _vp, ctypes.c_size_t, _vp]
    L.n3p_ir_scaled_half.argtypes = L.n3p_ir.argtypes
    L.n3p_gmres_ir.argtypes = [_int, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _vp, _vp, _f64, _int,
                               _int, _f64, _ip, _ip, _ip, _dp, _vp, ctypes.c_size_t, _vp]
    L.n3p_mfma_rate_probe.argtypes = [_int, _int, _int, _vp, _dp, _vp]
    L.n3p_gemv_resid_f32_noalloc.argtypes = [_i64, _vp, _i64, _vp, _vp, _vp, _vp]
    for name in ("n3p_problem_heq", "n3p_problem_dense_tanh", "n3p_problem_callbacks",
                 "n3p_solve", "n3p_getrf", "n3p_getrs", "n3p_gemv_resid_f32",
                 "n3p_gemv_resid_f32_noalloc", "n3p_heq_residual",
                 "n3p_heq_jacobian", "n3p_ir", "n3p_ir_scaled_half", "n3p_gmres_ir",
                 "n3p_mfma_rate_probe"):
        getattr(L, name).restype = _int


_setup()

_TORCH_DT = {FP16: torch.float16, BF16: torch.bfloat16, FP32: torch.float32, FP64: torch.float64}


def status_str(st: int) -> str:
    return lib.n3p_status_str(st).decode()


def version() -> str:
    return lib.n3p_version().decode()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    return t.data_ptr()


def _ws(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def _check(st: int, where: str, ok=(0,)):
    if st not in ok:
        raise N3PError(st, where)
    return st


def workspace_size(n: int, prec: int = FP16, solver: int = IR, opts: Optional[Options] = None) -> int:
    return int(lib.n3p_workspace_size(n, prec, solver, ctypes.byref(opts) if opts else None))


def solve(problem: "_Problem", x: torch.Tensor, prec: int = FP16, solver: int = IR,
          opts: Optional[Options] = None, ws: Optional[torch.Tensor] = None,
          raise_on_error: bool = True) -> Report:
    """n3p_solve: x (FP64 device, length n) is the initial iterate and the result."""
    opts = opts or Options.default()
    n = problem.n
    if x.dtype != torch.float64 or x.numel() != n or not x.is_contiguous():
        raise ValueError("x must be a contiguous FP64 device tensor of length n")
    need = workspace_size(n, prec, solver, opts)
    if ws is None or ws.numel() < need:
        ws = _ws(need, x.device)
    rep = _Report()
    st = lib.n3p_solve(ctypes.byref(problem), _ptr(x), prec, solver, ctypes.byref(opts),
                       _ptr(ws), ws.numel(), _stream(), ctypes.byref(rep))
    if raise_on_error:
        _check(st, "n3p_solve", ok=(0, 1))
    return Report.from_c(rep)


def solve_heq(n: int, c: float, x: Optional[torch.Tensor] = None, prec: int = FP16,
              solver: int = IR, opts: Optional[Options] = None, device="cuda",
              ws: Optional[torch.Tensor] = None):
    """H-equation (eq. (3.2)) from x0 = ones unless x is given; returns (x, report)."""
    p = _Problem()
    _check(lib.n3p_problem_heq(ctypes.byref(p), n, c), "n3p_problem_heq")
    if x is None:
        x = torch.ones(n, dtype=torch.float64, device=device)
    rep = solve(p, x, prec, solver, opts, ws)
    return x, rep


def solve_dense_tanh(A: torch.Tensor, b: torch.Tensor, x: torch.Tensor, prec: int = FP16,
                     solver: int = IR, opts: Optional[Options] = None,
                     ws: Optional[torch.Tensor] = None):
    """F(x) = A x + 0.1 tanh(x) - b; A FP64 column-major (A.T contiguous) on the device."""
    n = x.numel()
    if A.dtype != torch.float64 or A.shape != (n, n) or A.stride() != (1, n):
        raise ValueError("A must be an n x n FP64 column-major device tensor")
    p = _Problem()
    _check(lib.n3p_problem_dense_tanh(ctypes.byref(p), n, _ptr(A), n, _ptr(b)),
           "n3p_problem_dense_tanh")
    rep = solve(p, x, prec, solver, opts, ws)
    return x, rep


def _colmajor(A: torch.Tensor):
    n = A.shape[0]
    if A.dim() != 2 or A.shape[1] != n or A.stride() != (1, n):
        raise ValueError("expected a square column-major tensor (A.T contiguous)")
    return n


def getrf(A: torch.Tensor, prec: Optional[int] = None):
    """n3p_getrf in place on a column-major device matrix; returns (ipiv, info)."""
    n = _colmajor(A)
    if prec is None:
        prec = {v: k for k, v in _TORCH_DT.items()}[A.dtype]
    ipiv = torch.empty(n, dtype=torch.int32, device=A.device)
    ws = _ws(lib.n3p_getrf_workspace_size(n, prec), A.device)
    info = ctypes.c_int(0)
    st = lib.n3p_getrf(prec, n, _ptr(A), n, _ptr(ipiv), ctypes.byref(info), _ptr(ws), ws.numel(),
                       _stream())
    _check(st, "n3p_getrf", ok=(0, -3, -4))
    return ipiv, info.value


def getrs(LU: torch.Tensor, ipiv: torch.Tensor, b: torch.Tensor, prec: Optional[int] = None):
    """n3p_getrs: b (FP32, or FP64 for FP64 factors) is overwritten by the solution."""
    n = _colmajor(LU)
    if prec is None:
        prec = {v: k for k, v in _TORCH_DT.items()}[LU.dtype]
    ws = _ws(lib.n3p_getrf_workspace_size(n, prec), LU.device)
    _check(lib.n3p_getrs(prec, n, _ptr(LU), n, _ptr(ipiv), _ptr(b), _ptr(ws), ws.numel(),
                         _stream()), "n3p_getrs")
    return b


def mfma_rate_probe(prec: int = FP16, blocks: int = 1024, iters: int = 256,
                    device="cuda"):
    """n3p_mfma_rate_probe on the current stream; returns (out, flops).  Every
    entry of `out` is 2*iters when the work was done; time it with events."""
    out = torch.empty(blocks * 256, dtype=torch.float32, device=device)
    flops = ctypes.c_double(0.0)
    _check(lib.n3p_mfma_rate_probe(prec, blocks, iters, _ptr(out), ctypes.byref(flops),
                                   _stream()), "n3p_mfma_rate_probe")
    return out, flops.value


def gemv_resid(A: torch.Tensor, u: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    n = _colmajor(A)
    r = torch.empty_like(b)
    ws = _ws(8 * max(256, n * ((n + 255) // 256)), A.device)
    _check(lib.n3p_gemv_resid_f32(n, _ptr(A), n, _ptr(u), _ptr(b), _ptr(r), _ptr(ws), ws.numel(),
                                  _stream()), "n3p_gemv_resid_f32")
    return r


GEMV_NOALLOC_MAX_N = 16384  # N3P_GEMV_NOALLOC_MAX_N


def gemv_resid_noalloc(A: torch.Tensor, u: torch.Tensor, b: torch.Tensor,
                       r: Optional[torch.Tensor] = None) -> torch.Tensor:
    """r = b - A u through n3p_gemv_resid_f32_noalloc (no workspace; the
    library's fixed scratch, n <= GEMV_NOALLOC_MAX_N)."""
    n = _colmajor(A)
    if r is None:
        r = torch.empty_like(b)
    _check(lib.n3p_gemv_resid_f32_noalloc(n, _ptr(A), n, _ptr(u), _ptr(b), _ptr(r), _stream()),
           "n3p_gemv_resid_f32_noalloc")
    return r


def heq_residual(x: torch.Tensor, c: float):
    n = x.numel()
    F = torch.empty_like(x)
    D = torch.empty_like(x)
    _check(lib.n3p_heq_residual(n, c, _ptr(x), _ptr(F), _ptr(D), _stream()), "n3p_heq_residual")
    return F, D


def heq_jacobian(D: torch.Tensor, c: float) -> torch.Tensor:
    n = D.numel()
    J = torch.empty((n, n), dtype=torch.float32, device=D.device).t()  # column-major
    _check(lib.n3p_heq_jacobian(n, c, _ptr(D), _ptr(J), n, _stream()), "n3p_heq_jacobian")
    return J


def _lin_args(A, LU, ipiv, colscale, prec):
    n = _colmajor(A)
    _colmajor(LU)
    if prec is None:
        prec = {v: k for k, v in _TORCH_DT.items()}[LU.dtype]
    return n, prec, _ptr(ipiv) if ipiv is not None else None, _ptr(colscale) if colscale is not None else None


def ir(A: torch.Tensor, LU: torch.Tensor, ipiv, b: torch.Tensor, u: torch.Tensor,
       tol: float = 1e-6, max_sweeps: int = 10, colscale=None, prec: Optional[int] = None,
       scaled_half: bool = False):
    """n3p_ir (scaled_half: n3p_ir_scaled_half, the corrections of eq. (2.19));
    returns (sweeps, failed, rel_res); u is updated in place."""
    n, prec, pp, cp = _lin_args(A, LU, ipiv, colscale, prec)
    ws = _ws(lib.n3p_linsolve_workspace_size(n, 1), A.device)
    sw, fl, rr = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    fn, name = (lib.n3p_ir_scaled_half, "n3p_ir_scaled_half") if scaled_half else (lib.n3p_ir, "n3p_ir")
    _check(fn(prec, n, _ptr(A), n, _ptr(LU), n, pp, cp, _ptr(b), _ptr(u), tol, max_sweeps,
              ctypes.byref(sw), ctypes.byref(fl), ctypes.byref(rr), _ptr(ws), ws.numel(),
              _stream()), name)
    return sw.value, bool(fl.value), rr.value


def gmres_ir(A: torch.Tensor, LU: torch.Tensor, ipiv, b: torch.Tensor, u: torch.Tensor,
             tol: float = 1e-6, max_outer: int = 10, m: int = 20, gmres_tol: float = 1e-4,
             colscale=None, prec: Optional[int] = None):
    """n3p_gmres_ir; returns (sweeps, gmres_its, failed, rel_res)."""
    n, prec, pp, cp = _lin_args(A, LU, ipiv, colscale, prec)
    ws = _ws(lib.n3p_linsolve_workspace_size(n, m), A.device)
    sw, gi, fl, rr = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    _check(lib.n3p_gmres_ir(prec, n, _ptr(A), n, _ptr(LU), n, pp, cp, _ptr(b), _ptr(u), tol,
                            max_outer, m, gmres_tol, ctypes.byref(sw), ctypes.byref(gi),
                            ctypes.byref(fl), ctypes.byref(rr), _ptr(ws), ws.numel(), _stream()),
           "n3p_gmres_ir")
    return sw.value, gi.value, bool(fl.value), rr.value


# ----------------------------------------------------------- batched engine
class EngineConfig(ctypes.Structure):
    _fields_ = [("max_slots", _int), ("max_n", _i64), ("lu_prec", _int), ("use_graphs", _int),
                ("leaf_grid", _int), ("gemm_grid", _int), ("gemm_kc", _int), ("vec_grid", _int)]

    @classmethod
    def default(cls, **kw) -> "EngineConfig":
        c = cls()
        lib.n3p_engine_default_config(ctypes.byref(c))
        for k, v in kw.items():
            if not hasattr(c, k):
                raise AttributeError(k)
            setattr(c, k, v)
        return c

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ServeStats(ctypes.Structure):
    _fields_ = [("p50_ms", _f64), ("p99_ms", _f64), ("mean_ms", _f64), ("max_ms", _f64),
                ("makespan_s", _f64), ("solves_per_s", _f64), ("max_active", _int),
                ("steps", _int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def _setup_engine():
    L = lib
    L.n3p_engine_default_config.argtypes = [ctypes.POINTER(EngineConfig)]
    L.n3p_engine_default_config.restype = None
    L.n3p_engine_request_bytes.argtypes = [_i64, _int]
    L.n3p_engine_request_bytes.restype = ctypes.c_size_t
    L.n3p_engine_fixed_bytes.argtypes = [_int]
    L.n3p_engine_fixed_bytes.restype = ctypes.c_size_t
    L.n3p_engine_create.argtypes = [ctypes.POINTER(_vp), ctypes.POINTER(EngineConfig),
                                    ctypes.POINTER(Options), _vp, ctypes.c_size_t, _vp]
    L.n3p_engine_destroy.argtypes = [_vp]
    L.n3p_engine_admit.argtypes = [_vp, _i64, _f64, _ip]
    L.n3p_engine_step.argtypes = [_vp, _ip]
    L.n3p_engine_slot_state.argtypes = [_vp, _int, _ip, _ip]
    L.n3p_engine_collect.argtypes = [_vp, _int, _vp, ctypes.POINTER(_Report)]
    L.n3p_engine_largest_free.argtypes = [_vp, ctypes.POINTER(ctypes.c_size_t)]
    L.n3p_engine_autotune.argtypes = [_vp, ctypes.POINTER(EngineConfig),
                                      ctypes.POINTER(ctypes.c_float), _ip]
    L.n3p_serve.argtypes = [ctypes.POINTER(EngineConfig), ctypes.POINTER(Options), _vp,
                            ctypes.c_size_t, _int, ctypes.POINTER(_i64), _dp, _dp, _vp,
                            ctypes.POINTER(_i64), _ip, _ip, _dp, ctypes.POINTER(ServeStats), _vp]
    for name in ("n3p_engine_create", "n3p_engine_destroy", "n3p_engine_admit", "n3p_engine_step",
                 "n3p_engine_slot_state", "n3p_engine_collect", "n3p_engine_largest_free",
                 "n3p_engine_autotune", "n3p_serve"):
        getattr(L, name).restype = _int


_setup_engine()

PHASE_FREE, PHASE_ADMITTED, PHASE_RUNNING, PHASE_DONE = 0, 1, 2, 3


def engine_request_bytes(n: int, prec: int = FP16) -> int:
    return int(lib.n3p_engine_request_bytes(n, prec))


def engine_fixed_bytes(max_slots: int) -> int:
    return int(lib.n3p_engine_fixed_bytes(max_slots))


class Engine:
    """n3p_engine: batched H-equation solves sharing one device pool (a torch tensor)."""

    def __init__(self, pool: torch.Tensor, cfg: Optional[EngineConfig] = None,
                 opts: Optional[Options] = None):
        self.cfg = cfg or EngineConfig.default()
        self.opts = opts or Options.default()
        self.pool = pool
        h = _vp()
        _check(lib.n3p_engine_create(ctypes.byref(h), ctypes.byref(self.cfg), ctypes.byref(self.opts),
                                     _ptr(pool), pool.numel() * pool.element_size(), _stream()),
               "n3p_engine_create")
        self._h = h

    def admit(self, n: int, c: float) -> Optional[int]:
        """Slot index, or None if no slot / pool space is free right now."""
        slot = _int(-1)
        st = lib.n3p_engine_admit(self._h, n, c, ctypes.byref(slot))
        if st == -2:
            return None
        _check(st, "n3p_engine_admit")
        return slot.value

    def step(self) -> int:
        nd = _int(0)
        _check(lib.n3p_engine_step(self._h, ctypes.byref(nd)), "n3p_engine_step")
        return nd.value

    def state(self, slot: int):
        ph, its = _int(0), _int(0)
        _check(lib.n3p_engine_slot_state(self._h, slot, ctypes.byref(ph), ctypes.byref(its)),
               "n3p_engine_slot_state")
        return ph.value, its.value

    def collect(self, slot: int, x_out: Optional[torch.Tensor]) -> Report:
        rep = _Report()
        _check(lib.n3p_engine_collect(self._h, slot, _ptr(x_out), ctypes.byref(rep)),
               "n3p_engine_collect")
        return Report.from_c(rep)

    def largest_free(self) -> int:
        v = ctypes.c_size_t(0)
        _check(lib.n3p_engine_largest_free(self._h, ctypes.byref(v)), "n3p_engine_largest_free")
        return v.value

    def autotune(self):
        best = EngineConfig()
        ms = (ctypes.c_float * 64)()
        nc = _int(0)
        _check(lib.n3p_engine_autotune(self._h, ctypes.byref(best), ms, ctypes.byref(nc)),
               "n3p_engine_autotune")
        self.cfg = best
        return best, list(ms[: nc.value])

    def close(self):
        if self._h:
            lib.n3p_engine_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def serve(ns, cs, arrivals, pool: torch.Tensor, cfg: Optional[EngineConfig] = None,
          opts: Optional[Options] = None, x_out: Optional[torch.Tensor] = None, x_off=None):
    """n3p_serve: continuous batching of H-equation requests; returns (its, status,
    latency_ms, stats dict).  x_out (FP64 device) receives each result at x_off[i]."""
    cfg = cfg or EngineConfig.default()
    opts = opts or Options.default()
    k = len(ns)
    n_a = (_i64 * k)(*[int(v) for v in ns])
    c_a = (_f64 * k)(*[float(v) for v in cs])
    t_a = (_f64 * k)(*[float(v) for v in arrivals])
    off_a = (_i64 * k)(*[int(v) for v in x_off]) if x_off is not None else None
    its = (_int * k)()
    status = (_int * k)()
    lat = (_f64 * k)()
    stats = ServeStats()
    st = lib.n3p_serve(ctypes.byref(cfg), ctypes.byref(opts), _ptr(pool),
                       pool.numel() * pool.element_size(), k, n_a, c_a, t_a, _ptr(x_out), off_a,
                       its, status, lat, ctypes.byref(stats), _stream())
    _check(st, "n3p_serve")
    return list(its), list(status), list(lat), stats.as_dict()


# ------------------------------------------------------ FFT form of eq. (3.2)
def _setup_fft():
    L = lib
    L.n3p_heq_fft_workspace_size.argtypes = [_i64]
    L.n3p_heq_fft_workspace_size.restype = ctypes.c_size_t
    L.n3p_heq_residual_fft.argtypes = [_i64, _f64, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
    L.n3p_heq_residual_fft.restype = _int
    L.n3p_heq_jv.argtypes = [_i64, _f64, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
    L.n3p_heq_jv.restype = _int


_setup_fft()


def heq_residual_fft(x: torch.Tensor, c: float):
    """(F, D) of eq. (3.2) by the O(N log N) FFT form (FP64 device tensors)."""
    n = x.numel()
    F = torch.empty_like(x)
    D = torch.empty_like(x)
    ws = _ws(lib.n3p_heq_fft_workspace_size(n), x.device)
    _check(lib.n3p_heq_residual_fft(n, c, _ptr(x), _ptr(F), _ptr(D), _ptr(ws), ws.numel(),
                                    _stream()), "n3p_heq_residual_fft")
    return F, D


def heq_jv(D: torch.Tensor, v: torch.Tensor, c: float) -> torch.Tensor:
    """J v for eq. (3.2) from the operator (FP64 compute, FP32 result)."""
    n = v.numel()
    y = torch.empty(n, dtype=torch.float32, device=v.device)
    ws = _ws(lib.n3p_heq_fft_workspace_size(n), v.device)
    _check(lib.n3p_heq_jv(n, c, _ptr(D), _ptr(v), _ptr(y), _ptr(ws), ws.numel(), _stream()),
           "n3p_heq_jv")
    return y
