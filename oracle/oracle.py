"""CPU oracle for Newton's method in three precisions (arXiv 2307.16051).

TEST INFRASTRUCTURE ONLY: the independent reference that the GPU library is
checked against.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the GPU
library and never imports it.

Two layers:

* ``liboracle.so`` (``n3p_oracle.c``): plain FP64 C -- the H-equation
  residual (Section 3, eq. (3.2)) and its analytic Jacobian, the dense tanh
  test problem, Gaussian elimination with partial pivoting, substitution,
  Newton's method (Algorithm 1.1, Section 1.1) with a double-precision LU,
  and Picard iteration.
* numpy functions in this module: the three-precision method itself,
  Algorithm 2.1 (Section 2) with iterative refinement (the IR algorithm of
  Section 2.2) or GMRES-IR (end of Section 2.2), in the precisions the paper
  names: residual FP64, Jacobian stored FP32 (eq. (2.1)), a half-precision
  copy (I_s^h, Section 2) that is factored, the correction equation solved
  in single precision.  This emulation exists to pin the algorithm's
  reading against the paper's printed histories (Tables 2 and 3, columns
  "IR 32-16" and "IR-GM").
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Callable, List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# N3P_ORACLE_LIB: another build of n3p_oracle.c (the sanitizer test loads an
# AddressSanitizer / UndefinedBehaviorSanitizer build this way)
_LIB_PATH = os.environ.get("N3P_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b  # noqa: WPS433 (local import on first use)
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    i64, f64, i32 = ctypes.c_int64, ctypes.c_double, ctypes.c_int
    lib.orc_heq_residual.argtypes = [i64, f64, _dp, _dp, _dp]
    lib.orc_heq_jacobian.argtypes = [i64, f64, _dp, _dp, i64]
    lib.orc_dense_tanh_residual.argtypes = [i64, _dp, i64, _dp, _dp, _dp]
    lib.orc_dense_tanh_jacobian.argtypes = [i64, _dp, i64, _dp, _dp, i64]
    lib.orc_nrm2.argtypes = [i64, _dp]
    lib.orc_nrm2.restype = f64
    lib.orc_gemv.argtypes = [i64, i64, _dp, i64, _dp, _dp]
    lib.orc_getrf.argtypes = [i64, _dp, i64, _ip]
    lib.orc_getrs.argtypes = [i64, _dp, i64, _ip, _dp]
    lib.orc_newton_heq.argtypes = [i64, f64, _dp, f64, f64, i32, i32, _dp,
                                   ctypes.POINTER(ctypes.c_int)]
    lib.orc_newton_dense_tanh.argtypes = [i64, _dp, i64, _dp, _dp, f64, f64, i32, i32, _dp,
                                          ctypes.POINTER(ctypes.c_int)]
    lib.orc_heq_picard.argtypes = [i64, f64, _dp, i32, f64]
    lib.orc_num_threads.argtypes = []
    for name in ("orc_heq_residual", "orc_heq_jacobian", "orc_dense_tanh_residual",
                 "orc_dense_tanh_jacobian", "orc_gemv", "orc_getrf", "orc_getrs",
                 "orc_newton_heq", "orc_newton_dense_tanh", "orc_heq_picard",
                 "orc_num_threads"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return int(_load().orc_num_threads())


# --------------------------------------------------------------------------
# Problems
# --------------------------------------------------------------------------

def heq_residual(x: np.ndarray, c: float, want_d: bool = False):
    """F(x) of eq. (3.2); optionally also D_i = 1 - (c/2N) sum_j x_j mu_i/(mu_i+mu_j)."""
    x = _f64(x)
    n = x.size
    F = np.empty(n)
    D = np.empty(n)
    rc = _load().orc_heq_residual(n, float(c), _p(x), _p(F), _p(D))
    if rc != 0:
        raise ValueError("orc_heq_residual failed (%d)" % rc)
    return (F, D) if want_d else F


def heq_jacobian(x: np.ndarray, c: float) -> np.ndarray:
    """Analytic Jacobian of eq. (3.2), FP64, returned as a Fortran-ordered array."""
    x = _f64(x)
    n = x.size
    J = np.empty((n, n), order="F")
    rc = _load().orc_heq_jacobian(n, float(c), _p(x), J.ctypes.data_as(_dp), n)
    if rc != 0:
        raise ValueError("orc_heq_jacobian failed (%d)" % rc)
    return J


def dense_tanh_residual(A: np.ndarray, b: np.ndarray, x: np.ndarray) -> np.ndarray:
    A = np.asfortranarray(A, dtype=np.float64)
    b, x = _f64(b), _f64(x)
    n = x.size
    F = np.empty(n)
    _load().orc_dense_tanh_residual(n, A.ctypes.data_as(_dp), n, _p(b), _p(x), _p(F))
    return F


def dense_tanh_jacobian(A: np.ndarray, x: np.ndarray) -> np.ndarray:
    A = np.asfortranarray(A, dtype=np.float64)
    x = _f64(x)
    n = x.size
    J = np.empty((n, n), order="F")
    _load().orc_dense_tanh_jacobian(n, A.ctypes.data_as(_dp), n, _p(x), J.ctypes.data_as(_dp), n)
    return J


# --------------------------------------------------------------------------
# Dense linear algebra (FP64)
# --------------------------------------------------------------------------

def getrf(A: np.ndarray):
    """Gaussian elimination with partial pivoting (ties to the lowest row).

    Returns (LU, ipiv, info): LU packs unit-lower L below the diagonal and U on
    and above it; ipiv is 0-based (row ipiv[k] was swapped with row k at step
    k); info = k+1 for the first exactly-zero pivot, else 0.
    """
    LU = np.array(A, dtype=np.float64, order="F", copy=True)
    n = LU.shape[0]
    ipiv = np.zeros(n, dtype=np.int32)
    info = _load().orc_getrf(n, LU.ctypes.data_as(_dp), n, ipiv.ctypes.data_as(_ip))
    if info < 0:
        raise ValueError("orc_getrf: NaN in the matrix")
    return LU, ipiv, int(info)


def getrs(LU: np.ndarray, ipiv: np.ndarray, b: np.ndarray) -> np.ndarray:
    LU = np.asfortranarray(LU, dtype=np.float64)
    x = np.array(b, dtype=np.float64, copy=True)
    n = x.size
    ipiv = np.ascontiguousarray(ipiv, dtype=np.int32)
    _load().orc_getrs(n, LU.ctypes.data_as(_dp), n, ipiv.ctypes.data_as(_ip), _p(x))
    return x


def perm_from_ipiv(ipiv: np.ndarray) -> np.ndarray:
    """Row order p such that (P A)[k] = A[p[k]], from sequential interchanges."""
    n = ipiv.size
    p = np.arange(n)
    for k in range(n):
        j = int(ipiv[k])
        if j != k:
            p[k], p[j] = p[j], p[k]
    return p


def gemv(A: np.ndarray, x: np.ndarray) -> np.ndarray:
    """y = A x in FP64 for an m x n matrix (the product inside the refinement
    residual r = b - A u of the IR algorithm, Section 2.2)."""
    A = np.asfortranarray(_f64(A))
    m, n = A.shape
    x = _f64(x)
    assert x.size == n
    y = np.zeros(m)
    _load().orc_gemv(m, n, _p(A), m, _p(x), _p(y))
    return y


def nrm2(v: np.ndarray) -> float:
    v = _f64(v)
    return float(_load().orc_nrm2(v.size, _p(v)))


# --------------------------------------------------------------------------
# Newton, Algorithm 1.1 (FP64 Jacobian and LU)
# --------------------------------------------------------------------------

@dataclasses.dataclass
class NewtonResult:
    x: np.ndarray            # iterate when the stopping rule was met
    its: int                 # Newton steps to meet ||F|| <= tau_r ||F0|| + tau_a
    hist: np.ndarray         # ||F(x_n)||_2, n = 0..its
    x_floor: Optional[np.ndarray] = None  # iterate driven to the rounding floor

    @property
    def rel_hist(self) -> np.ndarray:
        return self.hist / self.hist[0]


def newton_heq(n: int, c: float, x0=None, tau_r: float = 1e-10, tau_a: float = 0.0,
               maxit: int = 20, floor: bool = True) -> NewtonResult:
    """FP64 Newton on eq. (3.2) from x0 (default: ones)."""
    x = np.ones(n) if x0 is None else _f64(x0).copy()
    hist = np.zeros(maxit + 1)
    its_rule = ctypes.c_int(0)
    its = _load().orc_newton_heq(n, float(c), _p(x), tau_r, tau_a, maxit, 0, _p(hist),
                                 ctypes.byref(its_rule))
    if its < 0:
        raise RuntimeError("oracle Newton failed (%d)" % its)
    res = NewtonResult(x=x, its=int(its), hist=hist[: its + 1].copy())
    if floor:
        xf = x.copy()
        h2 = np.zeros(maxit + 1)
        r = _load().orc_newton_heq(n, float(c), _p(xf), 0.0, 0.0, 0, 4, _p(h2),
                                   ctypes.byref(its_rule))
        if r < 0:
            raise RuntimeError("oracle floor steps failed (%d)" % r)
        res.x_floor = xf
    return res


def newton_dense_tanh(A: np.ndarray, b: np.ndarray, x0, tau_r: float = 1e-10,
                      tau_a: float = 0.0, maxit: int = 20, floor: bool = True) -> NewtonResult:
    A = np.asfortranarray(A, dtype=np.float64)
    b = _f64(b)
    x = _f64(x0).copy()
    n = x.size
    hist = np.zeros(maxit + 1)
    its_rule = ctypes.c_int(0)
    its = _load().orc_newton_dense_tanh(n, A.ctypes.data_as(_dp), n, _p(b), _p(x), tau_r, tau_a,
                                        maxit, 0, _p(hist), ctypes.byref(its_rule))
    if its < 0:
        raise RuntimeError("oracle Newton failed (%d)" % its)
    res = NewtonResult(x=x, its=int(its), hist=hist[: its + 1].copy())
    if floor:
        xf = x.copy()
        h2 = np.zeros(maxit + 1)
        r = _load().orc_newton_dense_tanh(n, A.ctypes.data_as(_dp), n, _p(b), _p(xf), 0.0, 0.0,
                                          0, 4, _p(h2), ctypes.byref(its_rule))
        if r < 0:
            raise RuntimeError("oracle floor steps failed (%d)" % r)
        res.x_floor = xf
    return res


def heq_picard(n: int, c: float, maxit: int = 100000, tol: float = 1e-15, x0=None) -> np.ndarray:
    """Fixed point of x = 1/D(x) for eq. (3.2) by plain Picard sweeps."""
    x = np.ones(n) if x0 is None else _f64(x0).copy()
    k = _load().orc_heq_picard(n, float(c), _p(x), maxit, tol)
    if k < 0:
        raise RuntimeError("Picard did not converge in %d sweeps" % maxit)
    return x


def heq_mean_closed_form(c: float) -> float:
    """Mean of the discrete solution of eq. (3.2).

    Multiplying 1/x_i = D_i by x_i, averaging over i and symmetrising with
    mu_i/(mu_i+mu_j) + mu_j/(mu_i+mu_j) = 1 gives alpha - 1 = (c/4) alpha^2 for
    alpha = mean(x), whose root continuous in c from alpha(0)=1 is
    2 (1 - sqrt(1 - c)) / c.  Equivalently 1 - (c/2) alpha = sqrt(1 - c), the
    moment identity of the continuous equation (3.1).  Exact for every N.
    """
    if c == 0.0:
        return 1.0
    return 2.0 * (1.0 - np.sqrt(1.0 - c)) / c


# --------------------------------------------------------------------------
# Three-precision method, emulated with numpy dtypes
# --------------------------------------------------------------------------

_HALF = {"fp16": np.float16, "fp32": np.float32}


def round_half(A: np.ndarray, prec: str = "fp16") -> np.ndarray:
    """I_s^h: round an FP32 array to the factorisation precision (RNE).

    "fp16" is IEEE binary16; "fp32" leaves the FP32 Jacobian as it is (the
    two-precision method of Section 3.1 factors the single-precision matrix).
    """
    return np.asarray(A, dtype=np.float32).astype(_HALF[prec])


class HalfLU:
    """Factors of a half-precision matrix, stored in half precision.

    The matrix J_h is factored by the FP64 Gaussian elimination above (its
    entries are exact in FP64) and the factors L, U are then rounded to half
    precision: the stored factorisation is half precision, as in Section 2.
    Solves promote the stored factors to ``work`` precision (interprecision
    transfer on the fly, Section 2.3) and substitute in that precision.
    """

    def __init__(self, Jh: np.ndarray, prec: str = "fp16"):
        LU, ipiv, info = getrf(np.asarray(Jh, dtype=np.float64))
        if info != 0:
            raise np.linalg.LinAlgError("singular half-precision matrix (info=%d)" % info)
        self.prec = prec
        self.LU_h = LU.astype(_HALF[prec])
        self.ipiv = ipiv
        self.perm = perm_from_ipiv(ipiv)
        self.L = np.tril(self.LU_h.astype(np.float64), -1) + np.eye(LU.shape[0])
        self.U = np.triu(self.LU_h.astype(np.float64))

    def solve(self, r: np.ndarray, work=np.float32) -> np.ndarray:
        """U^{-1} L^{-1} P r with the half factors promoted to ``work``."""
        import scipy.linalg as sla  # a library substitution routine is a step, not the method
        L = self.L.astype(work)
        U = self.U.astype(work)
        y = sla.solve_triangular(L, np.asarray(r, dtype=work)[self.perm], lower=True,
                                 unit_diagonal=True, check_finite=False)
        return sla.solve_triangular(U, y, lower=False, check_finite=False).astype(work)

    def solve_half(self, r: np.ndarray) -> np.ndarray:
        """U^{-1} L^{-1} P I_s^h(r) held in the factor precision (Section 2.3).

        The correction of eq. (2.19) solves "entirely in the lower precision":
        the right-hand side is rounded to the factor precision, and forward
        then back substitution form each solution entry from the entries
        before it with the sum taken in FP64 and rounded once to the factor
        precision (the same single rounding per stored value as the
        factorisation), before later entries use it.  Returns FP32.
        """
        h = _HALF[self.prec]
        n = len(r)
        z = np.asarray(r, dtype=np.float32).astype(h).astype(np.float64)[self.perm]
        y = np.zeros(n)
        for i in range(n):
            y[i] = h(z[i] - self.L[i, :i] @ y[:i])
        x = np.zeros(n)
        for i in range(n - 1, -1, -1):
            x[i] = h((y[i] - self.U[i, i + 1:] @ x[i + 1:]) / self.U[i, i])
        return x.astype(np.float32)


@dataclasses.dataclass
class IRResult:
    u: np.ndarray
    sweeps: int
    failed: bool
    rel_res: float


def ir(A32: np.ndarray, b: np.ndarray, lu: HalfLU, max_sweeps: int = 10, tol: float = 1e-6,
       u0: Optional[np.ndarray] = None, scaled_half: bool = False) -> IRResult:
    """Iterative refinement (Section 2.2), with the stopping policy of Section 3.1.

    r = b - A u;  while ||r|| too large: d = U^{-1} L^{-1} r;  u += d;  r = b - A u.
    Success when ||r|| < tol ||b||; failure when ||r|| increases, in which case
    the iterate with the best residual is returned.  A, b, u, r, d are single
    precision; the factors are half precision promoted on the fly, or, with
    ``scaled_half``, each correction is eq. (2.19) (Section 2.3):
    d = ||r|| I_h^s(U^{-1} L^{-1} I_s^h(r / ||r||)), ||.|| the 2-norm.
    """
    A32 = np.asarray(A32, dtype=np.float32)
    b = np.asarray(b, dtype=np.float32)
    u = np.zeros_like(b) if u0 is None else np.asarray(u0, dtype=np.float32).copy()
    r = (b - A32 @ u).astype(np.float32)
    nb = float(np.linalg.norm(b.astype(np.float64)))
    rn = float(np.linalg.norm(r.astype(np.float64)))
    best_u, best_rn = u.copy(), rn
    sweeps = 0
    failed = False
    while rn >= tol * nb and sweeps < max_sweeps:
        if scaled_half and rn > 0:
            d = (rn * lu.solve_half((r.astype(np.float64) / rn).astype(np.float32))
                 .astype(np.float64)).astype(np.float32)
        else:
            d = lu.solve(r, np.float32)
        u = (u + d).astype(np.float32)
        r = (b - A32 @ u).astype(np.float32)
        sweeps += 1
        rn_new = float(np.linalg.norm(r.astype(np.float64)))
        if rn_new > rn:
            failed = True
            if rn_new < best_rn:
                best_u, best_rn = u.copy(), rn_new
            break
        rn = rn_new
        if rn < best_rn:
            best_u, best_rn = u.copy(), rn
    if not failed and rn >= tol * nb:
        failed = True
    return IRResult(u=best_u, sweeps=sweeps, failed=failed, rel_res=best_rn / nb if nb else 0.0)


def gmres_lp(apply_A: Callable[[np.ndarray], np.ndarray], prec: Callable[[np.ndarray], np.ndarray],
             r: np.ndarray, m: int = 20, rtol: float = 1e-4, max_restarts: int = 10):
    """Left-preconditioned restarted GMRES(m) with modified Gram-Schmidt.

    Solves M^{-1} A d = M^{-1} r from d = 0 (GMRES-IR, end of Section 2.2),
    stopping when the preconditioned residual falls below rtol times its
    initial value.  Single precision vectors; Givens rotations in FP64.
    Returns (d, iterations).
    """
    n = r.size
    d = np.zeros(n, dtype=np.float32)
    z0 = prec(r).astype(np.float32)
    beta0 = float(np.linalg.norm(z0.astype(np.float64)))
    if beta0 == 0.0:
        return d, 0
    total = 0
    z = z0
    for _ in range(max_restarts):
        beta = float(np.linalg.norm(z.astype(np.float64)))
        if beta <= rtol * beta0:
            break
        V = np.zeros((m + 1, n), dtype=np.float32)
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = (z / beta).astype(np.float32)
        k_used = 0
        for j in range(m):
            w = prec(apply_A(V[j])).astype(np.float32)
            for i in range(j + 1):          # modified Gram-Schmidt
                H[i, j] = float(np.dot(V[i].astype(np.float64), w.astype(np.float64)))
                w = (w - np.float32(H[i, j]) * V[i]).astype(np.float32)
            H[j + 1, j] = float(np.linalg.norm(w.astype(np.float64)))
            if H[j + 1, j] > 0.0:
                V[j + 1] = (w / np.float32(H[j + 1, j])).astype(np.float32)
            for i in range(j):              # apply previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = (1.0, 0.0) if den == 0.0 else (H[j, j] / den, H[j + 1, j] / den)
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k_used = j + 1
            total += 1
            if abs(g[j + 1]) <= rtol * beta0 or H[j, j] == 0.0:
                break
        y = np.zeros(k_used)
        for i in range(k_used - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k_used] @ y[i + 1:k_used]) / H[i, i]
        d = (d + (V[:k_used].astype(np.float64).T @ y).astype(np.float32)).astype(np.float32)
        z = prec((r - apply_A(d)).astype(np.float32)).astype(np.float32)
        if abs(g[k_used]) <= rtol * beta0:
            break
    return d, total


def gmres_ir(A32: np.ndarray, b: np.ndarray, lu: HalfLU, max_outer: int = 10, tol: float = 1e-6,
             m: int = 20, gmres_tol: float = 1e-4) -> IRResult:
    """IR whose correction d solves the left-preconditioned system with GMRES."""
    A32 = np.asarray(A32, dtype=np.float32)
    b = np.asarray(b, dtype=np.float32)
    u = np.zeros_like(b)
    r = b.copy()
    nb = float(np.linalg.norm(b.astype(np.float64)))
    rn = nb
    best_u, best_rn = u.copy(), rn
    sweeps = 0
    failed = False

    def apply_A(v):
        return (A32 @ np.asarray(v, dtype=np.float32)).astype(np.float32)

    def prec(v):
        return lu.solve(v, np.float32)

    while rn >= tol * nb and sweeps < max_outer:
        d, _ = gmres_lp(apply_A, prec, r, m=m, rtol=gmres_tol)
        u = (u + d).astype(np.float32)
        r = (b - A32 @ u).astype(np.float32)
        sweeps += 1
        rn_new = float(np.linalg.norm(r.astype(np.float64)))
        if rn_new > rn:
            failed = True
            if rn_new < best_rn:
                best_u, best_rn = u.copy(), rn_new
            break
        rn = rn_new
        if rn < best_rn:
            best_u, best_rn = u.copy(), rn
    if not failed and rn >= tol * nb:
        failed = True
    return IRResult(u=best_u, sweeps=sweeps, failed=failed, rel_res=best_rn / nb if nb else 0.0)


@dataclasses.dataclass
class Newton3pResult:
    x: np.ndarray
    its: int
    hist: np.ndarray
    lin_its: List[int]
    lin_fail: List[bool]

    @property
    def rel_hist(self) -> np.ndarray:
        return self.hist / self.hist[0]


def newton3p(resid: Callable[[np.ndarray], np.ndarray], jac: Callable[[np.ndarray], np.ndarray],
             x0: np.ndarray, tau_r: float = 1e-10, tau_a: float = 0.0, maxit: int = 20,
             solver: str = "ir", prec: str = "fp16", eta: float = 1e-6,
             max_sweeps: int = 10, gmres_m: int = 20, gmres_tol: float = 1e-4) -> Newton3pResult:
    """Algorithm 2.1 (newton3p), Section 2.

    F in FP64; J = F'(x) stored in FP32 (eq. (2.1)); J_h = I_s^h(J) factored in
    half precision; the step equation is scaled to unit norm before it is
    handed to the linear solver (eqs. (2.17)-(2.18)): solve J u = -F/||F|| to
    relative residual ``eta`` by IR or GMRES-IR, then s = ||F|| u in FP64.

    ``solver="direct"`` is the two-precision method of Section 3.1 (the
    F32 and F16 columns of Tables 2 and 3): the step is one solve with the
    stored low-precision factors, promoted to FP32, with no refinement.
    """
    x = np.array(x0, dtype=np.float64, copy=True)
    F = resid(x)
    fn = float(np.linalg.norm(F))
    hist = [fn]
    tau = tau_r * fn + tau_a
    lin_its, lin_fail = [], []
    its = 0
    while fn > tau and its < maxit:
        J32 = np.asarray(jac(x), dtype=np.float32)
        lu = HalfLU(round_half(J32, prec), prec)
        b = (-F / fn).astype(np.float32)
        if solver == "ir":
            res = ir(J32, b, lu, max_sweeps=max_sweeps, tol=eta)
        elif solver == "direct":
            u = lu.solve(b, np.float32)
            res = IRResult(u=u, sweeps=1, failed=False, rel_res=0.0)
        elif solver == "gmres":
            res = gmres_ir(J32, b, lu, max_outer=max_sweeps, tol=eta, m=gmres_m,
                           gmres_tol=gmres_tol)
        else:
            raise ValueError(solver)
        lin_its.append(res.sweeps)
        lin_fail.append(res.failed)
        x = x + fn * res.u.astype(np.float64)
        F = resid(x)
        fn = float(np.linalg.norm(F))
        hist.append(fn)
        its += 1
    return Newton3pResult(x=x, its=its, hist=np.array(hist), lin_its=lin_its, lin_fail=lin_fail)
