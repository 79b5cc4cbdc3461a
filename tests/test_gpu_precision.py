"""LU precision comparison and the two-precision columns, against the oracle.

* FP16 / BF16 / FP32 LU with iterative refinement and the FP64-LU Newton
  baseline on the H-equation (eq. (3.2)) at N = 4096 and N = 16384 with
  c in {0.5, 0.9, 0.99}; GMRES-IR on the ill-conditioned cases N = 8192,
  c in {0.9999, 0.99999}.  Acceptance: relative error of the final iterate
  against the oracle's solution <= 1e-9 and the oracle's FP64 Newton
  iteration count or one more.  The oracle's FP64 Newton results at these
  sizes are stored in tests/golden/oracle_heq_*.txt (written by
  tests/golden/make_heq_large.py, oracle only); the full reference vector
  is the oracle's Picard fixed point, checked against the stored samples.
* Two-precision Newton (Section 3.1, the F32 column of Tables 2 and 3): the
  FP32 Jacobian factored in FP32 and one solve per step reproduces the
  printed histories.  The F16 column is parity unpinned (the paper's LU rounds
  every operation to half precision); the FP16 one-solve method is checked
  against the oracle's emulation instead.
* Dense tanh system: error against x* = 1 and the oracle's count on the
  identical matrix (N = 1024); at N = 16384 the error against x* = 1 (a
  property that holds at any size).  Gated where the theory promises
  convergence (see `gated`), reported otherwise.
"""
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from workloads import dense_tanh_system, dense_tanh_system_torch

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_heq_large as G  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2307_16051_amd as n3p
    assert torch.cuda.is_available()
    return n3p, torch


_REF = {}


def reference(n, c):
    """(x_ref, oracle its, golden dict) for the H-equation at (n, c)."""
    if (n, c) not in _REF:
        g = G.read(n, c)
        xr = O.heq_picard(n, c, tol=1e-15)
        d = np.abs(xr[g["idx"]] - g["x"]).max() / np.abs(g["x"]).max()
        # The stored iterate is at the rounding floor, or (kind "rule") only
        # within the stopping rule ||F|| <= 1e-10 ||F0|| of the solution.
        # Picard stops on small increments; its remaining error is about the
        # increment over (1 - contraction rate), which grows as c -> 1
        # (~1e-11 at c = 0.99999): still far below the 1e-9 acceptance bar.
        assert d < (1e-10 if g["kind"] == "floor" else 1e-8), \
            "Picard and Newton oracle solutions differ: %g" % d
        _REF[(n, c)] = (xr, g["its"], g)
    return _REF[(n, c)]


def rel_err(x, ref):
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))


def solve(n3p, torch, n, c, prec, solver, **kw):
    opts = n3p.Options.default(**kw)
    x, rep = n3p.solve_heq(n, c, prec=getattr(n3p, prec), solver=getattr(n3p, solver), opts=opts)
    return x.cpu().numpy(), rep


@pytest.mark.parametrize("c", [0.5, 0.9, 0.99])
@pytest.mark.parametrize("prec,solver", [("FP16", "IR"), ("BF16", "IR"), ("FP32", "IR"),
                                         ("FP64", "DIRECT")])
def test_precision_sweep_n4096(env, c, prec, solver):
    n3p, torch = env
    n = 4096
    print("case precision n=%d c=%g %s %s" % (n, c, prec, solver), flush=True)
    xr, its_ref, _ = reference(n, c)
    x, rep = solve(n3p, torch, n, c, prec, solver)
    err = rel_err(x, xr)
    print("  its=%d (oracle %d) err=%.2e lin=%s" % (rep.its, its_ref, err, rep.lin_its), flush=True)
    assert rep.status == 0
    assert rep.its in (its_ref, its_ref + 1)
    assert err <= 1e-9


@pytest.mark.parametrize("c", [0.5, 0.9, 0.99])
@pytest.mark.parametrize("prec,solver", [("FP16", "IR"), ("BF16", "IR"), ("FP32", "IR"),
                                         ("FP64", "DIRECT")])
def test_full_size_n16384(env, c, prec, solver):
    """The benchmark size: whole-vector parity with the oracle solution."""
    n3p, torch = env
    n = 16384
    print("case full-size n=%d c=%g %s %s" % (n, c, prec, solver), flush=True)
    xr, its_ref, g = reference(n, c)
    x, rep = solve(n3p, torch, n, c, prec, solver)
    err = rel_err(x, xr)
    print("  its=%d (oracle %d) err=%.2e" % (rep.its, its_ref, err), flush=True)
    assert rep.status == 0
    assert rep.its in (its_ref, its_ref + 1)
    assert err <= 1e-9
    # sampled entries against the stored oracle Newton iterate (which itself
    # meets the stopping rule: agreement to the rule's accuracy)
    samp = np.abs(x[g["idx"]] - g["x"]).max() / np.abs(g["x"]).max()
    assert samp <= (1e-9 if g["kind"] == "floor" else 1e-8)
    # the moment identity holds exactly for the discrete system
    assert abs(x.mean() - O.heq_mean_closed_form(c)) <= 1e-9


@pytest.mark.parametrize("c,min_frac", [(0.5, 0.99), (0.99, 0.5)])
def test_unscaled_fp16_copy_n16384(env, c, min_frac):
    """Section 1.2 and Table 1: with no column scaling (SCALE_NONE) the FP16
    copy of the N = 16384 Jacobian holds most off-diagonal entries,
    (c/(2N)) mu_i/(mu_i+mu_j) x_i^2, as subnormals (below 2^-14 ~ 6.1e-5),
    spaced 2^-24 apart: all of them at c = 0.5, over half at c = 0.99.
    Rounding costs at most 2^-25 per entry, so ||J_h - J||_2 <= ||J_h - J||_F
    <= N 2^-25 ~ 5e-4 -- small against 1/||J^{-1}|| for these c -- and IR must
    still converge in the oracle's count."""
    n3p, torch = env
    n = 16384
    print("case unscaled fp16 copy n=%d c=%g" % (n, c), flush=True)
    xr, its_ref, _ = reference(n, c)
    # the premise: most off-diagonal entries of J(x*) are FP16 subnormals
    F, D = n3p.heq_residual(torch.from_numpy(xr).cuda(), c)
    J = n3p.heq_jacobian(D, c)
    off = J.abs()
    off.diagonal().fill_(0.0)
    frac = float(((off < 2.0 ** -14) & (off > 0)).sum().item()) / (n * n - n)
    print("  subnormal fraction of the off-diagonal %.4f" % frac, flush=True)
    assert frac > min_frac
    del J, off
    x, rep = solve(n3p, torch, n, c, "FP16", "IR", scale_mode=n3p.SCALE_NONE)
    err = rel_err(x, xr)
    print("  its=%d (oracle %d) err=%.2e lin=%s" % (rep.its, its_ref, err, rep.lin_its), flush=True)
    assert rep.status == 0
    assert rep.its in (its_ref, its_ref + 1)
    assert err <= 1e-9


@pytest.mark.parametrize("n,c", [(4096, 0.99), (16384, 0.9)])
def test_scaled_half_corrections_newton(env, n, c):
    """Newton with the IR corrections of eq. (2.19): Section 2.3 expects the
    nonlinear iteration to be unchanged by the way precision is transferred,
    so the oracle's count (or one more) and its solution."""
    n3p, torch = env
    print("case scaled-half IR n=%d c=%g" % (n, c), flush=True)
    xr, its_ref, _ = reference(n, c)
    x, rep = solve(n3p, torch, n, c, "FP16", "IR", ir_scaled_half=1)
    err = rel_err(x, xr)
    print("  its=%d (oracle %d) err=%.2e lin=%s" % (rep.its, its_ref, err, rep.lin_its), flush=True)
    assert rep.status == 0
    assert rep.its in (its_ref, its_ref + 1)
    assert err <= 1e-9


@pytest.mark.parametrize("c", [0.9999, 0.99999])
@pytest.mark.parametrize("prec,solver", [("FP16", "GMRES_IR"), ("BF16", "GMRES_IR"),
                                         ("FP64", "DIRECT")])
def test_ill_conditioned_n8192(env, c, prec, solver):
    n3p, torch = env
    n = 8192
    print("case ill-conditioned n=%d c=%g %s %s" % (n, c, prec, solver), flush=True)
    xr, its_ref, _ = reference(n, c)
    x, rep = solve(n3p, torch, n, c, prec, solver)
    err = rel_err(x, xr)
    print("  its=%d (oracle %d) err=%.2e lin=%s fail=%s" % (rep.its, its_ref, err, rep.lin_its,
                                                         rep.lin_fail), flush=True)
    assert rep.status == 0
    assert rep.its in (its_ref, its_ref + 1)
    assert err <= 1e-9


@pytest.mark.parametrize("c", [0.9999, 0.99999])
def test_plain_ir_on_ill_conditioned_reported(env, c):
    """Plain IR at N = 8192 near c = 1: reported next to GMRES-IR, not gated
    on converging (Table 3 shows IR stagnating there).  What the report says
    must hold: a finite iterate; success means the oracle's accuracy within
    one Newton step of its count; failure means the step limit (20) was
    reached; no linear solve takes more than the sweep limit (10)."""
    n3p, torch = env
    n = 8192
    xr, its_ref, _ = reference(n, c)
    x, rep = solve(n3p, torch, n, c, "FP16", "IR")
    err = rel_err(x, xr)
    print("  IR its=%d (oracle %d) err=%.2e status=%d lin=%s fail=%s" % (
        rep.its, its_ref, err, rep.status, rep.lin_its, rep.lin_fail), flush=True)
    assert rep.status in (0, 1)
    assert np.all(np.isfinite(x))
    assert len(rep.lin_its) == len(rep.lin_fail) == rep.its
    assert all(1 <= k <= 10 for k in rep.lin_its)
    if rep.status == 0:
        assert rep.its in (its_ref, its_ref + 1)
        assert err <= 1e-9
    else:
        assert rep.its == 20


@pytest.mark.parametrize("tab,c,k", [("table2", 0.99, 5), ("table3", 0.9999, 8)])
def test_two_precision_f32_column_matches_table(env, request, tab, c, k):
    """Tables 2 and 3, F32 column: FP32 Jacobian, FP32 LU, one solve per step."""
    n3p, torch = env
    table = request.getfixturevalue(tab)
    x, rep = solve(n3p, torch, 4096, c, "FP32", "DIRECT", tau_r=1e-9)
    expect = [v for v in table["F32"] if v is not None]
    print("  its=%d hist=%s" % (rep.its, ["%.3e" % v for v in rep.resid_rel]), flush=True)
    assert rep.its == len(expect) - 1 == k
    got = [float("%.3e" % v) for v in rep.resid_rel]
    assert got[:k] == expect[:k]
    assert abs(rep.resid_rel[k] / expect[k] - 1.0) < 0.02


@pytest.mark.parametrize("prec", ["fp16", "fp32"])
def test_two_precision_tracks_oracle_emulation(env, prec):
    """One solve per step with FP16 (or FP32) factors against the oracle's
    emulation of the same method at N = 1024, c = 0.99."""
    n3p, torch = env
    n, c = 1024, 0.99
    R = lambda x: O.heq_residual(x, c)
    Jf = lambda x: O.heq_jacobian(x, c)
    ref = O.newton3p(R, Jf, np.ones(n), solver="direct", prec=prec)
    x, rep = solve(n3p, torch, n, c, prec.upper(), "DIRECT")
    print("  its=%d (emulation %d) hist=%s" % (rep.its, ref.its,
          ["%.3e" % v for v in rep.resid_rel]), flush=True)
    assert rep.status == 0
    assert abs(rep.its - ref.its) <= 1
    # Both factorisations are O(u) perturbations of J (u = 2^-11 for FP16),
    # but different ones: the GPU rounds column-scaled entries and
    # accumulates block updates in FP32 (in an order set by the blocking),
    # the emulation rounds the exact factors once.  The one-solve iteration
    # converges linearly at a rate proportional to that perturbation, so its
    # residuals agree only to the perturbation's relative size: a few percent
    # by the third step for FP16.
    rtol = 1e-1 if prec == "fp16" else 1e-3
    np.testing.assert_allclose(rep.resid_rel[1:4], ref.rel_hist[1:4], rtol=rtol)
    xr = O.heq_picard(n, c, tol=1e-15)
    assert rel_err(x, xr) <= 1e-9


def factor_errors(n3p, torch, n, cond, prec, steps=60):
    """For the factors n3p_getrf forms from the dense tanh matrix A of this
    size and condition, rounded to `prec` (E = P A - L U, in FP64 on the
    device):
    * eps_2 = ||E||_2 / ||A||_2, the normwise backward error;
    * rho = ||A^{-1} P^T E||_2 = ||(P A)^{-1} E||_2 (rho <= cond eps_2,
      since ||A||_2 = cond and ||A^{-1}||_2 = 1 by construction);
    * mu = ||(L U)^{-1} E||_2 = ||I - (L U)^{-1} P A||_2, the norm of the IR
      iteration matrix of Section 2.2 (mu <= rho / (1 - rho) for rho < 1).
    The 2-norms are estimated by power steps on B^T B (B = E; A^{-1} P^T E
    through an FP64 LU of A; U^{-1} L^{-1} E with the stored factors)."""
    if n <= 1024:
        A_np, _, _ = dense_tanh_system(n, cond)
        A = torch.from_numpy(np.ascontiguousarray(A_np.T)).cuda().t()
    else:
        A, _, _ = dense_tanh_system_torch(n, cond, "cuda")
    dt = {"FP16": torch.float16, "BF16": torch.bfloat16}[prec]
    T = A.t().to(dt).t()  # column-major copy in the factor precision
    ipiv, info = n3p.getrf(T)
    assert info == 0
    p = torch.from_numpy(O.perm_from_ipiv(ipiv.cpu().numpy())).cuda()
    F = T.double()
    del T
    L = torch.tril(F, -1)
    L.diagonal().fill_(1.0)
    U = torch.triu(F)
    del F
    E = A[p] - L @ U
    g = torch.Generator(device="cuda").manual_seed(11)

    def norm2(bmul, btmul):
        v = torch.randn(n, dtype=torch.float64, device="cuda", generator=g)
        v /= v.norm()
        for _ in range(steps):
            w = btmul(bmul(v))
            v = w / w.norm()
        return float(bmul(v).norm().item())

    eps2 = norm2(lambda v: E @ v, lambda y: E.t() @ y) / cond
    tri = torch.linalg.solve_triangular

    def mmul(v):  # U^{-1} L^{-1} E v
        y = tri(L, (E @ v)[:, None], upper=False, unitriangular=True)
        return tri(U, y, upper=True)[:, 0]

    def mtmul(y):  # E^T L^{-T} U^{-T} y
        z = tri(U.t(), y[:, None], upper=False)
        return E.t() @ tri(L.t(), z, upper=True, unitriangular=True)[:, 0]

    mu = norm2(mmul, mtmul)
    del L, U
    LUa, pa = torch.linalg.lu_factor(A)
    del A

    def bmul(v):  # A^{-1} P^T E v
        q = torch.zeros_like(v)
        q[p] = E @ v
        return torch.linalg.lu_solve(LUa, pa, q[:, None])[:, 0]

    def btmul(y):  # E^T P A^{-T} y
        z = torch.linalg.lu_solve(LUa, pa, y[:, None], adjoint=True)[:, 0]
        return E.t() @ z[p]

    rho = norm2(bmul, btmul)
    del E, LUa
    return eps2, rho, mu


# Measured by test_dense_tanh_factor_errors on the device (deterministic
# factorisation of seeded matrices) and stated here, rounded up by ~5%:
# (eps_2, rho, mu) per (precision, N, cond).  The gate is derived from mu.
ERR_BOUND = {
    ("FP16", 1024, 1e2): (3.0e-3, 0.11, 0.11), ("FP16", 1024, 1e4): (1.0e-3, 3.0, 6.5),
    ("BF16", 1024, 1e2): (2.1e-2, 0.77, 0.87), ("BF16", 1024, 1e4): (8.6e-3, 25.0, 3.2e3),
    ("FP16", 16384, 1e2): (9.0e-3, 0.37, 0.38), ("FP16", 16384, 1e4): (3.8e-3, 11.0, 1.24e4),
    ("BF16", 16384, 1e2): (7.2e-2, 3.0, 15.5), ("BF16", 16384, 1e4): (3.0e-2, 92.0, 5.3e4),
}


def gated(prec, solver, cond, n=1024):
    """Whether the theory promises convergence at this condition number.

    Section 2.2: IR is a stationary iteration with iteration matrix
    M = I - (L U)^{-1} P A; it converges when the low-precision factors
    approximate the matrix well against its conditioning (eq. (2.14) bounds
    this in the worst case by 3 N u_h cond(A) < 1).  Here ||M||_2 = mu is
    measured (ERR_BOUND, the factors of A standing in for those of the
    Jacobian A + 0.1 diag(sech^2 x), which differs from A by that diagonal):
    * IR: ten sweeps reach the 1e-6 target when mu^10 <= 1e-6, mu <= 0.25;
    * GMRES-IR: the preconditioned matrix is I - M, and the polynomial
      (1 - z)^20 bounds the residual reduction of one GMRES(20) cycle by
      mu^20, so its 1e-4 target is met within the ten cycles for mu <= 0.7.
    The normwise products are looser: mu <= rho / (1 - rho) with
    rho = ||(PA)^{-1} E||_2 <= cond eps_2 (E = P A - L U), and cond eps_2
    overstates rho about threefold here (A^{-1} amplifies only E's component
    along A's few smallest singular directions), so gating on it would
    exclude runs that provably converge.  Outside these ranges runs are
    reported, not gated.
    """
    if prec == "FP64":
        return True
    key = (prec, n, cond)
    if key not in ERR_BOUND:
        return False
    mu = ERR_BOUND[key][2]
    return mu <= (0.25 if solver == "IR" else 0.7)


@pytest.mark.parametrize("n", [1024, 16384])
@pytest.mark.parametrize("cond", [1e2, 1e4])
@pytest.mark.parametrize("prec", ["FP16", "BF16"])
def test_dense_tanh_factor_errors(env, n, cond, prec):
    """The measured quantities the gate rests on, against their stated bounds."""
    n3p, torch = env
    print("case dense factor errors n=%d cond=%g %s" % (n, cond, prec), flush=True)
    eps2, rho, mu = factor_errors(n3p, torch, n, cond, prec)
    be, br, bm = ERR_BOUND[(prec, n, cond)]
    print("  eps_2 = %.3e (bound %.1e)  cond*eps_2 = %.3e  rho = %.3e (bound %.1e)  "
          "mu = %.3e (bound %.2g)  gated IR %s GMRES-IR %s" % (
              eps2, be, cond * eps2, rho, br, mu, bm,
              gated(prec, "IR", cond, n), gated(prec, "GMRES_IR", cond, n)), flush=True)
    assert eps2 <= be
    assert rho <= br
    assert mu <= bm
    assert rho <= cond * eps2 * 1.01  # the normwise bound (power-step estimates)
    if rho < 1:
        assert mu <= rho / (1 - rho) * 1.01


@pytest.mark.parametrize("cond", [1e2, 1e4])
@pytest.mark.parametrize("prec,solver", [("FP16", "IR"), ("FP16", "GMRES_IR"), ("BF16", "IR"),
                                         ("BF16", "GMRES_IR"), ("FP64", "DIRECT")])
def test_dense_tanh_precisions_n1024(env, cond, prec, solver):
    n3p, torch = env
    n = 1024
    print("case dense n=%d cond=%g %s %s" % (n, cond, prec, solver), flush=True)
    A, b, x0 = dense_tanh_system(n, cond)
    ref = O.newton_dense_tanh(A, b, x0, floor=False)
    At = torch.from_numpy(np.ascontiguousarray(A.T)).cuda().t()
    bt = torch.from_numpy(b).cuda()
    x = torch.from_numpy(x0.copy()).cuda()
    x, rep = n3p.solve_dense_tanh(At, bt, x, prec=getattr(n3p, prec), solver=getattr(n3p, solver))
    err = float(np.abs(x.cpu().numpy() - 1.0).max())
    print("  its=%d (oracle %d) err=%.2e lin=%s gated=%s" % (rep.its, ref.its, err, rep.lin_its,
                                                           gated(prec, solver, cond)), flush=True)
    assert rep.status in (0, 1)
    if gated(prec, solver, cond):
        assert rep.status == 0
        assert rep.its in (ref.its, ref.its + 1)
        assert err <= 1e-9


@pytest.mark.parametrize("cond", [1e2, 1e4])
@pytest.mark.parametrize("prec,solver", [("FP16", "IR"), ("FP16", "GMRES_IR"), ("BF16", "IR"),
                                         ("BF16", "GMRES_IR")])
def test_dense_tanh_full_size_n16384(env, cond, prec, solver):
    """N = 16384: x* = 1 holds at any size; the count is compared with FP64-LU Newton."""
    n3p, torch = env
    n = 16384
    print("case dense full-size n=%d cond=%g %s %s" % (n, cond, prec, solver), flush=True)
    A, b, _ = dense_tanh_system_torch(n, cond, "cuda")
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    x, rep = n3p.solve_dense_tanh(A, b, x, prec=getattr(n3p, prec), solver=getattr(n3p, solver))
    err = float((x - 1.0).abs().max().item())
    x64 = torch.zeros(n, dtype=torch.float64, device="cuda")
    x64, rep64 = n3p.solve_dense_tanh(A, b, x64, prec=n3p.FP64, solver=n3p.DIRECT)
    print("  its=%d (FP64-LU %d) err=%.2e lin=%s gated=%s" % (rep.its, rep64.its, err, rep.lin_its,
                                                           gated(prec, solver, cond, n)), flush=True)
    del A
    assert rep64.status == 0
    assert rep.status in (0, 1)
    if gated(prec, solver, cond, n):
        assert rep.status == 0
        assert rep.its in (rep64.its, rep64.its + 1)
        assert err <= 1e-9
