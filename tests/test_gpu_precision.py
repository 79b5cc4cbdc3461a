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
@pytest.mark.parametrize("prec,solver", [("FP16", "IR"), ("FP64", "DIRECT")])
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
    on the iteration count (Table 3 shows IR stagnating there); it must
    still end with a finite iterate and a report."""
    n3p, torch = env
    n = 8192
    xr, its_ref, _ = reference(n, c)
    x, rep = solve(n3p, torch, n, c, "FP16", "IR")
    print("  IR its=%d (oracle %d) err=%.2e status=%d fail=%s" % (
        rep.its, its_ref, rel_err(x, xr), rep.status, rep.lin_fail), flush=True)
    assert rep.status in (0, 1)
    assert np.all(np.isfinite(x))


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


U_HALF = {"FP16": 2.0 ** -11, "BF16": 2.0 ** -8, "FP64": 2.0 ** -53}


def gated(prec, solver, cond, n=1024):
    """Whether the theory promises convergence at this condition number.

    IR with factors of unit roundoff u contracts when u cond(A) is well below
    one (Section 2.2); GMRES-IR tolerates u cond(A) up to about ten here (the
    preconditioned matrix then has a modest condition number, so restarted
    GMRES(20) reaches its 1e-4 tolerance).  Both bounds assume the factors'
    backward error is O(u); for this dense family under partial pivoting it
    grows about linearly with N (6e-3 at N = 1024 to 9e-2 at N = 16384 in
    FP16, ~8x more in BF16), so at N = 16384 only FP16 at cond = 1e2 keeps an
    error small against 1/cond.  Outside these ranges runs are reported, not
    gated.
    """
    if prec == "FP64":
        return True
    if n > 1024:
        return prec == "FP16" and cond <= 1e2
    k = U_HALF[prec] * cond
    return (solver == "IR" and k <= 0.5) or (solver == "GMRES_IR" and k <= 10.0)


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
@pytest.mark.parametrize("prec,solver", [("FP16", "IR"), ("FP16", "GMRES_IR"), ("BF16", "GMRES_IR")])
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
