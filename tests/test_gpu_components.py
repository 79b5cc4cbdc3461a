"""GPU parity of the library's components against the CPU oracle.

Inputs are seeded and synthetic; every expected value comes from the oracle
or from the definition evaluated in FP64 on the CPU.  Nothing produced by the
GPU is fed to the oracle.
"""
import numpy as np
import pytest

from oracle import oracle as O
from workloads import random_matrix

pytestmark = pytest.mark.gpu

U16 = 2.0 ** -11   # FP16 unit roundoff (IEEE binary16)
UBF = 2.0 ** -8    # BF16 unit roundoff
U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2307_16051_amd as n3p
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return n3p, torch


def to_cm(torch, A, dtype):
    """numpy (n x n) -> column-major device tensor (stride (1, n))."""
    return torch.from_numpy(np.ascontiguousarray(np.asarray(A, dtype=np.float64).T)).to(
        "cuda", dtype).t()


def from_cm(T):
    return T.double().cpu().numpy()


# ------------------------------------------------------------ H-equation
@pytest.mark.parametrize("n", [1, 7, 300, 1000])
@pytest.mark.parametrize("c", [0.5, 0.99])
def test_heq_residual_matches_oracle(env, n, c):
    n3p, torch = env
    print("case heq_residual n=%d c=%g" % (n, c), flush=True)
    x = np.random.default_rng(n).uniform(0.8, 2.5, n)
    F_ref, D_ref = O.heq_residual(x, c, want_d=True)
    F, D = n3p.heq_residual(torch.from_numpy(x).cuda(), c)
    torch.cuda.synchronize()
    np.testing.assert_allclose(F.cpu().numpy(), F_ref, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(D.cpu().numpy(), D_ref, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("n", [5, 257, 640])
def test_heq_jacobian_is_fp32_rounding_of_oracle(env, n):
    n3p, torch = env
    c = 0.9
    x = np.random.default_rng(n + 1).uniform(0.8, 2.5, n)
    J_ref = O.heq_jacobian(x, c)
    _, D = n3p.heq_residual(torch.from_numpy(x).cuda(), c)
    J = from_cm(n3p.heq_jacobian(D, c))
    # FP64 evaluation order differs from the oracle's by a few ulp of FP64;
    # after rounding to FP32 the results agree to one FP32 ulp
    assert np.all(np.abs(J - J_ref) <= 1.0 * U32 * 2 * np.abs(J_ref) + 1e-300)


# ---------------------------------------------------------------- getrf
def diag_dominant(n, seed):
    A = random_matrix(n, seed)
    return A + 2.0 * n * np.eye(n)


@pytest.mark.parametrize("n", [64, 100, 512, 777, 1024, 1536])
def test_getrf_fp64_no_interchange_path(env, n):
    """Diagonally dominant: the verified no-interchange path; pivots are the identity."""
    n3p, torch = env
    print("case getrf_fp64_spec n=%d" % n, flush=True)
    A = diag_dominant(n, n)
    LU_ref, piv_ref, info_ref = O.getrf(A)
    T = to_cm(torch, A, torch.float64)
    ipiv, info = n3p.getrf(T)
    assert info == info_ref == 0
    assert np.array_equal(ipiv.cpu().numpy(), piv_ref)
    np.testing.assert_allclose(from_cm(T), LU_ref, rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("n", [64, 100, 513, 1024, 2500, 4100])
def test_getrf_fp64_pivoting_path(env, n):
    """Gaussian matrix: explicit partial pivoting; pivots equal the oracle's.
    Sizes above 1024 span several outer blocks of 1024 columns (the last one
    partial), so interchanges reach rows below a block before its U row block
    is formed."""
    n3p, torch = env
    print("case getrf_fp64_pivot n=%d" % n, flush=True)
    A = random_matrix(n, 100 + n)
    LU_ref, piv_ref, info_ref = O.getrf(A)
    T = to_cm(torch, A, torch.float64)
    ipiv, info = n3p.getrf(T)
    assert info == 0
    assert np.array_equal(ipiv.cpu().numpy(), piv_ref)
    # same pivots, so the factors differ only by the order of FP64 sums
    # (blocked matrix-core updates against one sequential elimination)
    dev = np.abs(from_cm(T) - LU_ref).max() / np.abs(LU_ref).max()
    print("  max |LU - LU_ref| / max |LU_ref| = %.2e" % dev, flush=True)
    np.testing.assert_allclose(from_cm(T), LU_ref, rtol=1e-12, atol=1e-12 * np.abs(LU_ref).max())


def check_backward_error(A_in, LU, ipiv, u, nstages, u_acc, eta_sub):
    """Componentwise backward error of the stored factors, |L| <= 1.

    |P A - L U| <= (k + 2) (u (|P A| + |L| |U|) + eta_sub) + n u_acc |L| |U|:
    k roundings to the storage precision (relative u, or absolute eta_sub for
    subnormal results) plus the accumulation error of inner products of
    length <= n carried in the accumulation precision u_acc.
    """
    n = A_in.shape[0]
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    p = O.perm_from_ipiv(ipiv)
    PA = A_in[p]
    assert np.abs(np.tril(LU, -1)).max() <= 1.0 + 4 * u
    LUabs = np.abs(L) @ np.abs(U)
    err = np.abs(PA - L @ U)
    bound = (nstages + 2) * (u * (np.abs(PA) + LUabs) + eta_sub) + n * u_acc * LUabs
    ratio = (err / np.maximum(bound, 1e-300)).max()
    assert ratio <= 1.0, ratio


@pytest.mark.parametrize("prec,u", [("fp16", U16), ("bf16", UBF), ("fp32", U32)])
@pytest.mark.parametrize("kind", ["dominant", "gaussian", "heq"])
@pytest.mark.parametrize("n", [200, 1024, 2500])
def test_getrf_low_precision_backward_error(env, prec, u, kind, n):
    n3p, torch = env
    print("case getrf_%s_%s n=%d" % (prec, kind, n), flush=True)
    dt = {"fp16": torch.float16, "bf16": torch.bfloat16, "fp32": torch.float32}[prec]
    if kind == "dominant":
        A = diag_dominant(n, 7 + n) / (2.0 * n)
    elif kind == "gaussian":
        A = random_matrix(n, 9 + n)
    else:
        A = O.heq_jacobian(np.ones(n), 0.99)
    T = to_cm(torch, A, dt)
    A_in = from_cm(T)  # the rounded input actually factored
    ipiv, info = n3p.getrf(T)
    assert info == 0
    piv = ipiv.cpu().numpy()
    if kind != "gaussian":
        assert np.array_equal(piv, np.arange(n))  # no interchange is ever the max
    stages = (n + 511) // 512 + 8
    eta_sub = {"fp16": 2.0 ** -25, "bf16": 2.0 ** -134, "fp32": 2.0 ** -150}[prec]
    check_backward_error(A_in, from_cm(T), piv, u, stages, U32, eta_sub)


@pytest.mark.parametrize("prec,u", [("fp16", U16), ("bf16", UBF)])
@pytest.mark.parametrize("n", [3100, 4100])
def test_getrf_half_several_outer_blocks_backward_error(env, prec, u, n):
    """The half-precision path over several 1024-column outer blocks: each
    block's trailing update is split between the look-ahead (the next
    diagonal square) and the launch that factors that square (the rest, the
    rows below the square included), so every part of it is checked here
    against the componentwise backward-error bound."""
    n3p, torch = env
    print("case getrf_%s_blocks n=%d" % (prec, n), flush=True)
    dt = {"fp16": torch.float16, "bf16": torch.bfloat16}[prec]
    A = O.heq_jacobian(np.ones(n), 0.99)
    T = to_cm(torch, A, dt)
    A_in = from_cm(T)
    ipiv, info = n3p.getrf(T)
    assert info == 0
    piv = ipiv.cpu().numpy()
    assert np.array_equal(piv, np.arange(n))
    stages = (n + 511) // 512 + 8
    eta_sub = {"fp16": 2.0 ** -25, "bf16": 2.0 ** -134}[prec]
    check_backward_error(A_in, from_cm(T), piv, u, stages, U32, eta_sub)


def subnormal_matrix(kind, n, seed):
    """Every entry an FP16 subnormal or zero (|a| < 2^-14).  "gaussian":
    independent entries (partial pivoting interchanges rows).  "banded": A =
    L0 U0 with L0 unit lower with two subdiagonals of multipliers below 0.6
    in size and U0 upper, so partial pivoting keeps the diagonal (the
    verified no-interchange path, with room for the relative rounding of
    subnormal entries, up to 2^-8) and |a| <= 2.2 max|u| < 2^-14."""
    rng = np.random.default_rng(seed)
    if kind == "gaussian":
        return np.clip(rng.standard_normal((n, n)), -6, 6) * 2.0 ** -17.5
    U0 = np.triu(rng.uniform(-1.0, 1.0, (n, n))) * 2.0 ** -16
    U0[np.diag_indices(n)] = rng.choice([-1.0, 1.0], n) * rng.uniform(0.5, 1.0, n) * 2.0 ** -16
    L0 = np.eye(n)
    L0[np.arange(1, n), np.arange(n - 1)] = rng.uniform(-0.6, 0.6, n - 1)
    L0[np.arange(2, n), np.arange(n - 2)] = rng.uniform(-0.6, 0.6, n - 2)
    return L0 @ U0


@pytest.mark.parametrize("kind,n", [("gaussian", 512), ("banded", 1024), ("banded", 1536)])
def test_getrf_fp16_subnormal_only_matrix(env, kind, n):
    """Section 1.2, Table 1: FP16 keeps numbers down to 2^-24 as subnormals
    (spacing 2^-24).  A matrix whose every entry is subnormal must factor
    with the componentwise backward error of stored FP16 values, the
    subnormal floor eta_sub = 2^-25 per rounding included.  If any stage
    flushed subnormal operands to zero, the missing updates would be as large
    as the entries themselves (a pivot would even vanish)."""
    n3p, torch = env
    print("case getrf_fp16_subnormal %s n=%d" % (kind, n), flush=True)
    A = subnormal_matrix(kind, n, 41 + n)
    T = to_cm(torch, A, torch.float16)
    A_in = from_cm(T)
    nz = A_in[A_in != 0]
    assert nz.size > n and np.abs(nz).max() < 2.0 ** -14
    ipiv, info = n3p.getrf(T)
    assert info == 0
    piv = ipiv.cpu().numpy()
    if kind == "banded":
        assert np.array_equal(piv, np.arange(n))
    check_backward_error(A_in, from_cm(T), piv, U16, (n + 511) // 512 + 8, U32, 2.0 ** -25)


@pytest.mark.parametrize("n,zc", [(130, 5), (1500, 1200)])
def test_getrf_singular_reports_info(env, n, zc):
    n3p, torch = env
    A = random_matrix(n, 3)
    A[:, zc] = 0.0
    T = to_cm(torch, A, torch.float64)
    ipiv, info = n3p.getrf(T)
    _, piv_ref, info_ref = O.getrf(A)
    assert info == info_ref == zc + 1
    assert np.array_equal(ipiv.cpu().numpy(), piv_ref)


@pytest.mark.parametrize("n", [100, 1500])
def test_getrf_nan_reported(env, n):
    """A NaN in the matrix: the no-interchange check rejects it (NaN is never
    within the pivot bound), the explicit search flags it, and the
    factorisation reports a non-finite result (info = -1) instead of factors."""
    n3p, torch = env
    A = random_matrix(n, 8)
    A[n // 2, n // 3] = np.nan
    T = to_cm(torch, A, torch.float64)
    ipiv, info = n3p.getrf(T)
    assert info == -1


def test_getrf_fp16_overflow_reported(env):
    """Finite FP16 input whose partial-pivoting growth exceeds 65504: every
    kernel checks the value it stores, so the overflow is reported (info = -1)."""
    n3p, torch = env
    n = 1024
    A = np.clip(random_matrix(n, 9) * 1.5e4, -6.0e4, 6.0e4)
    T = to_cm(torch, A, torch.float16)
    assert torch.isfinite(T).all()
    ipiv, info = n3p.getrf(T)
    assert info == -1


def test_getrf_fp64_pivoting_large_properties(env):
    """N = 16500 (more than 64 panel workgroups): partial pivoting's
    |L| <= 1 and the backward error of P A = L U, checked on the GPU.  The
    oracle's factorisation at this size takes minutes, so the check is the
    defining property: ||P A - L U||_max <= c n u ||L|| ||U|| (Wilkinson)."""
    n3p, torch = env
    n = 16500
    print("case getrf_fp64_pivot_large n=%d" % n, flush=True)
    g = torch.Generator(device="cuda").manual_seed(5)
    A = torch.randn(n, n, dtype=torch.float64, device="cuda", generator=g)
    T = A.t().contiguous().t()          # column-major copy
    ipiv, info = n3p.getrf(T)
    assert info == 0
    piv = ipiv.cpu().numpy()
    assert np.all(piv >= np.arange(n)) and np.all(piv < n)
    p = torch.from_numpy(O.perm_from_ipiv(piv)).cuda()
    Lm = torch.tril(T, -1)
    assert Lm.abs().max().item() <= 1.0
    Lm.diagonal().fill_(1.0)
    Um = torch.triu(T)
    R = (A[p] - Lm @ Um).abs().max().item()
    bound = 4 * n * 2.0 ** -53 * Lm.abs().max().item() * Um.abs().max().item() * n
    print("  max|PA-LU| = %.3e (bound %.3e)" % (R, bound), flush=True)
    assert R <= bound


def pivot_pattern_matrix(kind, n, seed, eps):
    """A permutation matrix plus noise of size eps.  "shift": ones on the
    subdiagonal and in the corner, so column k's pivot is row k+1 and the row
    moved down is row k+1's again at the next column (the row a column moves
    is the next column's row k, every column).  "antidiag": ones on the
    antidiagonal, so the pivots come from the far end of the panel."""
    rng = np.random.default_rng(seed)
    A = eps * rng.standard_normal((n, n))
    if kind == "shift":
        A[np.arange(1, n), np.arange(n - 1)] += 1.0
        A[0, n - 1] += 1.0
    else:
        A[np.arange(n), np.arange(n)[::-1]] += 1.0
    return A


@pytest.mark.parametrize("kind", ["shift", "antidiag"])
@pytest.mark.parametrize("n", [300, 1100])
def test_getrf_fp64_pivot_patterns(env, kind, n):
    """Structured interchanges against the oracle: same pivots, factors to the
    order of the FP64 sums."""
    n3p, torch = env
    print("case getrf_fp64_pattern %s n=%d" % (kind, n), flush=True)
    A = pivot_pattern_matrix(kind, n, 31 + n, 1e-3)
    LU_ref, piv_ref, info_ref = O.getrf(A)
    if kind == "shift":
        assert np.array_equal(piv_ref[:-1], np.arange(1, n))  # the pattern holds
    T = to_cm(torch, A, torch.float64)
    ipiv, info = n3p.getrf(T)
    assert info == info_ref == 0
    assert np.array_equal(ipiv.cpu().numpy(), piv_ref)
    np.testing.assert_allclose(from_cm(T), LU_ref, rtol=1e-12, atol=1e-12 * np.abs(LU_ref).max())


@pytest.mark.parametrize("prec,u", [("fp16", U16), ("fp32", U32)])
@pytest.mark.parametrize("kind", ["shift", "antidiag"])
def test_getrf_low_precision_pivot_patterns(env, prec, u, kind):
    """The same patterns in the low precisions: the pivots are clear-cut
    (1 against noise of 1e-2), so they equal the oracle's, and the stored
    factors meet the componentwise backward-error bound."""
    n3p, torch = env
    n = 600
    print("case getrf_%s_pattern %s n=%d" % (prec, kind, n), flush=True)
    dt = {"fp16": torch.float16, "fp32": torch.float32}[prec]
    A = pivot_pattern_matrix(kind, n, 57, 1e-2)
    T = to_cm(torch, A, dt)
    A_in = from_cm(T)
    _, piv_ref, _ = O.getrf(A_in)
    ipiv, info = n3p.getrf(T)
    assert info == 0
    piv = ipiv.cpu().numpy()
    assert np.array_equal(piv, piv_ref)
    stages = (n + 511) // 512 + 8
    eta_sub = {"fp16": 2.0 ** -25, "fp32": 2.0 ** -150}[prec]
    check_backward_error(A_in, from_cm(T), piv, u, stages, U32, eta_sub)


def test_getrf_tie_break_lowest_row(env):
    n3p, torch = env
    n = 96
    A = random_matrix(n, 4) * 0.1
    A[:, 0] = 0.0
    A[[10, 20, 30], 0] = [-3.0, 3.0, -3.0]
    T = to_cm(torch, A, torch.float64)
    ipiv, info = n3p.getrf(T)
    _, piv_ref, _ = O.getrf(A)
    assert ipiv.cpu().numpy()[0] == piv_ref[0] == 10


@pytest.mark.parametrize("prec", ["FP16", "BF16"])
def test_mfma_rate_probe_does_its_work(env, prec):
    """The measurement helper: with every operand 1/32 each instruction adds
    1/64 to every accumulator entry, so each lane's sum of 8 x 16 entries is
    2 * iters exactly; the flop count is that of the instructions issued."""
    n3p, torch = env
    blocks, iters = 64, 100
    out, flops = n3p.mfma_rate_probe(getattr(n3p, prec), blocks, iters)
    torch.cuda.synchronize()
    assert bool((out == 2.0 * iters).all())
    assert flops == blocks * 4 * iters * 8 * (2 * 32 * 32 * 16)


# ------------------------------------------------------------- solves
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
@pytest.mark.parametrize("n", [1, 63, 64, 65, 100, 129, 700])
def test_getrs_with_oracle_factors(env, prec, n):
    """Single-block, exact-block and ragged sizes: each 64-row block inverts
    its diagonal block and folds in its nearest predecessor through one
    product, so the first, second and partial blocks are the edge cases."""
    n3p, torch = env
    A = random_matrix(n, 50 + n)
    b = np.random.default_rng(n).standard_normal(n)
    LU, piv, _ = O.getrf(A)
    dt = {"fp64": torch.float64, "fp32": torch.float32, "fp16": torch.float16}[prec]
    LUt = to_cm(torch, LU, dt)
    LU_r = from_cm(LUt)  # factors as the GPU stores them
    x_ref = O.getrs(LU_r, piv, b if prec == "fp64" else b.astype(np.float32).astype(np.float64))
    vdt = torch.float64 if prec == "fp64" else torch.float32
    bt = torch.from_numpy(b).to("cuda", vdt)
    n3p.getrs(LUt, torch.from_numpy(piv).cuda(), bt)
    x = bt.double().cpu().numpy()
    tol = 1e-12 if prec == "fp64" else 2e-4
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) < tol


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_getrs_many_blocks_with_oracle_factors(env, prec):
    """33 row blocks with a ragged last one, diagonally dominant so that the
    FP32 solve of the stored factors is compared at a conditioning-limited
    tolerance rather than against a growth factor."""
    n3p, torch = env
    n = 2049
    A = diag_dominant(n, 9)
    b = np.random.default_rng(n).standard_normal(n)
    LU, piv, info = O.getrf(A)
    assert info == 0
    dt = {"fp32": torch.float32, "fp16": torch.float16}[prec]
    LUt = to_cm(torch, LU, dt)
    LU_r = from_cm(LUt)
    x_ref = O.getrs(LU_r, piv, b.astype(np.float32).astype(np.float64))
    bt = torch.from_numpy(b).to("cuda", torch.float32)
    n3p.getrs(LUt, torch.from_numpy(piv).cuda(), bt)
    x = bt.double().cpu().numpy()
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) < 1e-5


@pytest.mark.parametrize("n", [1, 255, 1000, 2049])
def test_gemv_resid_matches_fp64_definition(env, n):
    n3p, torch = env
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n)).astype(np.float32)
    u = rng.standard_normal(n).astype(np.float32)
    b = rng.standard_normal(n).astype(np.float32)
    r_ref = b.astype(np.float64) - O.gemv(A, u)
    r = n3p.gemv_resid(to_cm(torch, A, torch.float32), torch.from_numpy(u).cuda(),
                       torch.from_numpy(b).cuda()).cpu().numpy().astype(np.float64)
    scale = np.abs(b) + np.abs(A.astype(np.float64)) @ np.abs(u.astype(np.float64))
    assert np.all(np.abs(r - r_ref) <= U32 * np.abs(r_ref) + 1e-14 * scale)


def half_factors(J32):
    """Oracle factorisation of the FP16-rounded matrix, factors rounded to FP16."""
    Jh = J32.astype(np.float16).astype(np.float64)
    LU, piv, info = O.getrf(Jh)
    assert info == 0
    return LU, piv


@pytest.mark.parametrize("n,c", [(1000, 0.99), (513, 0.9)])
def test_ir_converges_to_oracle_solution(env, n, c):
    n3p, torch = env
    x = O.newton_heq(n, c, floor=False).x * 0.999  # a point near the solution
    J32 = O.heq_jacobian(x, c).astype(np.float32)
    LU, piv = half_factors(J32)
    b = np.random.default_rng(n).standard_normal(n).astype(np.float32)
    b /= np.linalg.norm(b)
    u_ref = np.linalg.solve(J32.astype(np.float64), b.astype(np.float64))
    At = to_cm(torch, J32, torch.float32)
    LUt = to_cm(torch, LU, torch.float16)
    u = torch.zeros(n, dtype=torch.float32, device="cuda")
    sw, failed, rel = n3p.ir(At, LUt, torch.from_numpy(piv).cuda(), torch.from_numpy(b).cuda(), u)
    assert not failed and rel < 1e-6 and 1 <= sw <= 4
    ug = u.double().cpu().numpy()
    assert np.linalg.norm(ug - u_ref) / np.linalg.norm(u_ref) < 1e-5


@pytest.mark.parametrize("n,c", [(1000, 0.99), (513, 0.9), (64, 0.5)])
def test_scaled_half_ir_tracks_oracle_emulation(env, n, c):
    """The corrections of eq. (2.19) (n3p_ir_scaled_half) with the oracle's
    FP16 factors, against the oracle's emulation on the same factors: the
    same sweep count and the same converged iterate.  Entries of the two
    low-precision solves may round differently (FP32 sums in another order),
    so the iterates agree to the stopping tolerance, not bitwise."""
    n3p, torch = env
    x = O.newton_heq(n, c, floor=False).x * 0.999
    J32 = O.heq_jacobian(x, c).astype(np.float32)
    lu = O.HalfLU(O.round_half(J32), "fp16")
    b = np.random.default_rng(n + 5).standard_normal(n).astype(np.float32)
    b /= np.linalg.norm(b)
    ref = O.ir(J32, b, lu, scaled_half=True)
    assert not ref.failed
    At = to_cm(torch, J32, torch.float32)
    LUt = to_cm(torch, lu.LU_h.astype(np.float64), torch.float16)
    u = torch.zeros(n, dtype=torch.float32, device="cuda")
    sw, failed, rel = n3p.ir(At, LUt, torch.from_numpy(lu.ipiv).cuda(), torch.from_numpy(b).cuda(),
                             u, scaled_half=True)
    assert not failed and rel < 1e-6
    assert sw == ref.sweeps
    ug = u.double().cpu().numpy()
    assert np.linalg.norm(ug - ref.u) / np.linalg.norm(ref.u) < 2e-5


def test_gmres_ir_converges_on_ill_conditioned_heq(env):
    n3p, torch = env
    n, c = 1024, 0.9999
    x = O.newton_heq(n, c, floor=False).x
    J32 = O.heq_jacobian(x, c).astype(np.float32)
    LU, piv = half_factors(J32)
    b = np.random.default_rng(1).standard_normal(n).astype(np.float32)
    b /= np.linalg.norm(b)
    u_ref = np.linalg.solve(J32.astype(np.float64), b.astype(np.float64))
    At = to_cm(torch, J32, torch.float32)
    LUt = to_cm(torch, LU, torch.float16)
    u = torch.zeros(n, dtype=torch.float32, device="cuda")
    sw, gi, failed, rel = n3p.gmres_ir(At, LUt, torch.from_numpy(piv).cuda(),
                                       torch.from_numpy(b).cuda(), u)
    ug = u.double().cpu().numpy()
    assert rel < 1e-5
    assert np.linalg.norm(ug - u_ref) / np.linalg.norm(u_ref) < 1e-3


@pytest.mark.parametrize("n,kind", [(1000, "heq"), (4096, "heq"), (2048, "gaussian")])
def test_getrf_fp16_is_deterministic(env, n, kind):
    """Two factorisations of the same matrix are bitwise identical (every
    update is applied in a fixed order; no atomics or cross-block sums)."""
    n3p, torch = env
    A = O.heq_jacobian(np.ones(n), 0.99) if kind == "heq" else random_matrix(n, 77)
    T1 = to_cm(torch, A, torch.float16)
    T2 = T1.clone()
    p1, i1 = n3p.getrf(T1)
    p2, i2 = n3p.getrf(T2)
    assert i1 == i2 == 0
    assert torch.equal(p1, p2)
    assert torch.equal(T1, T2)
