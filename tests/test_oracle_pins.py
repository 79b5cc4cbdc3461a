"""Pins for the CPU oracle against facts the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values the
paper prints (Tables 2 and 3), closed forms (the moment identity, c = 0),
brute force (finite differences, tiny hand-worked eliminations), a library
special case (LAPACK through scipy) and invariants (P A = L U, quadratic
convergence, Picard reaching the same fixed point).
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import oracle as O
from workloads import dense_tanh_system, random_matrix


def printed(v):
    """Round to the four significant digits the paper prints."""
    return float("%.3e" % v)


# ---------------------------------------------------------------- Tables 2, 3

@pytest.mark.slow
def test_table2_f64_column_every_printed_digit(table2):
    """Table 2, F64 column: Newton with an FP64 Jacobian, N=4096, c=.99."""
    r = O.newton_heq(4096, 0.99, tau_r=1e-9, floor=False)
    expect = [v for v in table2["F64"] if v is not None]
    assert r.its == len(expect) - 1
    assert [printed(v) for v in r.rel_hist] == expect


@pytest.mark.slow
def test_table3_f64_column_every_printed_digit(table3):
    """Table 3, F64 column: N=4096, c=.9999."""
    r = O.newton_heq(4096, 0.9999, tau_r=1e-9, floor=False)
    expect = [v for v in table3["F64"] if v is not None]
    assert r.its == len(expect) - 1
    assert [printed(v) for v in r.rel_hist] == expect


def test_infinity_norm_does_not_reproduce_table2(table2):
    """The Euclidean norm is the reading the tables fix: the max norm differs."""
    n, c = 512, 0.99
    x = np.ones(n)
    F0 = O.heq_residual(x, c)
    J = O.heq_jacobian(x, c)
    LU, piv, _ = O.getrf(J)
    x1 = x + O.getrs(LU, piv, -F0)
    F1 = O.heq_residual(x1, c)
    rel_inf = np.abs(F1).max() / np.abs(F0).max()
    rel_2 = np.linalg.norm(F1) / np.linalg.norm(F0)
    assert printed(rel_2) == table2["F64"][1]
    assert printed(rel_inf) != table2["F64"][1]


@pytest.mark.slow
def test_table2_three_precision_columns(table2):
    """Table 2, IR 32-16 and IR-GM columns: the three-precision method tracks F64.

    Entries n = 1..4 agree to the printed digits; the last entry depends on
    rounding inside the half-precision factorisation and agrees within 2%.
    """
    n, c = 4096, 0.99
    R = lambda x: O.heq_residual(x, c)
    Jf = lambda x: O.heq_jacobian(x, c)
    for solver, col in (("ir", "IR32-16"), ("gmres", "IR-GM")):
        r = O.newton3p(R, Jf, np.ones(n), tau_r=1e-9, solver=solver)
        expect = [v for v in table2[col] if v is not None]
        assert r.its == len(expect) - 1
        got = r.rel_hist
        assert [printed(v) for v in got[:5]] == expect[:5]
        assert abs(got[5] / expect[5] - 1.0) < 0.02
        assert not any(r.lin_fail)


@pytest.mark.slow
def test_table3_gmres_ir_tracks_f64(table3):
    """Table 3, IR-GM column: GMRES-IR recovers the F64 history at c=.9999."""
    n, c = 4096, 0.9999
    R = lambda x: O.heq_residual(x, c)
    Jf = lambda x: O.heq_jacobian(x, c)
    r = O.newton3p(R, Jf, np.ones(n), tau_r=1e-9, solver="gmres")
    expect = [v for v in table3["IR-GM"] if v is not None]
    assert r.its == len(expect) - 1
    assert [printed(v) for v in r.rel_hist[:8]] == expect[:8]
    assert abs(r.rel_hist[8] / expect[8] - 1.0) < 0.02


@pytest.mark.slow
@pytest.mark.parametrize("tab,c,k", [("table2", 0.99, 5), ("table3", 0.9999, 8)])
def test_two_precision_f32_column(request, tab, c, k):
    """Tables 2 and 3, F32 column: the FP32 Jacobian factored in FP32, one solve per step.

    Entries before the last agree to every printed digit; the last depends on
    rounding inside the factorisation and agrees within 2%.  (The F16 column
    comes from a factorisation that rounds every operation to half precision,
    which the emulation here does not reproduce: that column is not pinned.)
    """
    table = request.getfixturevalue(tab)
    n = 4096
    R = lambda x: O.heq_residual(x, c)
    Jf = lambda x: O.heq_jacobian(x, c)
    r = O.newton3p(R, Jf, np.ones(n), tau_r=1e-9, solver="direct", prec="fp32")
    expect = [v for v in table["F32"] if v is not None]
    assert r.its == len(expect) - 1 == k
    assert [printed(v) for v in r.rel_hist[:k]] == expect[:k]
    assert abs(r.rel_hist[k] / expect[k] - 1.0) < 0.02


# ------------------------------------------------------------ closed forms

@pytest.mark.parametrize("c", [0.5, 0.9, 0.99, 0.9999])
@pytest.mark.parametrize("n", [64, 256])
def test_moment_identity_exact_for_discrete_system(n, c):
    """1 - (c/2) mean(x*) = sqrt(1 - c) holds exactly for eq. (3.2) at every N."""
    r = O.newton_heq(n, c)
    x = r.x_floor
    assert abs(x.mean() - O.heq_mean_closed_form(c)) < 1e-13 * O.heq_mean_closed_form(c) * 10
    assert abs(1.0 - 0.5 * c * x.mean() - np.sqrt(1.0 - c)) < 1e-12


def test_c_zero_is_identity():
    """c = 0: F(x) = x - 1, J = I, x0 = ones is already the solution."""
    n = 37
    x = np.ones(n)
    F = O.heq_residual(x, 0.0)
    assert np.all(F == 0.0)
    J = O.heq_jacobian(np.linspace(0.5, 2.0, n), 0.0)
    assert np.array_equal(J, np.eye(n))
    r = O.newton_heq(n, 0.0)
    assert r.its == 0 and np.all(r.x == 1.0)


def test_residual_matches_hand_evaluation_n2():
    """Eq. (3.2) written out by hand for N = 2 (mu = 1/4, 3/4)."""
    c = 0.7
    x = np.array([1.3, 0.8])
    mu = np.array([0.25, 0.75])
    D = [1 - c / 4 * (x[0] * mu[i] / (mu[0] + mu[i]) + x[1] * mu[i] / (mu[1] + mu[i]))
         for i in range(2)]
    F_hand = np.array([x[i] - 1 / D[i] for i in range(2)])
    np.testing.assert_allclose(O.heq_residual(x, c), F_hand, rtol=1e-15, atol=1e-15)


# --------------------------------------------------------- brute force / FD

@pytest.mark.parametrize("n,c", [(8, 0.9), (32, 0.99), (17, 0.5)])
def test_analytic_jacobian_vs_central_differences(n, c):
    x = np.random.default_rng(n).uniform(0.8, 2.5, n)
    J = O.heq_jacobian(x, c)
    h = 1e-6
    Jfd = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = h
        Jfd[:, j] = (O.heq_residual(x + e, c) - O.heq_residual(x - e, c)) / (2 * h)
    assert np.abs(J - Jfd).max() / np.abs(J).max() < 1e-7


def test_dense_tanh_jacobian_vs_central_differences():
    A, b, _ = dense_tanh_system(24, 1e2)
    x = np.random.default_rng(3).standard_normal(24)
    J = O.dense_tanh_jacobian(A, x)
    h = 1e-6
    Jfd = np.column_stack([
        (O.dense_tanh_residual(A, b, x + h * e) - O.dense_tanh_residual(A, b, x - h * e)) / (2 * h)
        for e in np.eye(24)])
    assert np.abs(J - Jfd).max() / np.abs(J).max() < 1e-7


def test_gemv_hand_product_and_closed_forms():
    """The oracle's matrix-vector product (the refinement residual's A u):
    a product evaluated by hand, a permutation matrix (y is x permuted) and a
    rank-one matrix (y = a * (b . x)), which catch a transposed operand, a
    dropped term or a wrong index."""
    A = np.array([[1.0, -2.0, 0.5], [3.0, 0.0, -1.0], [2.0, 4.0, 1.0]])
    x = np.array([2.0, -1.0, 4.0])
    # rows: 2 + 2 + 2 = 6;  6 + 0 - 4 = 2;  4 - 4 + 4 = 4
    np.testing.assert_array_equal(O.gemv(A, x), [6.0, 2.0, 4.0])
    n = 37
    rng = np.random.default_rng(3)
    p = rng.permutation(n)
    P = np.zeros((n, n))
    P[np.arange(n), p] = 1.0
    x = rng.standard_normal(n)
    np.testing.assert_array_equal(O.gemv(P, x), x[p])
    a, b = rng.standard_normal(n), rng.standard_normal(n)
    y = O.gemv(np.outer(a, b), x)
    np.testing.assert_allclose(y, a * float(b @ x), rtol=1e-13, atol=1e-13 * np.abs(a).max())
    # rectangular: the leading rows of the hand example
    np.testing.assert_array_equal(O.gemv(A[:2, :], np.array([2.0, -1.0, 4.0])), [6.0, 2.0])


def test_getrf_hand_worked_3x3():
    """Partial pivoting on a 3x3 example eliminated by hand."""
    A = np.array([[1.0, 2.0, 3.0], [4.0, 5.0, 6.0], [7.0, 8.0, 10.0]])
    LU, piv, info = O.getrf(A)
    # step 0: pivot 7 (row 2); step 1: rows [4,5,6] -> [0, 3/7, 6/7], [1,2,3] -> [0, 6/7, 11/7]
    assert info == 0 and list(piv) == [2, 2, 2]
    L = np.tril(LU, -1) + np.eye(3)
    U = np.triu(LU)
    np.testing.assert_allclose(U, [[7, 8, 10], [0, 6 / 7, 11 / 7], [0, 0, -0.5]], atol=1e-15)
    np.testing.assert_allclose(L, [[1, 0, 0], [1 / 7, 1, 0], [4 / 7, 0.5, 1]], atol=1e-15)


def test_getrf_tie_goes_to_lowest_row():
    """Column 0 holds |-3| = |3| = |-3| in rows 1..3: row 1 must be the pivot."""
    A = random_matrix(4, 5)
    A[:, 0] = [1.0, -3.0, 3.0, -3.0]
    LU, piv, info = O.getrf(A)
    assert info == 0 and piv[0] == 1


def test_getrf_singular_reports_first_zero_pivot():
    A = np.array([[1.0, 2.0, 3.0], [2.0, 4.0, 6.0], [1.0, 0.0, 1.0]])
    A[:, 1] = 2 * A[:, 0]
    LU, piv, info = O.getrf(A)
    assert info == 2


@pytest.mark.parametrize("n,seed", [(50, 0), (211, 1), (300, 2)])
def test_getrf_reconstruction_and_lapack(n, seed):
    A = random_matrix(n, seed)
    LU, piv, info = O.getrf(A)
    assert info == 0
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    p = O.perm_from_ipiv(piv)
    err = np.abs(A[p] - L @ U).max()
    assert err <= 10 * n * np.finfo(float).eps * np.abs(A).max()
    assert np.abs(L).max() <= 1.0
    lu_ref, piv_ref = sla.lu_factor(A)
    assert np.array_equal(piv, piv_ref)
    np.testing.assert_allclose(LU, lu_ref, rtol=1e-10, atol=1e-12)


def test_getrs_matches_lapack_solve():
    n = 120
    A = random_matrix(n, 9)
    b = np.random.default_rng(10).standard_normal(n)
    LU, piv, _ = O.getrf(A)
    x = O.getrs(LU, piv, b)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-10)


# --------------------------------------------------------------- invariants

@pytest.mark.parametrize("c", [0.5, 0.9])
def test_picard_reaches_the_newton_solution(c):
    n = 64
    xn = O.newton_heq(n, c).x_floor
    xp = O.heq_picard(n, c, tol=1e-15)
    assert np.abs(xn - xp).max() < 1e-13


def test_quadratic_convergence_of_the_error():
    n, c = 256, 0.9
    xs = []
    x = np.ones(n)
    ref = O.newton_heq(n, c).x_floor
    for _ in range(4):
        xs.append(x.copy())
        F = O.heq_residual(x, c)
        LU, piv, _ = O.getrf(O.heq_jacobian(x, c))
        x = x + O.getrs(LU, piv, -F)
    e = [np.linalg.norm(v - ref) for v in xs]
    ratios = [e[k + 1] / e[k] ** 2 for k in range(3) if e[k + 1] > 1e-13]
    assert len(ratios) >= 2 and max(ratios) < 1.0


def test_iteration_counts_mesh_independent():
    """Iterations to ||F|| <= 1e-10 ||F0|| do not change with N."""
    expected = {0.5: 3, 0.9: 4, 0.99: 6, 0.9999: 9}
    for c, its in expected.items():
        for n in (256, 1024):
            assert O.newton_heq(n, c, floor=False).its == its, (n, c)


def test_dense_tanh_root_is_ones():
    A, b, x0 = dense_tanh_system(128, 1e2)
    r = O.newton_dense_tanh(A, b, x0)
    assert r.its <= 4
    assert np.abs(r.x_floor - 1.0).max() < 1e-12


def test_three_precision_gmres_ir_matches_f64_iterations_small():
    """Theory (eq. (2.13)): with eta_J = O(u_s) the iteration count is Newton's."""
    n = 256
    for c in (0.9, 0.99):
        R = lambda x: O.heq_residual(x, c)
        Jf = lambda x: O.heq_jacobian(x, c)
        r3 = O.newton3p(R, Jf, np.ones(n), solver="ir")
        r64 = O.newton_heq(n, c)
        assert r3.its == r64.its
        assert np.linalg.norm(r3.x - r64.x_floor) / np.linalg.norm(r64.x_floor) < 1e-9


# ------------------------------------------- the correction of eq. (2.19)

def _factors(L, U, prec="fp16"):
    lu = O.HalfLU.__new__(O.HalfLU)
    lu.prec = prec
    lu.L = np.asarray(L, dtype=np.float64)
    lu.U = np.asarray(U, dtype=np.float64)
    lu.perm = np.arange(lu.L.shape[0])
    return lu


def test_solve_half_hand_worked_2x2():
    """Section 2.3: both solves held in FP16, by hand.  rhs (1, 1/3) rounds
    to (1, 1365/4096); y1 = 1365/4096 - 1/2 = -683/4096 (exact in FP16);
    x1 = y1 / 4 = -683/16384 (exact); x0 = (1 - x1) / 2 = 17067/32768, which
    lies between the FP16 neighbours 1066/2048 and 1067/2048 and rounds up."""
    lu = _factors([[1.0, 0.0], [0.5, 1.0]], [[2.0, 1.0], [0.0, 4.0]])
    x = lu.solve_half(np.array([1.0, 1.0 / 3.0], dtype=np.float32))
    assert x[0] == 1067.0 / 2048.0 and x[1] == -683.0 / 16384.0


def test_solve_half_diagonal_closed_form():
    """L = I, U = diag(d): each entry is round(round(r_i) / d_i)."""
    rng = np.random.default_rng(7)
    d = rng.uniform(0.5, 4.0, 64)
    r = rng.standard_normal(64).astype(np.float32)
    lu = _factors(np.eye(64), np.diag(d))
    want = (r.astype(np.float16).astype(np.float64) / d).astype(np.float16).astype(np.float32)
    assert np.array_equal(lu.solve_half(r), want)


def test_solve_half_entries_in_fp16_and_close_to_exact_solve():
    """Every entry is an FP16 number, and the result is the exact solve of
    the rounded right-hand side up to a few FP16 roundings per entry (a
    dropped term, a wrong index or a transposed factor fails by far more)."""
    rng = np.random.default_rng(3)
    n = 96
    L = np.tril(rng.uniform(-0.5, 0.5, (n, n)) / n, -1) + np.eye(n)
    U = np.triu(rng.uniform(-0.5, 0.5, (n, n)) / n, 1) + np.diag(rng.uniform(1.0, 2.0, n))
    r = rng.standard_normal(n).astype(np.float32)
    lu = _factors(L, U)
    x = lu.solve_half(r)
    assert np.array_equal(x.astype(np.float16).astype(np.float32), x)
    exact = sla.solve_triangular(U, sla.solve_triangular(L, r.astype(np.float16).astype(np.float64),
                                                         lower=True, unit_diagonal=True))
    assert np.max(np.abs(x - exact)) <= 4 * 2.0 ** -11 * np.max(np.abs(exact))
    # with FP32 storage the same routine is the FP32 rounding of the exact solve
    x32 = _factors(L, U, "fp32").solve_half(r.astype(np.float16).astype(np.float32))
    assert np.max(np.abs(x32 - exact)) <= 4 * 2.0 ** -24 * np.max(np.abs(exact))


def test_scaled_half_ir_matches_on_the_fly_ir_when_well_conditioned():
    """Section 2.3: the two ways of transferring precision give the same
    results except for the most ill-conditioned problems -- same sweep
    count and the same converged correction on a well-conditioned Jacobian."""
    n, c = 256, 0.9
    x = O.heq_picard(n, c, tol=1e-6)
    J32 = O.heq_jacobian(x, c).astype(np.float32)
    lu = O.HalfLU(O.round_half(J32), "fp16")
    F = O.heq_residual(x, c)
    b = (-F / np.linalg.norm(F)).astype(np.float32)
    a = O.ir(J32, b, lu)
    h = O.ir(J32, b, lu, scaled_half=True)
    assert not a.failed and not h.failed
    assert a.sweeps == h.sweeps
    ref = np.linalg.solve(J32.astype(np.float64), b.astype(np.float64))
    for res in (a, h):
        assert np.linalg.norm(res.u - ref) <= 1e-5 * np.linalg.norm(ref)
