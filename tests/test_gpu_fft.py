"""FFT form of the H-equation (eq. (3.2)) against the oracle.

The Hankel sum S_i = sum_j x_j / (i + j + 1) is evaluated as a convolution
with a complex FP64 FFT of length L = 2^p >= 2N - 1.  The forward error of
such a convolution is bounded by a modest multiple of
eps * log2(L) * ||h||_2 * ||x||_2 (h_k = 1/(k+1)), which sets the tolerances
below; D and F inherit it through the factor (c/2N)(i + 1/2) <= c/2 and 1/D^2.
"""
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_heq_large as G  # noqa: E402

pytestmark = pytest.mark.gpu
EPS = 2.0 ** -53


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2307_16051_amd as n3p
    assert torch.cuda.is_available()
    return n3p, torch


def fft_bound(n, x):
    L = 2
    while L < 2 * n - 1:
        L *= 2
    h = 1.0 / np.arange(1, 2 * n, dtype=np.float64)
    return 20.0 * EPS * np.log2(L) * np.linalg.norm(h) * np.linalg.norm(x)


@pytest.mark.parametrize("n", [1, 2, 7, 300, 1000, 4096, 16384])
@pytest.mark.parametrize("c", [0.5, 0.99])
def test_fft_residual_matches_oracle(env, n, c):
    n3p, torch = env
    print("case fft residual n=%d c=%g" % (n, c), flush=True)
    x = np.random.default_rng(n).uniform(0.8, 2.5, n)
    F_ref, D_ref = O.heq_residual(x, c, want_d=True)
    F, D = n3p.heq_residual_fft(torch.from_numpy(x).cuda(), c)
    F, D = F.cpu().numpy(), D.cpu().numpy()
    tS = fft_bound(n, x)
    tD = 0.5 * c * tS + 4 * EPS * np.abs(D_ref)
    assert np.all(np.abs(D - D_ref) <= tD), np.abs(D - D_ref).max()
    tF = tD / D_ref ** 2 + 8 * EPS * (np.abs(x) + np.abs(1.0 / D_ref))
    assert np.all(np.abs(F - F_ref) <= tF), np.abs(F - F_ref).max()


@pytest.mark.parametrize("n", [5, 257, 1000, 4096])
def test_matrix_free_jv_matches_oracle_jacobian(env, n):
    n3p, torch = env
    c = 0.9
    rng = np.random.default_rng(n + 3)
    x = rng.uniform(0.8, 2.5, n)
    v = rng.standard_normal(n).astype(np.float32)
    _, D_ref = O.heq_residual(x, c, want_d=True)
    J = O.heq_jacobian(x, c)                       # FP64 J = I - diag(1/D^2) K
    y_ref = J @ v.astype(np.float64)
    y = n3p.heq_jv(torch.from_numpy(D_ref).cuda(), torch.from_numpy(v).cuda(), c).cpu().numpy()
    # FFT error in K v plus the final rounding to FP32
    tS = fft_bound(n, v.astype(np.float64))
    tol = 0.5 * c * tS / D_ref ** 2 + 2.0 ** -24 * np.abs(y_ref) + 1e-30
    assert np.all(np.abs(y.astype(np.float64) - y_ref) <= tol), np.abs(y - y_ref).max()


@pytest.mark.parametrize("n,c,solver", [(4096, 0.9, "IR"), (4096, 0.99, "IR"),
                                        (8192, 0.9999, "GMRES_IR")])
def test_solve_with_fft_residual_and_matrix_free_products(env, n, c, solver):
    """Algorithm 2.1 with the O(N log N) residual and J v from the operator."""
    n3p, torch = env
    print("case fft solve n=%d c=%g %s" % (n, c, solver), flush=True)
    g = G.read(n, c)
    xr = O.heq_picard(n, c, tol=1e-15)
    opts = n3p.Options.default(fft_residual=1, matrix_free=1)
    x, rep = n3p.solve_heq(n, c, prec=n3p.FP16, solver=getattr(n3p, solver), opts=opts)
    err = float(np.linalg.norm(x.cpu().numpy() - xr) / np.linalg.norm(xr))
    print("  its=%d (oracle %d) err=%.2e lin=%s" % (rep.its, g["its"], err, rep.lin_its), flush=True)
    assert rep.status == 0
    assert rep.its in (g["its"], g["its"] + 1)
    assert err <= 1e-9

