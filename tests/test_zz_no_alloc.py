"""The allocation-free residual matvec, n3p_gemv_resid_f32_noalloc.

It computes r = b - A u (the refinement residual of the IR algorithm,
Section 2.2) with the same kernels as n3p_gemv_resid_f32 but keeps its FP64
partial sums in the library's fixed scratch array instead of a caller
workspace.  Checked through the C ABI against the workspace entry point
(bit-identical: same kernels, same summation order) and against the oracle's
FP64 product, on consecutive calls whose sizes shrink, so a call that read
what an earlier, larger call left in the shared scratch would show.
"""
import ctypes

import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2307_16051_amd as n3p
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return n3p, torch


def _inputs(torch, n, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    # column-major A: the transpose of a contiguous tensor
    A = torch.randn((n, n), generator=g, device="cuda", dtype=torch.float32).t()
    u = torch.randn(n, generator=g, device="cuda", dtype=torch.float32)
    b = torch.randn(n, generator=g, device="cuda", dtype=torch.float32)
    return A, u, b


def _call_noalloc(n3p, torch, A, u, b):
    n = A.shape[0]
    r = torch.full_like(b, float("nan"))
    st = n3p.lib.n3p_gemv_resid_f32_noalloc(n, A.data_ptr(), n, u.data_ptr(), b.data_ptr(),
                                             r.data_ptr(),
                                             torch.cuda.current_stream().cuda_stream)
    assert st == 0, n3p.status_str(st)
    return r


def _check_rows(A, u, b, r, rows):
    """The oracle's FP64 product on the sampled rows; the FP32 result is
    within one rounding of the FP64 residual (FP64 partial sums)."""
    An = A[rows, :].double().cpu().numpy()
    un = u.double().cpu().numpy()
    bn = b[rows].double().cpu().numpy()
    ref = bn - O.gemv(An, un)
    scale = np.abs(bn) + np.abs(An) @ np.abs(un)
    rr = r[rows].double().cpu().numpy()
    assert np.all(np.abs(rr - ref) <= U32 * np.abs(ref) + 1e-14 * scale)


def test_noalloc_matches_workspace_entry_point_shrinking_calls(env):
    n3p, torch = env
    # largest allowed size, then a ragged size, then a smaller ragged size
    for n, seed in ((n3p.GEMV_NOALLOC_MAX_N, 11), (2049, 12), (700, 13)):
        print("noalloc gemv: n=%d seed=%d" % (n, seed), flush=True)
        A, u, b = _inputs(torch, n, seed)
        r_na = _call_noalloc(n3p, torch, A, u, b)
        r_ws = n3p.gemv_resid(A, u, b)
        torch.cuda.synchronize()
        assert torch.equal(r_na, r_ws), (n, (r_na - r_ws).abs().max().item())
        if n <= 4096:
            rows = np.arange(n)
        else:
            rows = np.unique(np.concatenate([[0, n - 1], np.random.default_rng(seed).integers(0, n, 24)]))
        _check_rows(A, u, b, r_na, torch.from_numpy(rows).cuda())


def test_noalloc_rejects_sizes_beyond_the_scratch(env):
    n3p, torch = env
    n = n3p.GEMV_NOALLOC_MAX_N + 1
    dummy = torch.zeros(1, device="cuda")
    p = dummy.data_ptr()
    st = n3p.lib.n3p_gemv_resid_f32_noalloc(n, p, n, p, p, p, torch.cuda.current_stream().cuda_stream)
    assert st == -1  # N3P_E_INVALID, before any device work
