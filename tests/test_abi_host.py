"""Host-side checks of the C ABI (no GPU needed).

The library must load and export every entry point include/n3p.h declares;
the pure-host entry points (status strings, options, problem set-up,
workspace sizing) are exercised directly.
"""
import ctypes
import os
import re
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "n3p.h")
LIB = os.path.join(ROOT, "paper_2307_16051_amd", "libn3p.so")


def declared_symbols():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"N3P_API\s+[^;(]*?\b(n3p_\w+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libn3p.so not built; run __graft_entry__.build()")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for must in ("n3p_solve", "n3p_workspace_size", "n3p_getrf", "n3p_getrs", "n3p_ir",
                 "n3p_gmres_ir", "n3p_problem_heq", "n3p_problem_dense_tanh"):
        assert must in syms


def test_library_exports_every_declared_symbol(lib):
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_status_strings_and_version(lib):
    lib.n3p_status_str.restype = ctypes.c_char_p
    lib.n3p_version.restype = ctypes.c_char_p
    assert lib.n3p_status_str(0) == b"N3P_OK"
    assert lib.n3p_status_str(-3) == b"N3P_E_SINGULAR"
    assert lib.n3p_status_str(1) == b"N3P_NOT_CONVERGED"
    assert b"gfx950" in lib.n3p_version()


def test_binding_defaults_and_workspace():
    import paper_2307_16051_amd as n3p
    o = n3p.Options.default()
    assert o.tau_r == 1e-10 and o.tau_a == 0.0 and o.eta == 1e-6
    assert o.maxit == 20 and o.max_ir_sweeps == 10 and o.gmres_restart == 20
    assert o.gmres_tol == 1e-4
    # workspace: FP16 copy (2 N^2 padded) + FP32 J (4 N^2) dominate; the rest
    # is the two L-panel buffers (2 x N x 1024 halves), the diagonal square's
    # publication words and inverse side buffer, and the vectors
    n = 16384
    ws = n3p.workspace_size(n, n3p.FP16, n3p.IR)
    assert 6 * n * n <= ws <= 6 * n * n + 128 * 1024 * 1024
    ws64 = n3p.workspace_size(n, n3p.FP64, n3p.DIRECT)
    assert ws64 > 12 * n * n
    assert n3p.workspace_size(0, n3p.FP16, n3p.IR) == 0
    assert n3p.workspace_size(100, 7, n3p.IR) == 0


def test_problem_setup_validates_arguments():
    import paper_2307_16051_amd as n3p
    from paper_2307_16051_amd import _binding as B
    p = B._Problem()
    assert B.lib.n3p_problem_heq(ctypes.byref(p), 256, 0.9) == 0
    assert p.kind == 0 and p.n == 256 and p.c == 0.9
    assert B.lib.n3p_problem_heq(ctypes.byref(p), 0, 0.9) == -1
    assert B.lib.n3p_problem_heq(ctypes.byref(p), 10, 1.5) == -1
    assert B.lib.n3p_problem_dense_tanh(ctypes.byref(p), 10, None, 10, None) == -1
    assert n3p.status_str(-1) == "N3P_E_INVALID"


def test_matrix_free_workspace_drops_the_fp32_jacobian():
    """matrix_free: the stored FP32 J (4 N^2 bytes) is not part of the workspace."""
    import paper_2307_16051_amd as n3p
    n = 4096
    full = n3p.workspace_size(n, n3p.FP16, n3p.IR, n3p.Options.default())
    mf = n3p.workspace_size(n, n3p.FP16, n3p.IR, n3p.Options.default(matrix_free=1))
    fft_bufs = 5 * 16 * 8192 + 5 * 256
    assert abs((full - mf) - (4 * n * n - fft_bufs)) <= 2048
    # the FFT form is limited to N <= 32768
    assert n3p.workspace_size(40000, n3p.FP16, n3p.IR, n3p.Options.default(fft_residual=1)) == 0


def test_mfma_rate_probe_rejects_bad_arguments(lib):
    """Argument checks happen before any device call (no GPU here)."""
    import ctypes
    fl = ctypes.c_double(0.0)
    buf = ctypes.c_void_p(1)  # never dereferenced: validation fails first
    FP16, FP32 = 0, 2
    assert lib.n3p_mfma_rate_probe(FP32, 1, 1, buf, ctypes.byref(fl), None) == -1
    assert lib.n3p_mfma_rate_probe(FP16, 0, 1, buf, ctypes.byref(fl), None) == -1
    assert lib.n3p_mfma_rate_probe(FP16, 1, 0, buf, ctypes.byref(fl), None) == -1
    assert lib.n3p_mfma_rate_probe(FP16, 1, (1 << 20) + 1, buf, ctypes.byref(fl), None) == -1
    assert lib.n3p_mfma_rate_probe(FP16, 1, 1, None, ctypes.byref(fl), None) == -1


def test_scaled_half_option_is_ir_only():
    """eq. (2.19) is an IR option (Section 2.3: it does not suffice for
    GMRES-IR); other solvers, other values and the batched engine reject it
    before any device work."""
    import paper_2307_16051_amd as n3p
    from paper_2307_16051_amd import _binding as B
    p = B._Problem()
    assert B.lib.n3p_problem_heq(ctypes.byref(p), 256, 0.9) == 0
    x = (ctypes.c_double * 256)()
    ws = (ctypes.c_char * 64)()
    for solver, val in ((n3p.GMRES_IR, 1), (n3p.DIRECT, 1), (n3p.IR, 2), (n3p.IR, -1)):
        o = n3p.Options.default(ir_scaled_half=val)
        assert B.lib.n3p_solve(ctypes.byref(p), x, n3p.FP16, solver, ctypes.byref(o), ws,
                               ctypes.sizeof(ws), None, None) == -1
    cfg = n3p.EngineConfig()
    B.lib.n3p_engine_default_config(ctypes.byref(cfg))
    eng = ctypes.c_void_p()
    o = n3p.Options.default(ir_scaled_half=1)
    assert B.lib.n3p_engine_create(ctypes.byref(eng), ctypes.byref(cfg), ctypes.byref(o), ws,
                                   ctypes.sizeof(ws), None) == -1


def test_gemv_noalloc_rejects_bad_arguments(lib):
    """The allocation-free matvec validates sizes and pointers before it
    touches a device (no GPU here): n beyond the fixed scratch, n < 1, a
    short leading dimension, a null pointer."""
    import ctypes
    p = ctypes.c_void_p(1)  # never dereferenced: validation fails first
    nmax = 16384
    f = lib.n3p_gemv_resid_f32_noalloc
    f.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert f(nmax + 1, p, nmax + 1, p, p, p, None) == -1
    assert f(0, p, 1, p, p, p, None) == -1
    assert f(100, p, 99, p, p, p, None) == -1
    assert f(100, p, 100, None, p, p, None) == -1


def test_traffic_counters_are_keyed_to_kernels_and_schedule(tmp_path):
    """The stored HBM-traffic figure is reported only for the factorisation
    it was measured on: its key changes with the kernel source and with the
    launch schedule, and not with unrelated host code."""
    import shutil
    sys.path.insert(0, ROOT)
    import bench
    csrc = os.path.join(ROOT, "paper_2307_16051_amd", "csrc")
    root2 = tmp_path / "r"
    dst = root2 / "paper_2307_16051_amd" / "csrc"
    dst.mkdir(parents=True)
    for f in ("k_getrf.hip", "k_panel.hip", "n3p_api.cpp"):
        shutil.copy(os.path.join(csrc, f), dst / f)
    base = bench.factor_source_sha(str(root2))
    assert base == bench.factor_source_sha(ROOT)
    api = (dst / "n3p_api.cpp").read_text()
    (dst / "n3p_api.cpp").write_text(api + "\n// unrelated host code\n")
    assert bench.factor_source_sha(str(root2)) == base
    i = api.index("int getrf_spec(")
    (dst / "n3p_api.cpp").write_text(api[:i] + api[i:].replace("NB_MID", "NB_OUT", 1))
    assert bench.factor_source_sha(str(root2)) != base
    (dst / "n3p_api.cpp").write_text(api)
    (dst / "k_getrf.hip").write_text((dst / "k_getrf.hip").read_text() + "\n")
    assert bench.factor_source_sha(str(root2)) != base
