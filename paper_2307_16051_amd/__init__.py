"""Newton's method in three precisions on AMD MI355X (gfx950).

Python binding of libn3p (C ABI declared in include/n3p.h).  This module only
marshals arguments: torch provides device memory and the current stream, and
every step of the computation runs in the library's HIP kernels.  If the
compiled library is missing the import of the binding fails loudly; there is
no CPU fallback.

Method: C. T. Kelley, "Newton's Method in Three Precisions" (arXiv
2307.16051) -- residual in FP64, Jacobian stored in FP32, a half-precision
LU reused by iterative refinement or GMRES-IR (Algorithm 2.1, Section 2).
"""
from ._binding import (  # noqa: F401
    FP16, BF16, FP32, FP64, IR, GMRES_IR, DIRECT, SCALE_AUTO, SCALE_NONE,
    Options, Report, N3PError, lib, lib_path, status_str, version,
    workspace_size, solve_heq, solve_dense_tanh, solve,
    getrf, getrs, gemv_resid, gemv_resid_noalloc, GEMV_NOALLOC_MAX_N, heq_residual, heq_jacobian, ir, gmres_ir,
    EngineConfig, ServeStats, Engine, serve, engine_request_bytes, engine_fixed_bytes,
    PHASE_FREE, PHASE_ADMITTED, PHASE_RUNNING, PHASE_DONE, heq_residual_fft, heq_jv,
    mfma_rate_probe,
)
