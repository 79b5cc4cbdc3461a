/*
 * n3p.h -- C ABI of libn3p: Newton's method in three precisions on AMD
 * Instinct MI355X (gfx950).
 *
 * Method: C. T. Kelley, "Newton's Method in Three Precisions" (arXiv
 * 2307.16051).  The nonlinear residual is evaluated in FP64, the Jacobian is
 * stored in FP32, a half-precision copy of it is LU-factored, and the Newton
 * step is computed by iterative refinement (IR) or GMRES-IR that reuse that
 * factorisation (Algorithm 2.1 in Section 2; IR and GMRES-IR in Section 2.2).
 *
 * Conventions for every entry point:
 *   - Matrices are column-major: element (i, j) is at a[i + j*ld], ld >= n.
 *   - Pointers documented as "device" must point to device memory of the
 *     current HIP device; "host" pointers to host memory.  The library never
 *     takes ownership of caller memory.
 *   - The library never allocates device memory.  Entry points that need
 *     scratch take a caller-provided workspace (device pointer + byte size);
 *     the matching *_workspace_size function gives the minimum size.  A
 *     workspace is owned by one call at a time: concurrent calls must use
 *     different workspaces.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     All device work is enqueued on it.  Entry points that return results
 *     to host memory (reports, info codes) synchronise the stream before
 *     returning; the others are asynchronous.
 *   - Pivot vectors are 0-based LAPACK-style interchange lists: at step k
 *     row k was swapped with row ipiv[k] (ipiv[k] >= k).
 *   - No C++ exception crosses this boundary; every entry point returns an
 *     n3p_status (0 on success).
 */
#ifndef N3P_H
#define N3P_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(_WIN32)
#define N3P_API
#else
#define N3P_API __attribute__((visibility("default")))
#endif

/* ------------------------------------------------------------------ status */
typedef enum n3p_status {
    N3P_OK = 0,
    N3P_NOT_CONVERGED = 1,  /* maxit reached; x holds the last iterate */
    N3P_E_INVALID = -1,     /* bad argument (size, pointer, enum, option) */
    N3P_E_NOMEM = -2,       /* workspace smaller than *_workspace_size */
    N3P_E_SINGULAR = -3,    /* an exactly zero pivot (info > 0) */
    N3P_E_NONFINITE = -4,   /* Inf/NaN in F, J or the factors after the scaling retry */
    N3P_E_CALLBACK = -5,    /* a user callback returned non-zero */
    N3P_E_HIP = -6,         /* a HIP runtime call failed */
    N3P_E_TIMEOUT = -7,     /* a device-side bounded wait expired (never expected) */
    N3P_E_PIVOTING = -8     /* batched engine only: the matrix needs row interchanges
                               (partial pivoting would not keep the diagonal); solve it
                               with n3p_solve, which pivots */
} n3p_status;

/* Human-readable name of a status code (static storage). */
N3P_API const char *n3p_status_str(int status);
/* Library version string, e.g. "n3p 0.1.0 gfx950". */
N3P_API const char *n3p_version(void);

/* ----------------------------------------------------------------- enums */
/* Precision in which the Jacobian copy is stored and LU-factored.  FP16 and
 * BF16 give the three-precision method of Section 2 (half precision as in
 * Table 1; BF16 has FP32's range); FP32 and FP64 give the comparison points
 * (Newton with a single- or double-precision factorisation, Section 1.3). */
typedef enum n3p_prec { N3P_FP16 = 0, N3P_BF16 = 1, N3P_FP32 = 2, N3P_FP64 = 3 } n3p_prec;

/* Linear solver for the step equation J s = -F.
 *   N3P_IR        iterative refinement with the low-precision factors
 *                 (the IR algorithm of Section 2.2; stopping rule of Section 3.1)
 *   N3P_GMRES_IR  GMRES left-preconditioned by the low-precision factors
 *                 computes each IR correction (end of Section 2.2)
 *   N3P_DIRECT    one triangular solve with the factors (two-precision
 *                 Newton of Section 1.3: the "F16"/"F32"/"F64" columns of
 *                 Tables 2 and 3) */
typedef enum n3p_linsolver { N3P_IR = 0, N3P_GMRES_IR = 1, N3P_DIRECT = 2 } n3p_linsolver;

/* Half-precision range handling (Section 1.2 warns about the range of half
 * precision; eqs. (2.17)-(2.18) scale the right-hand side).
 *   N3P_SCALE_AUTO  FP16: power-of-two column scaling of the half copy; on
 *                   overflow the factorisation is redone once with targets
 *                   2^6 smaller, which are then kept for the rest of the
 *                   solve; other precisions: no scaling
 *   N3P_SCALE_NONE  plain rounding I_s^h(J) */
typedef enum n3p_scale { N3P_SCALE_AUTO = 0, N3P_SCALE_NONE = 1 } n3p_scale;

/* --------------------------------------------------------------- options */
typedef struct n3p_options {
    double tau_r;            /* relative nonlinear tolerance (default 1e-10) */
    double tau_a;            /* absolute nonlinear tolerance (default 0) */
    double tau_abs_override; /* if >= 0: stop at ||F|| <= this, ignoring tau_r/tau_a
                                (resuming a solve from a saved iterate); default -1 */
    double eta;              /* linear relative residual target eta_J, eq. (2.3)
                                (default 1e-6, Section 3.1) */
    int maxit;               /* maximum Newton steps (default 20) */
    int max_ir_sweeps;       /* maximum IR sweeps / GMRES-IR outer sweeps (default 10) */
    int gmres_restart;       /* GMRES Krylov dimension m (default 20, at most 64) */
    double gmres_tol;        /* GMRES relative tolerance on the preconditioned
                                residual (default 1e-4) */
    int gmres_max_restarts;  /* restart cycles per GMRES call (default 10) */
    int scale_mode;          /* n3p_scale (default N3P_SCALE_AUTO) */
    int timing;              /* 1: record per-phase times in the report
                                (timestamps written on the GPU timeline in
                                the workspace, read once when the solve ends:
                                no extra host waits; default 1) */
    int fft_residual;        /* built-in H-equation only: 1 = evaluate F by the
                                O(N log N) FFT form of eq. (3.2) (the Hankel sum as
                                a convolution, FP64); N <= 32768; default 0 */
    int matrix_free;         /* built-in H-equation only: 1 = the IR residual and the
                                GMRES products J v are formed from the operator
                                (J v = v - diag(1/D^2) K v by FFT in FP64, rounded to
                                FP32) instead of the stored FP32 J, which is then not
                                formed (4 N^2 fewer bytes); N <= 32768; default 0 */
    int ir_scaled_half;      /* IR only (N3P_E_INVALID with another solver): 1 = each
                                correction by eq. (2.19) (Section 2.3),
                                d = ||r|| I_h^s(U^{-1} L^{-1} I_s^h(r/||r||)): the unit-
                                scaled residual and every entry of the triangular
                                solves' results rounded to the factor precision
                                (sums in FP32); 0 (default) = the factors promoted to
                                FP32 on the fly, eq. (2.16) */
} n3p_options;

/* Fill *opt with the defaults listed above. */
N3P_API void n3p_default_options(n3p_options *opt);

/* ---------------------------------------------------------------- report */
#define N3P_MAX_HIST 64
typedef struct n3p_report {
    int status;                      /* n3p_status of the solve */
    int its;                         /* Newton steps taken */
    double f0;                       /* ||F(x_0)||_2 */
    double fnorm;                    /* ||F(x_its)||_2 */
    double resid_rel[N3P_MAX_HIST];  /* ||F(x_n)||_2 / ||F(x_0)||_2, n = 0..its */
    int lin_its[N3P_MAX_HIST];       /* IR sweeps (or GMRES iterations) at step n+1 */
    int lin_outer[N3P_MAX_HIST];     /* IR / GMRES-IR outer sweeps at step n+1 */
    uint8_t lin_fail[N3P_MAX_HIST];  /* 1 if the linear solve at step n+1 failed */
    uint8_t pivoted[N3P_MAX_HIST];   /* 1 if the factorisation at step n+1 needed
                                        row interchanges */
    double lin_rel[N3P_MAX_HIST];    /* final ||b - J u|| / ||b|| at step n+1 */
    float ms_jac;                    /* total time building J and its copy */
    float ms_getrf;                  /* total factorisation time */
    float ms_solve;                  /* total linear-solver time */
    float ms_resid;                  /* total residual + update time */
    float ms_total;                  /* wall time of the solve on the stream */
} n3p_report;

/* --------------------------------------------------------------- problems */
/* Residual callback: F = F(x) in FP64.  x, F are device pointers of length n.
 * Must enqueue all work on `stream` and return 0 (non-zero aborts the solve
 * with N3P_E_CALLBACK). */
typedef int (*n3p_residual_fn)(void *ctx, const double *x, double *F, int64_t n, void *stream);
/* Jacobian callback: J = F'(x), column-major FP32, device pointer, leading
 * dimension ldj (eq. (2.1): the Jacobian is stored in single precision). */
typedef int (*n3p_jacobian_fn)(void *ctx, const double *x, float *J, int64_t ldj, int64_t n,
                               void *stream);

typedef struct n3p_problem {
    int kind;          /* 0 = H-equation, 1 = dense tanh, 2 = callbacks */
    int64_t n;
    double c;          /* H-equation parameter */
    const double *A;   /* dense tanh: device, column-major n x n, leading dim lda */
    const double *b;   /* dense tanh: device, length n */
    int64_t lda;
    n3p_residual_fn residual;
    n3p_jacobian_fn jacobian;
    void *ctx;
} n3p_problem;

/* Chandrasekhar H-equation, midpoint rule, eq. (3.2) of Section 3:
 *   F(x)_i = x_i - (1 - (c/(2N)) sum_j x_j mu_i/(mu_j + mu_i))^{-1},
 *   mu_i = (i - 1/2)/N.  Requires n >= 1 and 0 <= c < 1 (c = 1 is accepted;
 * its Jacobian is singular at the solution). */
N3P_API int n3p_problem_heq(n3p_problem *p, int64_t n, double c);
/* Dense system F(x) = A x + 0.1 tanh(x) - b with Jacobian
 * A + 0.1 diag(1 - tanh(x)^2); A, b are caller-owned device FP64 arrays that
 * must stay valid for every solve using p. */
N3P_API int n3p_problem_dense_tanh(n3p_problem *p, int64_t n, const double *A, int64_t lda,
                                   const double *b);
/* User-defined problem through the two callbacks above. */
N3P_API int n3p_problem_callbacks(n3p_problem *p, int64_t n, n3p_residual_fn F,
                                  n3p_jacobian_fn J, void *ctx);

/* ----------------------------------------------------------- solve (main) */
/* Device bytes needed by n3p_solve for this size / precision / solver. */
N3P_API size_t n3p_workspace_size(int64_t n, int lu_prec, int linsolver, const n3p_options *opt);

/*
 * newton3p(F, x, tau_a, tau_r, eta_J): Algorithm 2.1 of Section 2.
 *   evaluate F(x) (FP64); tau = tau_r ||F|| + tau_a
 *   while ||F|| > tau:
 *     J = F'(x) stored FP32; J_h = I_s^h(J) in lu_prec (column-scaled for FP16)
 *     (lu_prec FP64 with a built-in problem factors the FP64 Jacobian itself,
 *     i.e. plain double-precision Newton; with callbacks it factors J)
 *     factor J_h (partial pivoting); find s with ||J s + F|| <= eta ||F||
 *     by `linsolver` on the unit right-hand side -F/||F|| (eqs. (2.17)-(2.18));
 *     x += s (FP64); evaluate F(x)
 * x: device FP64 array of length p->n, the initial iterate on entry and the
 * last iterate on exit.  opt may be NULL (defaults).  ws/ws_bytes: device
 * workspace of at least n3p_workspace_size bytes.  rep: host struct filled
 * on return (may be NULL).  Synchronises `stream` before returning.
 * Returns N3P_OK, N3P_NOT_CONVERGED or an error code.  A linear-solver
 * failure is not an error: as in Section 3.1 the best iterate is used,
 * rep->lin_fail is set and the Newton iteration continues.
 */
N3P_API int n3p_solve(const n3p_problem *p, double *x, int lu_prec, int linsolver,
                      const n3p_options *opt, void *ws, size_t ws_bytes, void *stream,
                      n3p_report *rep);

/* ---------------------------------------------------- component entry points */
/* Device bytes needed by n3p_getrf / n3p_getrs for size n in `prec`. */
N3P_API size_t n3p_getrf_workspace_size(int64_t n, int prec);

/*
 * LU factorisation with partial pivoting, P A = L U (Gaussian elimination,
 * Section 1.3; the half-precision factorisation of Section 2).  A: device,
 * n x n, column-major, leading dimension lda, element type given by prec
 * (FP16 = IEEE binary16, BF16 = bfloat16, FP32, FP64); overwritten by L
 * (unit lower, below the diagonal) and U.  ipiv: device int32[n], 0-based.
 * Low-precision products accumulate in FP32 (FP64 for FP64) and are rounded
 * to prec when stored.  Pivots: the largest magnitude in the column, ties to
 * the lowest row.  *info (host): 0, or k+1 if U(k,k) is exactly zero, or -1
 * if the factors are not finite.  Synchronises the stream.  The input is
 * factored as given (no scaling); n3p_solve adds the column scaling.
 * Size limit of the pivoting path: a matrix that partial pivoting would
 * factor with row interchanges (rather than with the diagonal pivots the
 * factorisation tries first) is factored by the pivoting path, which holds
 * one row per thread in at most 128 resident workgroups of 256 threads, so it
 * takes n <= 32768; a larger matrix that needs interchanges returns
 * N3P_E_INVALID (n3p_solve likewise).
 */
N3P_API int n3p_getrf(int prec, int64_t n, void *A, int64_t lda, int32_t *ipiv, int *info,
                      void *ws, size_t ws_bytes, void *stream);

/*
 * Solve A x = b with the factors from n3p_getrf: x = U^{-1} L^{-1} P b.  The
 * factors are read in `prec` and promoted to FP32 (FP64 for FP64 factors) on
 * the fly (Section 2.3); b is a device FP32 vector (FP64 when prec is FP64),
 * overwritten by x.  Asynchronous.
 */
N3P_API int n3p_getrs(int prec, int64_t n, const void *LU, int64_t lda, const int32_t *ipiv,
                      void *b, void *ws, size_t ws_bytes, void *stream);

/* Measurement helper, not a step of the method: the rate the matrix cores
 * reach on this device, against which the factorisation is also measured.
 * Launches `blocks` workgroups of 256 threads (prec N3P_FP16 or N3P_BF16);
 * every wavefront issues 8 independent chains of `iters` back-to-back
 * 32x32x16 matrix-core instructions on register operands.  `out` (device,
 * FP32, blocks * 256 entries, caller-owned) receives 2 * iters in every entry,
 * which checks that the work was done; *flops (host) receives the number of
 * floating-point operations issued.  iters in [1, 2^20].  Asynchronous on
 * `stream`: time it with events.  N3P_E_INVALID for other arguments. */
N3P_API int n3p_mfma_rate_probe(int prec, int blocks, int iters, float *out, double *flops,
                                void *stream);

/* r = b - A u for FP32 column-major A (n x n, leading dim lda) and FP32
 * vectors (device); products accumulate in FP64, r is rounded to FP32.  The
 * residual of the IR algorithm, Section 2.2.  Asynchronous. */
N3P_API int n3p_gemv_resid_f32(int64_t n, const float *A, int64_t lda, const float *u,
                               const float *b, float *r, void *ws, size_t ws_bytes, void *stream);

/* r = b - A u exactly as n3p_gemv_resid_f32 (same kernels, same FP64
 * partial sums in the same order, so bit-identical results), for callers that
 * cannot allocate device memory: code being captured into a HIP graph,
 * serving loops that must not call hipMalloc, harnesses that forbid it.  No
 * workspace is passed: the FP64 partial sums (n * ceil(n/256) doubles) live
 * in a scratch array compiled into the library, N3P_GEMV_NOALLOC_MAX_N *
 * (N3P_GEMV_NOALLOC_MAX_N / 256) doubles = 8 MiB, one copy per device, held
 * until the process ends.  Its device address is looked up once per device,
 * on the first call made with that device current.  n <= 16384
 * (N3P_GEMV_NOALLOC_MAX_N); a larger n returns N3P_E_INVALID before any
 * device work.  Every partial sum is written before it is read, so no call
 * depends on what an earlier call left in the scratch; but all calls on one
 * device share it, so calls that overlap in time on one device (different
 * streams, threads or processes without ordering) race and must be
 * serialised by the caller.  Asynchronous on `stream`. */
#define N3P_GEMV_NOALLOC_MAX_N 16384
N3P_API int n3p_gemv_resid_f32_noalloc(int64_t n, const float *A, int64_t lda, const float *u,
                                       const float *b, float *r, void *stream);

/* H-equation residual, eq. (3.2): F (and D_i = the bracket) in FP64, device
 * arrays of length n (D may be NULL).  Asynchronous. */
N3P_API int n3p_heq_residual(int64_t n, double c, const double *x, double *F, double *D,
                             void *stream);
/* H-equation Jacobian J_ij = delta_ij - (c/(2N)) mu_i/(mu_i+mu_j) / D_i^2
 * computed in FP64 and stored FP32 (eq. (2.1)); device, column-major, ldj.
 * Needs D from n3p_heq_residual.  Asynchronous. */
N3P_API int n3p_heq_jacobian(int64_t n, double c, const double *D, float *J, int64_t ldj,
                             void *stream);

/*
 * Iterative refinement for A u = b (the IR algorithm of Section 2.2) with
 * A FP32 (device, n x n, lda), b FP32 (device), and factors LU/ipiv of a
 * low-precision copy of A from n3p_getrf in `prec` (column scale vector
 * `colscale` may be NULL; if given, the factors are those of A*diag(colscale)).
 * u (device FP32) is the initial iterate on entry and the result on exit.
 * Stops when ||b - A u|| < tol ||b||, after max_sweeps sweeps, or when the
 * residual norm increases (failure: the best iterate is returned), as in
 * Section 3.1.  *sweeps, *failed, *rel_res (host) report the outcome.
 * Synchronises the stream.
 */
N3P_API int n3p_ir(int prec, int64_t n, const float *A, int64_t lda, const void *LU,
                   int64_t ldlu, const int32_t *ipiv, const float *colscale, const float *b,
                   float *u, double tol, int max_sweeps, int *sweeps, int *failed,
                   double *rel_res, void *ws, size_t ws_bytes, void *stream);

/* n3p_ir with each correction formed by eq. (2.19) (Section 2.3): r scaled to
 * unit 2-norm and rounded to the factor precision, both triangular solves
 * with every solution entry rounded to that precision as it is formed (sums
 * in FP32), the result promoted and multiplied by ||r||.  Same arguments,
 * workspace, stopping rule and errors as n3p_ir.  Synchronises the stream. */
N3P_API int n3p_ir_scaled_half(int prec, int64_t n, const float *A, int64_t lda, const void *LU,
                               int64_t ldlu, const int32_t *ipiv, const float *colscale,
                               const float *b, float *u, double tol, int max_sweeps, int *sweeps,
                               int *failed, double *rel_res, void *ws, size_t ws_bytes,
                               void *stream);

/* GMRES-IR: as n3p_ir, but each correction solves M^{-1} A d = M^{-1} r
 * (M = the low-precision LU) with restarted GMRES(m), modified Gram-Schmidt,
 * relative tolerance gmres_tol (end of Section 2.2).  *gmres_its (host)
 * returns the total Arnoldi steps.  Synchronises the stream. */
N3P_API int n3p_gmres_ir(int prec, int64_t n, const float *A, int64_t lda, const void *LU,
                         int64_t ldlu, const int32_t *ipiv, const float *colscale,
                         const float *b, float *u, double tol, int max_outer, int m,
                         double gmres_tol, int *sweeps, int *gmres_its, int *failed,
                         double *rel_res, void *ws, size_t ws_bytes, void *stream);

/* Workspace bytes for n3p_ir / n3p_gmres_ir / n3p_gemv_resid_f32 at size n
 * with Krylov dimension m (ignored for IR). */
N3P_API size_t n3p_linsolve_workspace_size(int64_t n, int m);

/* FFT form of the H-equation (eq. (3.2); the cost model of Section 3).  The
 * Hankel sum S_i = sum_j x_j / (i + j + 1) is a convolution, evaluated with a
 * complex FP64 FFT of length L = 2^p >= 2N - 1 (N <= 32768).  Device pointers;
 * ws: device workspace of n3p_heq_fft_workspace_size(n) bytes.  Each call
 * also prepares the twiddles and the transform of the kernel (O(L log L)). */
N3P_API size_t n3p_heq_fft_workspace_size(int64_t n);
/* F (and D if non-null), FP64, as n3p_heq_residual. */
N3P_API int n3p_heq_residual_fft(int64_t n, double c, const double *x, double *F, double *D,
                                 void *ws, size_t ws_bytes, void *stream);
/* y = J v with J = I - diag(1/D^2) K (eq. (3.2)), computed in FP64 from the FP32
 * vector v and rounded to FP32; D from the residual at the current iterate. */
N3P_API int n3p_heq_jv(int64_t n, double c, const double *D, const float *v, float *y, void *ws,
                       size_t ws_bytes, void *stream);

/* ===================================================== batched engine (serving)
 * Many independent H-equation solves (eq. (3.2), x0 = ones) advance through
 * Algorithm 2.1 together: one engine step is one Newton iteration for every
 * admitted request (Jacobian stored FP32 and rounded to lu_prec, the
 * no-interchange half-precision LU verified against partial pivoting, IR
 * sweeps of the IR algorithm of Section 2.2 with the Section 3.1 policy, FP64 update and
 * residual), as batched kernels over a device table of slots, replayed from
 * captured HIP graphs.  Requests join between steps as slots and pool memory
 * free up and leave when their stopping test passes.  A request's arithmetic
 * does not depend on the other requests present: results are identical alone
 * and in any mix.  Limits: N <= 4096, lu_prec FP16 or BF16, linear solver IR;
 * a matrix that needs row interchanges ends with N3P_E_PIVOTING (use
 * n3p_solve).  All device memory comes from the caller's pool; the engine
 * runs on a stream of its own (default priority) that waits for `stream` at
 * creation, and every call returns after that stream has drained. */
typedef struct n3p_engine n3p_engine; /* opaque host object */

typedef struct n3p_engine_config {
    int max_slots;   /* requests in flight at once, 1..256 */
    int64_t max_n;   /* largest admitted N, padded size <= 4096 */
    int lu_prec;     /* N3P_FP16 or N3P_BF16 */
    int use_graphs;  /* 1: capture the step phases once and replay them */
    int leaf_grid;   /* persistent grid of the leaf kernel (workgroups) */
    int gemm_grid;   /* persistent grid of the rank-64 update */
    int gemm_kc;     /* K chunk of the update tile (32 or 64) */
    int vec_grid;    /* grid of the residual, Jacobian and matvec kernels */
} n3p_engine_config;

typedef struct n3p_serve_stats {
    double p50_ms, p99_ms, mean_ms, max_ms; /* arrival to result, per request */
    double makespan_s, solves_per_s;        /* wall time of the whole stream */
    int max_active, steps;                  /* most requests in flight; engine steps */
} n3p_serve_stats;

N3P_API void n3p_engine_default_config(n3p_engine_config *cfg);
/* Pool bytes one request of size n holds while admitted (0 if not allowed). */
N3P_API size_t n3p_engine_request_bytes(int64_t n, int lu_prec);
/* Pool bytes the engine itself keeps for max_slots slots (the slot table). */
N3P_API size_t n3p_engine_fixed_bytes(int max_slots);
/* pool: caller-owned device memory, kept until destroy; opt may be NULL
 * (opt->ir_scaled_half must be 0: the engine's IR promotes on the fly). */
N3P_API int n3p_engine_create(n3p_engine **e, const n3p_engine_config *cfg,
                              const n3p_options *opt, void *pool, size_t pool_bytes,
                              void *stream);
N3P_API int n3p_engine_destroy(n3p_engine *e);
/* Admit H-equation (n, c); returns the slot.  N3P_E_NOMEM: no slot or pool
 * space free right now (try again after a step frees one). */
N3P_API int n3p_engine_admit(n3p_engine *e, int64_t n, double c, int *slot);
/* One Newton iteration for every admitted request; n_done = requests whose
 * result is ready to collect. */
N3P_API int n3p_engine_step(n3p_engine *e, int *n_done);
/* phase: 0 free, 1 admitted, 2 iterating, 3 done; its: Newton steps so far. */
N3P_API int n3p_engine_slot_state(const n3p_engine *e, int slot, int *phase, int *its);
/* Copy a finished request's x (FP64, n entries) to device x_out (may be NULL),
 * fill rep (may be NULL) and free the slot. */
N3P_API int n3p_engine_collect(n3p_engine *e, int slot, double *x_out, n3p_report *rep);
N3P_API int n3p_engine_largest_free(const n3p_engine *e, size_t *bytes);
/* Time the factorisation phase of the admitted (not yet stepped) requests for
 * each candidate (leaf grid, update grid, update K chunk), keep the fastest
 * in the engine and return it; ms_out (may be NULL) gets one time per
 * candidate (24 candidates). */
N3P_API int n3p_engine_autotune(n3p_engine *e, n3p_engine_config *chosen, float *ms_out,
                                int *n_candidates);
/* Continuous batching over `count` requests (n[i], c[i]) arriving at
 * arrival_s[i] seconds (non-decreasing) after the call starts: admitted in
 * order as slots and pool memory allow, stepped together, results copied to
 * x_out + x_off[i] (device FP64; x_out may be NULL).  its/status/latency_ms
 * (host, may be NULL) per request; stats (may be NULL) for the stream.
 * N3P_E_NOMEM if a request can never fit the pool. */
N3P_API int n3p_serve(const n3p_engine_config *cfg, const n3p_options *opt, void *pool,
                      size_t pool_bytes, int count, const int64_t *n, const double *c,
                      const double *arrival_s, double *x_out, const int64_t *x_off, int *its,
                      int *status, double *latency_ms, n3p_serve_stats *stats, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* N3P_H */
