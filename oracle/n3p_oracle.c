/*
 * n3p_oracle.c -- CPU FP64 oracle for Newton's method in three precisions
 * (C. T. Kelley, "Newton's Method in Three Precisions", arXiv 2307.16051).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it.  It shares no code, header,
 * table or helper with the GPU library, and the GPU library never calls it.
 *
 * Everything here is plain double precision, written as the textbook
 * definitions with no blocking or reordering:
 *   - the midpoint-rule H-equation residual, eq. (3.2), Section 3;
 *   - its analytic Jacobian (Section 3 states one is computed in O(N^2) work;
 *     the formula is the derivative of eq. (3.2));
 *   - the dense test problem F(x) = A x + 0.1 tanh(x) - b (a synthetic
 *     workload, not from the paper) and its Jacobian;
 *   - Gaussian elimination with partial pivoting (Section 1.3 names the LU
 *     factorisation; partial pivoting with ties to the lowest row index is the
 *     LAPACK convention, a reading the paper leaves open);
 *   - forward/back substitution;
 *   - Newton's method, Algorithm 1.1 of Section 1.1, with the step from a
 *     double-precision LU (the "F64" column of Tables 2 and 3);
 *   - Picard (fixed-point) iteration on eq. (3.2), an independent route to
 *     the same discrete solution.
 *
 * Storage is column-major: element (i, j) of an n-by-n matrix with leading
 * dimension ld is at a[i + j*ld].  Row and column indices are 0-based; so is
 * the pivot vector (ipiv[k] = row swapped with row k at step k).
 *
 * Parallelism: OpenMP only splits independent loop iterations (rows of a
 * matrix-vector product, columns of a rank-one update); the arithmetic of
 * every output element is the same sequence as in the serial loop.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_API __attribute__((visibility("default")))

/* ---------------------------------------------------------------------------
 * H-equation, Section 3.
 * Quadrature nodes mu_i = (i - 1/2)/N, i = 1..N (0-based: (i + 1/2)/N), with
 * midpoint weights 1/N, so the discrete operator is eq. (3.2):
 *     F(x)_i = x_i - ( 1 - (c/(2N)) sum_j x_j mu_i / (mu_j + mu_i) )^{-1}.
 * D_i denotes the bracket 1 - (c/(2N)) sum_j x_j mu_i/(mu_j + mu_i).
 * ------------------------------------------------------------------------- */
static double orc_mu(int64_t i, int64_t n) { return ((double)i + 0.5) / (double)n; }

ORC_API int orc_heq_residual(int64_t n, double c, const double *x, double *F, double *D)
{
    if (n <= 0) return -1;
    const double w = c / (2.0 * (double)n);
#pragma omp parallel for schedule(static) if (n >= 512)
    for (int64_t i = 0; i < n; ++i) {
        const double mui = orc_mu(i, n);
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double muj = orc_mu(j, n);
            s += x[j] * mui / (muj + mui);
        }
        const double d = 1.0 - w * s;
        if (D) D[i] = d;
        F[i] = x[i] - 1.0 / d;
    }
    return 0;
}

/*
 * Analytic Jacobian of eq. (3.2).  With K_ij = (c/(2N)) mu_i/(mu_i + mu_j),
 * D_i = 1 - sum_j K_ij x_j and F_i = x_i - 1/D_i:
 *     dF_i/dx_j = delta_ij - K_ij / D_i^2.
 */
ORC_API int orc_heq_jacobian(int64_t n, double c, const double *x, double *J, int64_t ldj)
{
    if (n <= 0 || ldj < n) return -1;
    double *D = (double *)malloc(sizeof(double) * (size_t)n);
    double *F = (double *)malloc(sizeof(double) * (size_t)n);
    if (!D || !F) { free(D); free(F); return -2; }
    orc_heq_residual(n, c, x, F, D);
    const double w = c / (2.0 * (double)n);
#pragma omp parallel for schedule(static) if (n >= 512)
    for (int64_t j = 0; j < n; ++j) {
        const double muj = orc_mu(j, n);
        for (int64_t i = 0; i < n; ++i) {
            const double mui = orc_mu(i, n);
            const double kij = w * mui / (mui + muj);
            J[i + j * ldj] = (i == j ? 1.0 : 0.0) - kij / (D[i] * D[i]);
        }
    }
    free(D);
    free(F);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Dense synthetic problem F(x) = A x + 0.1 tanh(x) - b, Jacobian
 * A + 0.1 diag(1 - tanh(x)^2).  Not from the paper: it exercises row
 * interchanges, which the H-equation never triggers.
 * ------------------------------------------------------------------------- */
ORC_API int orc_dense_tanh_residual(int64_t n, const double *A, int64_t lda, const double *b,
                                    const double *x, double *F)
{
    if (n <= 0 || lda < n) return -1;
#pragma omp parallel for schedule(static) if (n >= 512)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) s += A[i + j * lda] * x[j];
        F[i] = s + 0.1 * tanh(x[i]) - b[i];
    }
    return 0;
}

ORC_API int orc_dense_tanh_jacobian(int64_t n, const double *A, int64_t lda, const double *x,
                                    double *J, int64_t ldj)
{
    if (n <= 0 || lda < n || ldj < n) return -1;
#pragma omp parallel for schedule(static) if (n >= 512)
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < n; ++i) J[i + j * ldj] = A[i + j * lda];
        const double t = tanh(x[j]);
        J[j + j * ldj] += 0.1 * (1.0 - t * t);
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Dense linear algebra.
 * ------------------------------------------------------------------------- */

/* Euclidean norm, accumulated in the obvious order. */
ORC_API double orc_nrm2(int64_t n, const double *v)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += v[i] * v[i];
    return sqrt(s);
}

/* y = A x for column-major A (m-by-n): each y_i summed over j in order. */
ORC_API int orc_gemv(int64_t m, int64_t n, const double *A, int64_t lda, const double *x,
                     double *y)
{
#pragma omp parallel for schedule(static) if (m >= 512)
    for (int64_t i = 0; i < m; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) s += A[i + j * lda] * x[j];
        y[i] = s;
    }
    return 0;
}

/*
 * Gaussian elimination with partial pivoting, in place: P A = L U with L unit
 * lower triangular (stored below the diagonal) and U upper triangular.  At
 * step k the pivot is the entry of largest magnitude in column k on or below
 * the diagonal; among equal magnitudes the lowest row index wins.  Returns 0,
 * or k+1 if the pivot at step k is exactly zero (the factorisation is then
 * continued without dividing, as LAPACK does), or -1 on a NaN pivot column.
 */
ORC_API int orc_getrf(int64_t n, double *A, int64_t lda, int32_t *ipiv)
{
    if (n < 0 || lda < (n > 0 ? n : 1)) return -100;
    int info = 0;
    for (int64_t k = 0; k < n; ++k) {
        /* pivot search: largest |a_ik|, i >= k, first occurrence */
        int64_t p = k;
        double best = fabs(A[k + k * lda]);
        if (isnan(best)) return -1;
        for (int64_t i = k + 1; i < n; ++i) {
            const double v = fabs(A[i + k * lda]);
            if (isnan(v)) return -1;
            if (v > best) { best = v; p = i; }
        }
        ipiv[k] = (int32_t)p;
        /* interchange whole rows k and p */
        if (p != k) {
            for (int64_t j = 0; j < n; ++j) {
                const double t = A[k + j * lda];
                A[k + j * lda] = A[p + j * lda];
                A[p + j * lda] = t;
            }
        }
        const double piv = A[k + k * lda];
        if (piv == 0.0) {
            if (info == 0) info = (int)(k + 1);
            continue;
        }
        /* multipliers l_ik = a_ik / a_kk */
        for (int64_t i = k + 1; i < n; ++i) A[i + k * lda] /= piv;
        /* Schur complement: a_ij -= l_ik u_kj for i, j > k */
#pragma omp parallel for schedule(static) if (n - k >= 384)
        for (int64_t j = k + 1; j < n; ++j) {
            const double ukj = A[k + j * lda];
            if (ukj != 0.0) {
                for (int64_t i = k + 1; i < n; ++i) A[i + j * lda] -= A[i + k * lda] * ukj;
            }
        }
    }
    return info;
}

/* Solve A x = b from the factors of orc_getrf; b is overwritten by x. */
ORC_API int orc_getrs(int64_t n, const double *LU, int64_t lda, const int32_t *ipiv, double *b)
{
    if (n < 0 || lda < (n > 0 ? n : 1)) return -100;
    /* apply the interchanges in the order they were made */
    for (int64_t k = 0; k < n; ++k) {
        const int64_t p = ipiv[k];
        if (p != k) { const double t = b[k]; b[k] = b[p]; b[p] = t; }
    }
    /* L y = P b, L unit lower */
    for (int64_t j = 0; j < n; ++j) {
        const double yj = b[j];
        for (int64_t i = j + 1; i < n; ++i) b[i] -= LU[i + j * lda] * yj;
    }
    /* U x = y */
    for (int64_t j = n - 1; j >= 0; --j) {
        b[j] /= LU[j + j * lda];
        const double xj = b[j];
        for (int64_t i = 0; i < j; ++i) b[i] -= LU[i + j * lda] * xj;
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Newton's method, Algorithm 1.1 (Section 1.1), with a double-precision
 * analytic Jacobian factored by orc_getrf: the "F64" column of Tables 2, 3.
 *
 *   evaluate F(x); tau = tau_r ||F|| + tau_a
 *   while ||F|| > tau (and fewer than maxit steps):
 *       solve F'(x) s = -F(x);  x = x + s;  evaluate F(x)
 *
 * Norms are Euclidean.  hist[0..its] receives ||F(x_n)||_2 (absolute; divide
 * by hist[0] for the relative histories the tables print).  Returns the
 * number of Newton steps taken, or a negative code on failure:
 *   -2 allocation, -3 singular Jacobian, -4 non-finite residual.
 * If extra > 0, that many further steps are taken after the stopping rule is
 * met, as long as ||F|| keeps falling below half its previous value; this
 * drives x to the rounding floor (used as the reference solution).
 * ------------------------------------------------------------------------- */
typedef struct {
    int kind;          /* 0: H-equation, 1: dense tanh */
    double c;          /* H-equation parameter */
    const double *A;   /* dense problem matrix (column-major) */
    const double *b;
    int64_t lda;
} orc_problem;

static int orc_eval(const orc_problem *p, int64_t n, const double *x, double *F)
{
    if (p->kind == 0) return orc_heq_residual(n, p->c, x, F, NULL);
    return orc_dense_tanh_residual(n, p->A, p->lda, p->b, x, F);
}

static int orc_jac(const orc_problem *p, int64_t n, const double *x, double *J)
{
    if (p->kind == 0) return orc_heq_jacobian(n, p->c, x, J, n);
    return orc_dense_tanh_jacobian(n, p->A, p->lda, x, J, n);
}

static int orc_newton_impl(const orc_problem *p, int64_t n, double *x, double tau_r, double tau_a,
                           int maxit, int extra, double *hist, int *its_rule)
{
    double *F = (double *)malloc(sizeof(double) * (size_t)n);
    double *s = (double *)malloc(sizeof(double) * (size_t)n);
    double *J = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n);
    int32_t *ipiv = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!F || !s || !J || !ipiv) { free(F); free(s); free(J); free(ipiv); return -2; }

    int ret = 0;
    orc_eval(p, n, x, F);
    double fn = orc_nrm2(n, F);
    if (!isfinite(fn)) { ret = -4; goto done; }
    hist[0] = fn;
    const double tau = tau_r * fn + tau_a;
    int it = 0;
    int rule_met = (fn <= tau);
    if (its_rule) *its_rule = rule_met ? 0 : -1;
    int extra_left = extra;
    while (it < maxit + extra) {
        if (rule_met) {
            if (extra_left <= 0) break;
        } else if (it >= maxit) {
            break;
        }
        orc_jac(p, n, x, J);
        if (orc_getrf(n, J, n, ipiv) != 0) { ret = -3; goto done; }
        for (int64_t i = 0; i < n; ++i) s[i] = -F[i];
        orc_getrs(n, J, n, ipiv, s);
        /* after the rule is met, only keep steps that halve ||F|| */
        if (rule_met) {
            double *xt = (double *)malloc(sizeof(double) * (size_t)n);
            if (!xt) { ret = -2; goto done; }
            for (int64_t i = 0; i < n; ++i) xt[i] = x[i] + s[i];
            orc_eval(p, n, xt, F);
            const double ft = orc_nrm2(n, F);
            if (!(ft <= 0.5 * fn)) { free(xt); orc_eval(p, n, x, F); break; }
            memcpy(x, xt, sizeof(double) * (size_t)n);
            free(xt);
            fn = ft;
            --extra_left;
            continue;
        }
        for (int64_t i = 0; i < n; ++i) x[i] += s[i];
        orc_eval(p, n, x, F);
        fn = orc_nrm2(n, F);
        ++it;
        hist[it] = fn;
        if (!isfinite(fn)) { ret = -4; goto done; }
        if (fn <= tau) {
            rule_met = 1;
            if (its_rule) *its_rule = it;
        }
    }
    ret = it;
done:
    free(F); free(s); free(J); free(ipiv);
    return ret;
}

ORC_API int orc_newton_heq(int64_t n, double c, double *x, double tau_r, double tau_a, int maxit,
                           int extra, double *hist, int *its_rule)
{
    orc_problem p = {0, c, NULL, NULL, 0};
    return orc_newton_impl(&p, n, x, tau_r, tau_a, maxit, extra, hist, its_rule);
}

ORC_API int orc_newton_dense_tanh(int64_t n, const double *A, int64_t lda, const double *b,
                                  double *x, double tau_r, double tau_a, int maxit, int extra,
                                  double *hist, int *its_rule)
{
    orc_problem p = {1, 0.0, A, b, lda};
    return orc_newton_impl(&p, n, x, tau_r, tau_a, maxit, extra, hist, its_rule);
}

/* ---------------------------------------------------------------------------
 * Picard iteration on eq. (3.2): x_i <- 1 / D_i(x).  Its fixed point is the
 * discrete solution; it uses no Jacobian and no factorisation, so it pins
 * the Newton oracle through an independent route.  Stops when
 * max_i |x_new - x_old| <= tol or after maxit sweeps; returns the sweeps
 * taken (or -1 if maxit was reached).
 * ------------------------------------------------------------------------- */
ORC_API int orc_heq_picard(int64_t n, double c, double *x, int maxit, double tol)
{
    double *F = (double *)malloc(sizeof(double) * (size_t)n);
    double *D = (double *)malloc(sizeof(double) * (size_t)n);
    if (!F || !D) { free(F); free(D); return -2; }
    int k;
    for (k = 1; k <= maxit; ++k) {
        orc_heq_residual(n, c, x, F, D);
        double dmax = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            const double xn = 1.0 / D[i];
            const double d = fabs(xn - x[i]);
            if (d > dmax) dmax = d;
            x[i] = xn;
        }
        if (dmax <= tol) break;
    }
    free(F); free(D);
    return k > maxit ? -1 : k;
}

ORC_API int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
