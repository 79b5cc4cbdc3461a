// k_problem.hip -- residuals, Jacobians, interprecision transfers, reductions.
//
// H-equation (Section 3, eq. (3.2)): with mu_i = (i + 1/2)/N (0-based),
//   mu_i / (mu_i + mu_j) = (i + 1/2) / (i + j + 1),
// so K_ij = (c/(2N)) (i + 1/2) h_{i+j} with h_k = 1/(k+1): a diagonal times a
// Hankel matrix.  D_i = 1 - sum_j K_ij x_j and F_i = x_i - 1/D_i are formed in
// FP64 (the residual is evaluated in double precision, Section 2); the
// Jacobian J_ij = delta_ij - K_ij / D_i^2 is computed in FP64 and stored in
// FP32 (eq. (2.1)), and in the same pass rounded to the factorisation
// precision (J_h = I_s^h(J), Section 2), optionally with a power-of-two column
// scale against the narrow FP16 range (Section 1.2, Table 1).
#include <algorithm>

#include <type_traits>
#include "n3p_internal.hpp"

namespace n3p {

// ----------------------------------------------------------- H-equation
// h_k = 1/(k+1), k = 0 .. 2n-2
__global__ void k_hinv(int64_t m, double *h)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m) h[k] = 1.0 / (double)(k + 1);
}

// Each block computes HR rows of D and F.  Thread t accumulates over
// j = t, t + 256, ... in FP64; the block reduces in a fixed order.
constexpr int HR = 16;

// sum_j x_j h_{i+j} for rows i0 .. i0+HR-1 over this thread's columns, in
// column order (HH: the Hankel table is given; FULL: every row is < n)
template <bool HH, bool FULL>
__device__ __forceinline__ void heq_residual_acc(int64_t i0, int64_t n, const double *__restrict__ x,
                                                 const double *__restrict__ h, double (&acc)[HR])
{
    for (int64_t j = threadIdx.x; j < n; j += 256) {
        const double xj = x[j];
#pragma unroll
        for (int r = 0; r < HR; ++r) {
            const int64_t i = i0 + r;
            if (FULL || i < n) {
                double hk;
                if constexpr (HH) hk = h[i + j];
                else hk = 1.0 / (double)(i + j + 1);
                acc[r] += xj * hk;
            }
        }
    }
}

__device__ __forceinline__ void heq_residual_rows(int64_t i0, int64_t n, double c,
                                                  const double *__restrict__ x,
                                                  const double *__restrict__ h,
                                                  double *__restrict__ F, double *__restrict__ D,
                                                  double (*red)[257])
{
    const int t = threadIdx.x;
    double acc[HR];
#pragma unroll
    for (int r = 0; r < HR; ++r) acc[r] = 0.0;
    // the operand form and the row bound decided once, so the inner loop has
    // no branch and its HR reads per column are issued together
    const bool full = i0 + HR <= n;
    if (h) {
        if (full) heq_residual_acc<true, true>(i0, n, x, h, acc);
        else heq_residual_acc<true, false>(i0, n, x, h, acc);
    } else {
        if (full) heq_residual_acc<false, true>(i0, n, x, h, acc);
        else heq_residual_acc<false, false>(i0, n, x, h, acc);
    }
#pragma unroll
    for (int r = 0; r < HR; ++r) red[r][t] = acc[r];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
#pragma unroll
            for (int r = 0; r < HR; ++r) red[r][t] += red[r][t + w];
        }
        __syncthreads();
    }
    if (t < HR) {
        const int64_t i = i0 + t;
        if (i < n) {
            const double wgt = c / (2.0 * (double)n);
            const double d = 1.0 - wgt * ((double)i + 0.5) * red[t][0];
            if (D) D[i] = d;
            F[i] = x[i] - 1.0 / d;
        }
    }
}

__global__ __launch_bounds__(256) void k_heq_residual(int64_t n, double c, const double *__restrict__ x,
                                                      const double *__restrict__ h,
                                                      double *__restrict__ F, double *__restrict__ D)
{
    __shared__ double red[HR][257];
    heq_residual_rows((int64_t)blockIdx.x * HR, n, c, x, h, F, D, red);
}

// Column-scale exponent: scale 2^e maps the column max m into
// [2^(tl-1), 2^tl).  A zero column keeps scale 1.
__device__ __forceinline__ float col_scale_from_max(float m, float target_log2)
{
    if (!(m > 0.0f) || !isfinite(m)) return 1.0f;
    int E;
    frexpf(m, &E);  // m = f 2^E, f in [0.5, 1)
    int e = (int)target_log2 - E;
    e = e < -100 ? -100 : (e > 100 ? 100 : e);
    return ldexpf(1.0f, e);
}

template <typename T>
__device__ __forceinline__ T cvt_out(float v) { return (T)v; }
template <>
__device__ __forceinline__ double cvt_out<double>(float v) { return (double)v; }

// Block max-reduction helper (256 threads).
__device__ __forceinline__ float block_max_256(float v, float *sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) sh[t] = fmaxf(sh[t], sh[t + w]);
        __syncthreads();
    }
    float r = sh[0];
    __syncthreads();
    return r;
}

// Fused H-equation Jacobian: one block per column j of the padded Np x Np
// matrix.  Writes J (FP32, rows < n) and the factorisation copy Ah (type T,
// Np rows, identity padding) with column scale colscale[j] (if non-null).
// rowq (may be null): rowq[i] = (c/2N)(i + 1/2) / D_i^2, so that an entry
// costs one product instead of a division (the FP64 value may differ from
// the division form in the last bits; its FP32 rounding stays within the
// FP32 rounding bound of the exact entry).
// The column for one combination of the optional operands (HH: the Hankel
// table h, RQ: the row factors rowq, HJ: J is written), so that the row loop
// has no branch on them and its operand loads are issued several rows ahead.
template <typename T, bool HH, bool RQ, bool HJ>
__device__ __forceinline__ void heq_jac_column_m(int64_t j, int64_t n, int64_t Np, double c,
                                                 const double *__restrict__ D,
                                                 const double *__restrict__ h,
                                                 float *__restrict__ J, int64_t ldj,
                                                 T *__restrict__ Ah, int64_t ldh,
                                                 float *__restrict__ colscale, float target_log2,
                                                 int *flags, float *sh,
                                                 const double *__restrict__ rowq)
{
    const int t = threadIdx.x;
    T *col = Ah ? Ah + j * ldh : nullptr;
    if (j >= n) {  // padding column: e_j
        if (col)
            for (int64_t i = t; i < Np; i += 256) col[i] = cvt_out<T>(i == j ? 1.0f : 0.0f);
        if (colscale && t == 0) colscale[j] = 1.0f;
        return;
    }
    const double wgt = c / (2.0 * (double)n);
    float mx = 0.0f;
    bool bad = false;
    auto entry = [&](int64_t i) -> double {
        double hk;
        if constexpr (HH) hk = h[i + j];
        else hk = 1.0 / (double)(i + j + 1);
        if constexpr (RQ) {
            return (i == j ? 1.0 : 0.0) - rowq[i] * hk;
        } else {
            const double di = D[i];
            const double kij = wgt * ((double)i + 0.5) * hk;
            return (i == j ? 1.0 : 0.0) - kij / (di * di);
        }
    };
#pragma unroll 8
    for (int64_t i = t; i < n; i += 256) {
        const float vf = (float)entry(i);
        if constexpr (HJ) J[i + j * ldj] = vf;
        bad |= !isfinite(vf);
        mx = fmaxf(mx, fabsf(vf));
    }
    if (bad && flags) set_flag(&flags[FLAG_NONFINITE], 1);
    if (!col) return;
    float s = 1.0f;
    if (colscale) {
        s = col_scale_from_max(block_max_256(mx, sh), target_log2);
        if (t == 0) colscale[j] = s;
    }
#pragma unroll 8
    for (int64_t i = t; i < n; i += 256) {
        // recompute in the same order so the FP32 value is identical to J's
        const double v = entry(i);
        if constexpr (std::is_same<T, double>::value) {
            col[i] = v;  // a double-precision factorisation takes the FP64 Jacobian itself
        } else {
            const T o = cvt_out<T>((float)v * s);
            bad |= !isfinite((float)o);  // the stored value (FP16 range)
            col[i] = o;
        }
    }
    if (bad && flags) set_flag(&flags[FLAG_NONFINITE], 1);
    for (int64_t i = n + t; i < Np; i += 256) col[i] = cvt_out<T>(0.0f);
}

template <typename T>
__device__ __forceinline__ void heq_jac_column(int64_t j, int64_t n, int64_t Np, double c,
                                               const double *__restrict__ D,
                                               const double *__restrict__ h,
                                               float *__restrict__ J, int64_t ldj,
                                               T *__restrict__ Ah, int64_t ldh,
                                               float *__restrict__ colscale, float target_log2,
                                               int *flags, float *sh,
                                               const double *__restrict__ rowq = nullptr)
{
#define N3P_JAC(HH_, RQ_)                                                                            \
    do {                                                                                             \
        if (J) heq_jac_column_m<T, HH_, RQ_, true>(j, n, Np, c, D, h, J, ldj, Ah, ldh, colscale,     \
                                                   target_log2, flags, sh, rowq);                    \
        else heq_jac_column_m<T, HH_, RQ_, false>(j, n, Np, c, D, h, J, ldj, Ah, ldh, colscale,      \
                                                  target_log2, flags, sh, rowq);                     \
    } while (0)
    if (h && rowq) N3P_JAC(true, true);
    else if (h) N3P_JAC(true, false);
    else if (rowq) N3P_JAC(false, true);
    else N3P_JAC(false, false);
#undef N3P_JAC
}

template <typename T>
__global__ __launch_bounds__(256) void k_heq_jac_round(int64_t n, int64_t Np, double c,
                                                       const double *__restrict__ D,
                                                       const double *__restrict__ h,
                                                       float *__restrict__ J, int64_t ldj,
                                                       T *__restrict__ Ah, int64_t ldh,
                                                       float *__restrict__ colscale,
                                                       float target_log2, int *flags,
                                                       const double *__restrict__ rowq)
{
    __shared__ float sh[256];
    heq_jac_column<T>(blockIdx.x, n, Np, c, D, h, J, ldj, Ah, ldh, colscale, target_log2, flags, sh,
                      rowq);
}

// One-pass form for n <= JR_TH * JR_NPT: a column stays in registers between
// its max reduction and its rounding, so every operand is read once (the
// two-pass form reads the FP64 operands of every entry twice and is bound by
// that cache traffic).  JR_NC columns per workgroup (they would share the row
// factors; one column keeps the registers low enough for two workgroups per
// CU, which measured faster).  Branch-free rows (clamped reads, masked
// values), so the reads are issued ahead of their use.  Identical values.
constexpr int JR_TH = 1024, JR_NPT = 16, JR_NC = 1;

template <int NC>
__device__ __forceinline__ void block_max_jr(float (&m)[NC], float (*sh)[JR_TH / 64])
{
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        float v = m[c];
        for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
        if (lane == 0) sh[c][w] = v;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        float r = sh[c][0];
#pragma unroll
        for (int i = 1; i < JR_TH / 64; ++i) r = fmaxf(r, sh[c][i]);
        m[c] = r;
    }
}

template <typename T, bool HH, bool RQ, bool HJ>
__global__ __launch_bounds__(JR_TH, 8) void k_heq_jac_round1(int64_t n, int64_t Np, double c,
                                                          const double *__restrict__ D,
                                                          const double *__restrict__ h,
                                                          float *__restrict__ J, int64_t ldj,
                                                          T *__restrict__ Ah, int64_t ldh,
                                                          float *__restrict__ colscale,
                                                          float target_log2, int *flags,
                                                          const double *__restrict__ rowq)
{
    __shared__ float sh[JR_NC][JR_TH / 64];
    const int t = threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.x * JR_NC;
    const double wgt = c / (2.0 * (double)n);
    float vf[JR_NC][JR_NPT], mx[JR_NC];
    bool bad = false;
#pragma unroll
    for (int cc = 0; cc < JR_NC; ++cc) mx[cc] = 0.0f;
#pragma unroll
    for (int q = 0; q < JR_NPT; ++q) {
        const int64_t i = t + (int64_t)JR_TH * q;
        const bool iin = i < n;
        const int64_t ic = iin ? i : n - 1;  // clamped read, value masked below
        double rq = 0.0, di = 1.0;
        if constexpr (RQ) rq = rowq[ic];
        else di = D[ic];
#pragma unroll
        for (int cc = 0; cc < JR_NC; ++cc) {
            const int64_t j = j0 + cc;
            const int64_t jc = j < n ? j : n - 1;
            // the entry exactly as heq_jac_column forms it
            double hk;
            if constexpr (HH) hk = h[ic + jc];
            else hk = 1.0 / (double)(ic + jc + 1);
            double v;
            if constexpr (RQ) {
                v = (ic == jc ? 1.0 : 0.0) - rq * hk;
            } else {
                const double kij = wgt * ((double)ic + 0.5) * hk;
                v = (ic == jc ? 1.0 : 0.0) - kij / (di * di);
            }
            const bool ok = iin && j < n;
            const float x = ok ? (float)v : 0.0f;
            if constexpr (HJ) {
                if (ok) J[i + j * ldj] = x;
            }
            bad |= !isfinite(x);
            mx[cc] = fmaxf(mx[cc], fabsf(x));
            vf[cc][q] = x;
        }
    }
    if (bad && flags) set_flag(&flags[FLAG_NONFINITE], 1);
    if (!Ah) return;
    block_max_jr<JR_NC>(mx, sh);
    bool over = false;
#pragma unroll
    for (int cc = 0; cc < JR_NC; ++cc) {
        const int64_t j = j0 + cc;
        if (j >= Np) continue;
        T *col = Ah + j * ldh;
        if (j >= n) {  // padding column: e_j
            for (int64_t i = t; i < Np; i += JR_TH) col[i] = cvt_out<T>(i == j ? 1.0f : 0.0f);
            if (colscale && t == 0) colscale[j] = 1.0f;
            continue;
        }
        const float sc = colscale ? col_scale_from_max(mx[cc], target_log2) : 1.0f;
        if (colscale && t == 0) colscale[j] = sc;
#pragma unroll
        for (int q = 0; q < JR_NPT; ++q) {
            const int64_t i = t + (int64_t)JR_TH * q;
            const T o = cvt_out<T>(vf[cc][q] * sc);
            if (i < n) {
                over |= !isfinite((float)o);  // the stored value (FP16 range)
                col[i] = o;
            }
        }
        for (int64_t i = n + t; i < Np; i += JR_TH) col[i] = cvt_out<T>(0.0f);
    }
    if (over && flags) set_flag(&flags[FLAG_NONFINITE], 1);
}

template <typename T, bool HH, bool RQ>
static void launch_jac1(int64_t n, int64_t Np, double c, const double *D, const double *h, float *J,
                        int64_t ldj, T *Ah, int64_t ldh, float *colscale, float tl, int *flags,
                        const double *rowq, hipStream_t s)
{
    const int64_t ncol = Ah ? Np : n;
    const dim3 g((unsigned)((ncol + JR_NC - 1) / JR_NC)), b(JR_TH);
    if (J)
        hipLaunchKernelGGL((k_heq_jac_round1<T, HH, RQ, true>), g, b, 0, s, n, Np, c, D, h, J, ldj, Ah, ldh,
                           colscale, tl, flags, rowq);
    else
        hipLaunchKernelGGL((k_heq_jac_round1<T, HH, RQ, false>), g, b, 0, s, n, Np, c, D, h, J, ldj, Ah, ldh,
                           colscale, tl, flags, rowq);
}

// the one-pass form for any combination of the optional operands
template <typename T>
static void launch_jac_onepass(int64_t n, int64_t Np, double c, const double *D, const double *h, float *J,
                               int64_t ldj, T *Ah, int64_t ldh, float *colscale, float tl, int *flags,
                               const double *rowq, hipStream_t s)
{
    if (h && rowq) launch_jac1<T, true, true>(n, Np, c, D, h, J, ldj, Ah, ldh, colscale, tl, flags, rowq, s);
    else if (h) launch_jac1<T, true, false>(n, Np, c, D, h, J, ldj, Ah, ldh, colscale, tl, flags, rowq, s);
    else if (rowq) launch_jac1<T, false, true>(n, Np, c, D, h, J, ldj, Ah, ldh, colscale, tl, flags, rowq, s);
    else launch_jac1<T, false, false>(n, Np, c, D, h, J, ldj, Ah, ldh, colscale, tl, flags, rowq, s);
}

// rowq[i] = (c/2N)(i + 1/2) / D_i^2 (the Jacobian's row factor)
__global__ void k_heq_rowq(int64_t n, double c, const double *__restrict__ D, double *__restrict__ rowq)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double di = D[i];
    rowq[i] = (c / (2.0 * (double)n)) * ((double)i + 0.5) / (di * di);
}

// Generic J (FP32) -> Ah rounding with optional column scaling.
template <typename T>
__global__ __launch_bounds__(256) void k_round_scale(int64_t n, int64_t Np, const float *__restrict__ J,
                                                     int64_t ldj, T *__restrict__ Ah, int64_t ldh,
                                                     float *__restrict__ colscale, float target_log2,
                                                     int *flags)
{
    __shared__ float sh[256];
    const int64_t j = blockIdx.x;
    const int t = threadIdx.x;
    T *col = Ah + j * ldh;
    if (j >= n) {
        for (int64_t i = t; i < Np; i += 256) col[i] = cvt_out<T>(i == j ? 1.0f : 0.0f);
        if (colscale && t == 0) colscale[j] = 1.0f;
        return;
    }
    const float *src = J + j * ldj;
    float s = 1.0f;
    float mx = 0.0f;
    bool bad = false;
#pragma unroll 8
    for (int64_t i = t; i < n; i += 256) {  // branch-free, so the reads go out together
        const float v = src[i];
        bad |= !isfinite(v);
        mx = fmaxf(mx, fabsf(v));
    }
    if (bad && flags) set_flag(&flags[FLAG_NONFINITE], 1);
    if (colscale) {
        s = col_scale_from_max(block_max_256(mx, sh), target_log2);
        if (t == 0) colscale[j] = s;
    }
    bool over = false;
#pragma unroll 8
    for (int64_t i = t; i < n; i += 256) {
        const T o = cvt_out<T>(src[i] * s);
        over |= !isfinite((double)o);  // the stored value (FP16 range)
        col[i] = o;
    }
    if (over && flags) set_flag(&flags[FLAG_NONFINITE], 1);
    for (int64_t i = n + t; i < Np; i += 256) col[i] = cvt_out<T>(0.0f);
}

// ------------------------------------------------------------ dense tanh
// F = A x + 0.1 tanh(x) - b: partial sums over column chunks, then a fixed
// order reduction.  Block (rb, cb): rows [rb*256, +256), columns [cb*CH, +CH).
constexpr int GV_ROWS = 256, GV_CH = 512;

__global__ __launch_bounds__(256) void k_gemv_f64_part(int64_t n, const double *__restrict__ A,
                                                       int64_t lda, const double *__restrict__ x,
                                                       double *__restrict__ part)
{
    const int64_t i = (int64_t)blockIdx.x * GV_ROWS + threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.y * GV_CH;
    const int64_t j1 = min(j0 + GV_CH, n);
    double s = 0.0;
    if (i < n)
        for (int64_t j = j0; j < j1; ++j) s += A[i + j * lda] * x[j];
    if (i < n) part[(int64_t)blockIdx.y * n + i] = s;
}

__global__ void k_dense_tanh_finish(int64_t n, int nch, const double *__restrict__ part,
                                    const double *__restrict__ x, const double *__restrict__ b,
                                    double *__restrict__ F)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int c = 0; c < nch; ++c) s += part[(int64_t)c * n + i];
    F[i] = s + 0.1 * tanh(x[i]) - b[i];
}

__global__ __launch_bounds__(256) void k_dense_tanh_jac(int64_t n, const double *__restrict__ A,
                                                        int64_t lda, const double *__restrict__ x,
                                                        float *__restrict__ J, int64_t ldj)
{
    const int64_t j = blockIdx.x;
    const double tj = tanh(x[j]);
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        double v = A[i + j * lda];
        if (i == j) v += 0.1 * (1.0 - tj * tj);
        J[i + j * ldj] = (float)v;
    }
}

// The same Jacobian for a double-precision factorisation: FP32 copy J (used
// by the refinement residual) plus the unrounded FP64 values in the padded
// Np x Np factor buffer Ah (identity padding).  One block per column of Ah.
__global__ __launch_bounds__(256) void k_dense_tanh_jac_f64(int64_t n, int64_t Np,
                                                            const double *__restrict__ A,
                                                            int64_t lda, const double *__restrict__ x,
                                                            float *__restrict__ J, int64_t ldj,
                                                            double *__restrict__ Ah, int64_t ldh)
{
    const int64_t j = blockIdx.x;
    double *col = Ah + j * ldh;
    if (j >= n) {
        for (int64_t i = threadIdx.x; i < Np; i += 256) col[i] = i == j ? 1.0 : 0.0;
        return;
    }
    const double tj = tanh(x[j]);
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        double v = A[i + j * lda];
        if (i == j) v += 0.1 * (1.0 - tj * tj);
        J[i + j * ldj] = (float)v;
        col[i] = v;
    }
    for (int64_t i = n + threadIdx.x; i < Np; i += 256) col[i] = 0.0;
}

// ----------------------------------------------------------- reductions
// Deterministic Euclidean norm in FP64: block partial sums of squares, then a
// single block sums the partials in index order.
template <typename V>
__global__ __launch_bounds__(256) void k_sumsq_part(int64_t n, const V *__restrict__ x,
                                                    double *__restrict__ part)
{
    __shared__ double sh[256];
    const int t = threadIdx.x;
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + t; i < n; i += (int64_t)gridDim.x * 256) {
        const double v = (double)x[i];
        s += v * v;
    }
    sh[t] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    if (t == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_sum_sqrt(int m, const double *__restrict__ part,
                                                  double *__restrict__ out)
{
    __shared__ double sh[256];
    const int t = threadIdx.x;
    double s = 0.0;
    for (int i = t; i < m; i += 256) s += part[i];
    sh[t] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    if (t == 0) out[0] = sqrt(sh[0]);
}

constexpr int NRM_BLOCKS = 256;

// ---------------------------------------------------------- vector kernels
__global__ void k_fill_i32(int *p, int v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_fill_f32(float *p, float v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_iota_i32(int32_t *p, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (int32_t)i;
}
// b = I_d^s(-F/||F||), eq. (2.17); tail [n, np) zeroed
__global__ void k_rhs_unit(int64_t n, int64_t np, const double *F, const double *fn, float *b)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)(-F[i] / fn[0]);
    else if (i < np) b[i] = 0.0f;
}
// FP64 right-hand side -F/||F|| (Newton with a double-precision factorisation)
__global__ void k_rhs_unit_f64(int64_t n, int64_t np, const double *F, const double *fn, double *b)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = -F[i] / fn[0];
    else if (i < np) b[i] = 0.0;
}
__global__ void k_scal_copy_f32(int64_t n, float *d, const float *s, double a)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = (float)((double)s[i] * a);
}
// x += ||F|| I_s^d(u), eq. (2.18)
__global__ void k_newton_update_f32(int64_t n, double *x, const double *fn, const float *u)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] += fn[0] * (double)u[i];
}
__global__ void k_newton_update_f64(int64_t n, double *x, const double *fn, const double *u)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] += fn[0] * u[i];
}
__global__ void k_axpy_f32(int64_t n, float *y, const float *x, float a)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] += a * x[i];
}
__global__ void k_vcopy_f32(int64_t n, float *d, const float *s)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = s[i];
}
__global__ void k_f32_to_f64(int64_t n, const float *s, double *d)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = (double)s[i];
}
__global__ void k_f64_to_f32(int64_t n, const double *s, float *d)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = (float)s[i];
}
__global__ void k_copy_u32(int64_t n, uint32_t *d, const uint32_t *s)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = s[i];
}
__global__ void k_copy_u8(int64_t n, uint8_t *d, const uint8_t *s)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = s[i];
}

// padded copies (one block per column of the Np x Np buffer)
template <typename T>
__global__ __launch_bounds__(256) void k_pad_in(int64_t n, int64_t Np, const T *__restrict__ A,
                                                int64_t lda, T *__restrict__ P)
{
    const int64_t j = blockIdx.x;
    T *col = P + j * Np;
    for (int64_t i = threadIdx.x; i < Np; i += 256) {
        T v;
        if (j < n) v = i < n ? A[i + j * lda] : (T)0.0f;
        else v = (T)(i == j ? 1.0f : 0.0f);
        col[i] = v;
    }
}
template <typename T>
__global__ __launch_bounds__(256) void k_pad_out(int64_t n, int64_t Np, const T *__restrict__ P,
                                                 T *__restrict__ A, int64_t lda)
{
    const int64_t j = blockIdx.x;
    for (int64_t i = threadIdx.x; i < n; i += 256) A[i + j * lda] = P[i + j * Np];
}

// --------------------------------------------------------------- launchers
static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }


// ====================================================== batched engine kernels
// Slot masks: bit (1 << phase) selects the slots a launch works on.

// x = ones for freshly admitted slots
__global__ __launch_bounds__(256) void k_b_fill_x0(const BDesc *__restrict__ d,
                                                   const BState *__restrict__ st, int nslots)
{
    const int s = blockIdx.x;
    if (s >= nslots || st[s].phase != BP_FRESH) return;
    for (int64_t i = threadIdx.x; i < d[s].n; i += 256) d[s].x[i] = 1.0;
    if (threadIdx.x == 0) d[s].flags[FLAG_FAIL] = 0;
}

// F(x), D(x) of eq. (3.2) for every selected slot; items are 16-row blocks
__global__ __launch_bounds__(256) void k_b_residual(const BDesc *__restrict__ d,
                                                    const BState *__restrict__ st, int nslots,
                                                    int mask)
{
    __shared__ double red[HR][257];
    __shared__ int off[B_MAX_SLOTS + 1];
    const int total = b_offsets(nslots, off, [&](int s) {
        return (mask >> st[s].phase & 1) ? (int)((d[s].n + HR - 1) / HR) : 0;
    });
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int s = b_find(off, nslots, item);
        const BDesc &q = d[s];
        heq_residual_rows((int64_t)(item - off[s]) * HR, q.n, q.c, q.x, q.h, q.F, q.D, red);
        __syncthreads();
    }
}

// deterministic FP64 Euclidean norm of v[0 .. n) by one 256-thread block
template <typename V>
__device__ __forceinline__ double block_nrm2(int64_t n, const V *__restrict__ v, double *sh)
{
    const int t = threadIdx.x;
    double a = 0.0;
    for (int64_t i = t; i < n; i += 256) {
        const double e = (double)v[i];
        a += e * e;
    }
    sh[t] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    const double r = sqrt(sh[0]);
    __syncthreads();
    return r;
}

// ||F||, the stopping test of Algorithm 2.1 and the per-slot bookkeeping.
// Fresh slots: F(x0) gives f0 and tau = tau_r f0 + tau_a.
__global__ __launch_bounds__(256) void k_b_newton_check(const BDesc *__restrict__ d,
                                                        BState *__restrict__ st, int nslots,
                                                        int mask, BParams p)
{
    __shared__ double sh[256];
    const int s = blockIdx.x;
    if (s >= nslots || !(mask >> st[s].phase & 1)) return;
    const double fn = block_nrm2(d[s].n, d[s].F, sh);
    if (threadIdx.x != 0) return;
    BState &q = st[s];
    if (q.phase == BP_FRESH) {
        q.f0 = fn;
        q.tau = p.tau_r * fn + p.tau_a;
        q.its = 0;
        q.rel[0] = 1.0;
        q.phase = BP_RUN;
    } else {
        q.rel[q.its] = q.f0 > 0.0 ? fn / q.f0 : 0.0;
    }
    q.fn = fn;
    q.factor = 0;
    if (!isfinite(fn)) {
        q.phase = BP_DONE;
        q.status = N3P_E_NONFINITE;
    } else if (fn <= q.tau) {
        q.phase = BP_DONE;
        q.status = N3P_OK;
    } else if (q.its >= p.maxit || q.its >= N3P_MAX_HIST - 1) {
        q.phase = BP_DONE;
        q.status = N3P_NOT_CONVERGED;
    } else {
        q.factor = 1;
    }
}

// J (FP32) and the rounded, column-scaled factor copy, one column per item
template <typename T>
__global__ __launch_bounds__(256) void k_b_jac(const BDesc *__restrict__ d,
                                               const BState *__restrict__ st, int nslots, float tl)
{
    __shared__ float sh[256];
    __shared__ int off[B_MAX_SLOTS + 1];
    const int total = b_offsets(nslots, off, [&](int s) {
        return (st[s].phase == BP_RUN && st[s].factor) ? (int)d[s].Np : 0;
    });
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int s = b_find(off, nslots, item);
        const BDesc &q = d[s];
        if (item == off[s] && threadIdx.x == 0) {
            q.flags[FLAG_FAIL] = 0;
            q.flags[FLAG_NONFINITE] = 0;
        }
        heq_jac_column<T>(item - off[s], q.n, q.Np, q.c, q.D, q.h, q.J, q.n, (T *)q.A, q.Np,
                          q.colscale, tl, nullptr, sh);
        __syncthreads();
    }
}

// After the factorisation: unit right-hand side b = -F/||F|| (eq. (2.17)),
// u = 0, r = b, and the IR state (the IR algorithm of Section 2.2).  A slot whose matrix needs
// row interchanges, or whose factors are not finite, ends here.
__global__ __launch_bounds__(256) void k_b_ir_init(const BDesc *__restrict__ d,
                                                   BState *__restrict__ st, int nslots, BParams p)
{
    __shared__ double sh[256];
    const int s = blockIdx.x;
    if (s >= nslots || st[s].phase != BP_RUN || !st[s].factor) return;
    const BDesc &q = d[s];
    const int t = threadIdx.x;
    const int fail = ld_flag(&q.flags[FLAG_FAIL]), bad = ld_flag(&q.flags[FLAG_NONFINITE]);
    if (fail || bad) {
        if (t == 0) {
            st[s].phase = BP_DONE;
            st[s].status = fail ? N3P_E_PIVOTING : N3P_E_NONFINITE;
            st[s].factor = 0;
        }
        return;
    }
    const double fn = st[s].fn;
    for (int64_t i = t; i < q.Np; i += 256) {
        const float v = i < q.n ? (float)(-q.F[i] / fn) : 0.0f;
        q.b[i] = v;
        q.r[i] = v;
        q.u[i] = 0.0f;
    }
    __syncthreads();
    const double nb = block_nrm2(q.Np, q.b, sh);
    if (t == 0) {
        BState &z = st[s];
        z.nb = nb;
        z.rn = nb;
        z.sweeps = 0;
        z.ir_failed = 0;
        z.ir_on = (p.max_sweeps > 0 && !(nb < p.eta * nb)) ? 1 : 0;
    }
}

// One IR sweep's bookkeeping: ||r||, growth test, success test, sweep cap.
// On growth the previous iterate is restored (Section 3.1).
__global__ __launch_bounds__(256) void k_b_ir_check(const BDesc *__restrict__ d,
                                                    BState *__restrict__ st, int nslots, BParams p)
{
    __shared__ double sh[256];
    __shared__ int grew;
    const int s = blockIdx.x;
    if (s >= nslots || st[s].phase != BP_RUN || !st[s].factor || !st[s].ir_on) return;
    const BDesc &q = d[s];
    const double rnew = block_nrm2(q.Np, q.r, sh);
    if (threadIdx.x == 0) {
        BState &z = st[s];
        z.sweeps += 1;
        grew = !(rnew <= z.rn);
        if (grew) {
            z.ir_failed = 1;
            z.ir_on = 0;
        } else {
            z.rn = rnew;
            z.ir_on = (!(z.rn < p.eta * z.nb) && z.sweeps < p.max_sweeps) ? 1 : 0;
        }
    }
    __syncthreads();
    if (grew)
        for (int64_t i = threadIdx.x; i < q.Np; i += 256) q.u[i] = q.uprev[i];
}

// x += ||F|| u in FP64 (eq. (2.18)); close the step's bookkeeping
__global__ __launch_bounds__(256) void k_b_ir_final(const BDesc *__restrict__ d,
                                                    BState *__restrict__ st, int nslots, BParams p)
{
    const int s = blockIdx.x;
    if (s >= nslots || st[s].phase != BP_RUN || !st[s].factor) return;
    const BDesc &q = d[s];
    const double fn = st[s].fn;
    for (int64_t i = threadIdx.x; i < q.n; i += 256) q.x[i] += fn * (double)q.u[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        BState &z = st[s];
        if (!z.ir_failed && !(z.rn < p.eta * z.nb)) z.ir_failed = 1;
        z.lin[z.its] = z.sweeps;
        z.its += 1;
        z.factor = 0;
    }
}

hipError_t launch_hinv(int64_t n, double *h, hipStream_t s)
{
    hipLaunchKernelGGL(k_hinv, dim3(nblk(2 * n - 1, 256)), dim3(256), 0, s, 2 * n - 1, h);
    return hipGetLastError();
}

// h: Hankel table from launch_hinv (2n-1 entries) or null (computed inline)
hipError_t launch_heq_residual(int64_t n, double c, const double *x, const double *h, double *F,
                               double *D, hipStream_t s)
{
    hipLaunchKernelGGL(k_heq_residual, dim3(nblk(n, HR)), dim3(256), 0, s, n, c, x, h, F, D);
    return hipGetLastError();
}

template <typename T>
static hipError_t heq_jac_round_t(int64_t n, int64_t Np, double c, const double *D,
                                  const double *h, float *J, int64_t ldj, void *Ah, int64_t ldh,
                                  float *colscale, float tl, int *flags, double *rowq, hipStream_t s)
{
    if (rowq)
        hipLaunchKernelGGL(k_heq_rowq, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, c, D, rowq);
    if constexpr (!std::is_same<T, double>::value) {
        if (n <= (int64_t)JR_TH * JR_NPT) {
            launch_jac_onepass<T>(n, Np, c, D, h, J, ldj, (T *)Ah, ldh, colscale, tl, flags, rowq, s);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL(k_heq_jac_round<T>, dim3((unsigned)(Ah ? Np : n)), dim3(256), 0, s, n, Np,
                       c, D, h, J, ldj, (T *)Ah, ldh, colscale, tl, flags, (const double *)rowq);
    return hipGetLastError();
}

// Fused H-equation Jacobian + rounding (declared in the host driver).
hipError_t launch_heq_jac_round(int prec, int64_t n, int64_t Np, double c, const double *D,
                                const double *h, float *J, int64_t ldj, void *Ah, int64_t ldh,
                                float *colscale, float tl, int *flags, double *rowq, hipStream_t s)
{
    switch (prec) {
    case N3P_FP16: return heq_jac_round_t<f16>(n, Np, c, D, h, J, ldj, Ah, ldh, colscale, tl, flags, rowq, s);
    case N3P_BF16: return heq_jac_round_t<bf16>(n, Np, c, D, h, J, ldj, Ah, ldh, colscale, tl, flags, rowq, s);
    case N3P_FP32: return heq_jac_round_t<float>(n, Np, c, D, h, J, ldj, Ah, ldh, colscale, tl, flags, rowq, s);
    case N3P_FP64: return heq_jac_round_t<double>(n, Np, c, D, h, J, ldj, Ah, ldh, colscale, tl, flags, nullptr, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_heq_jacobian(int64_t n, double c, const double *D, const double *h, float *J,
                               int64_t ldj, hipStream_t s)
{
    hipLaunchKernelGGL(k_heq_jac_round<float>, dim3((unsigned)n), dim3(256), 0, s, n, n, c, D, h, J,
                       ldj, (float *)nullptr, (int64_t)0, (float *)nullptr, 0.0f, (int *)nullptr,
                       (const double *)nullptr);
    return hipGetLastError();
}

hipError_t launch_dense_tanh_residual(int64_t n, const double *A, int64_t lda, const double *b,
                                      const double *x, double *F, double *part, hipStream_t s)
{
    const int nch = (int)((n + GV_CH - 1) / GV_CH);
    hipLaunchKernelGGL(k_gemv_f64_part, dim3(nblk(n, GV_ROWS), nch), dim3(256), 0, s, n, A, lda,
                       x, part);
    hipLaunchKernelGGL(k_dense_tanh_finish, dim3(nblk(n, 256)), dim3(256), 0, s, n, nch,
                       (const double *)part, x, b, F);
    return hipGetLastError();
}

hipError_t launch_dense_tanh_jacobian(int64_t n, const double *A, int64_t lda, const double *x,
                                      float *J, int64_t ldj, hipStream_t s)
{
    hipLaunchKernelGGL(k_dense_tanh_jac, dim3((unsigned)n), dim3(256), 0, s, n, A, lda, x, J, ldj);
    return hipGetLastError();
}

hipError_t launch_dense_tanh_jacobian_f64(int64_t n, int64_t Np, const double *A, int64_t lda,
                                          const double *x, float *J, int64_t ldj, double *Ah,
                                          int64_t ldh, hipStream_t s)
{
    hipLaunchKernelGGL(k_dense_tanh_jac_f64, dim3((unsigned)Np), dim3(256), 0, s, n, Np, A, lda, x,
                       J, ldj, Ah, ldh);
    return hipGetLastError();
}

hipError_t launch_round_scale(int prec, int64_t n, int64_t Np, const float *J, int64_t ldj,
                              void *Ah, int64_t ldh, float *colscale, float tl, int *flags,
                              hipStream_t s)
{
    dim3 g((unsigned)Np), b(256);
    switch (prec) {
    case N3P_FP16: hipLaunchKernelGGL(k_round_scale<f16>, g, b, 0, s, n, Np, J, ldj, (f16 *)Ah, ldh, colscale, tl, flags); break;
    case N3P_BF16: hipLaunchKernelGGL(k_round_scale<bf16>, g, b, 0, s, n, Np, J, ldj, (bf16 *)Ah, ldh, colscale, tl, flags); break;
    case N3P_FP32: hipLaunchKernelGGL(k_round_scale<float>, g, b, 0, s, n, Np, J, ldj, (float *)Ah, ldh, colscale, tl, flags); break;
    case N3P_FP64: hipLaunchKernelGGL(k_round_scale<double>, g, b, 0, s, n, Np, J, ldj, (double *)Ah, ldh, colscale, tl, flags); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pad_copy_in(int prec, int64_t n, int64_t Np, const void *A, int64_t lda,
                              void *Ap, hipStream_t s)
{
    dim3 g((unsigned)Np), b(256);
    switch (prec) {
    case N3P_FP16: hipLaunchKernelGGL(k_pad_in<f16>, g, b, 0, s, n, Np, (const f16 *)A, lda, (f16 *)Ap); break;
    case N3P_BF16: hipLaunchKernelGGL(k_pad_in<bf16>, g, b, 0, s, n, Np, (const bf16 *)A, lda, (bf16 *)Ap); break;
    case N3P_FP32: hipLaunchKernelGGL(k_pad_in<float>, g, b, 0, s, n, Np, (const float *)A, lda, (float *)Ap); break;
    case N3P_FP64: hipLaunchKernelGGL(k_pad_in<double>, g, b, 0, s, n, Np, (const double *)A, lda, (double *)Ap); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pad_copy_out(int prec, int64_t n, int64_t Np, const void *Ap, void *A,
                               int64_t lda, hipStream_t s)
{
    dim3 g((unsigned)n), b(256);
    switch (prec) {
    case N3P_FP16: hipLaunchKernelGGL(k_pad_out<f16>, g, b, 0, s, n, Np, (const f16 *)Ap, (f16 *)A, lda); break;
    case N3P_BF16: hipLaunchKernelGGL(k_pad_out<bf16>, g, b, 0, s, n, Np, (const bf16 *)Ap, (bf16 *)A, lda); break;
    case N3P_FP32: hipLaunchKernelGGL(k_pad_out<float>, g, b, 0, s, n, Np, (const float *)Ap, (float *)A, lda); break;
    case N3P_FP64: hipLaunchKernelGGL(k_pad_out<double>, g, b, 0, s, n, Np, (const double *)Ap, (double *)A, lda); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_copy_bytes(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    if (bytes % 4 == 0) {
        int64_t m = (int64_t)(bytes / 4);
        hipLaunchKernelGGL(k_copy_u32, dim3(nblk(m, 256)), dim3(256), 0, s, m, (uint32_t *)dst,
                           (const uint32_t *)src);
    } else {
        int64_t m = (int64_t)bytes;
        hipLaunchKernelGGL(k_copy_u8, dim3(nblk(m, 256)), dim3(256), 0, s, m, (uint8_t *)dst,
                           (const uint8_t *)src);
    }
    return hipGetLastError();
}

hipError_t launch_nrm2_f64(int64_t n, const double *x, double *part, double *out, hipStream_t s)
{
    const int nb = (int)std::min<int64_t>(NRM_BLOCKS, std::max<int64_t>(1, (n + 255) / 256));
    hipLaunchKernelGGL(k_sumsq_part<double>, dim3(nb), dim3(256), 0, s, n, x, part);
    hipLaunchKernelGGL(k_sum_sqrt, dim3(1), dim3(256), 0, s, nb, (const double *)part, out);
    return hipGetLastError();
}

hipError_t launch_nrm2_f32(int64_t n, const float *x, double *part, double *out, hipStream_t s)
{
    const int nb = (int)std::min<int64_t>(NRM_BLOCKS, std::max<int64_t>(1, (n + 255) / 256));
    hipLaunchKernelGGL(k_sumsq_part<float>, dim3(nb), dim3(256), 0, s, n, x, part);
    hipLaunchKernelGGL(k_sum_sqrt, dim3(1), dim3(256), 0, s, nb, (const double *)part, out);
    return hipGetLastError();
}

// A timestamp on the GPU timeline (the 100 MHz real-time counter), for the
// report's per-phase times without host synchronisation: one lane of one
// wavefront writes it (a vector store).
__global__ __launch_bounds__(64) void k_stamp(uint64_t *p)
{
    if (threadIdx.x == 0) *p = __builtin_amdgcn_s_memrealtime();
}

hipError_t launch_stamp(uint64_t *p, hipStream_t s)
{
    hipLaunchKernelGGL(k_stamp, dim3(1), dim3(64), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int *p, int v, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_i32, dim3(nblk(n, 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}
hipError_t launch_fill_f32(float *p, float v, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_f32, dim3(nblk(n, 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}
hipError_t launch_iota_i32(int32_t *p, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_iota_i32, dim3(nblk(n, 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}
hipError_t launch_rhs_unit(int64_t n, int64_t np, const double *F, const double *fnorm, float *b,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_rhs_unit, dim3(nblk(np, 256)), dim3(256), 0, s, n, np, F, fnorm, b);
    return hipGetLastError();
}
hipError_t launch_rhs_unit_f64(int64_t n, int64_t np, const double *F, const double *fnorm,
                               double *b, hipStream_t s)
{
    hipLaunchKernelGGL(k_rhs_unit_f64, dim3(nblk(np, 256)), dim3(256), 0, s, n, np, F, fnorm, b);
    return hipGetLastError();
}
hipError_t launch_scal_copy_f32(int64_t n, float *dst, const float *src, double a, hipStream_t s)
{
    hipLaunchKernelGGL(k_scal_copy_f32, dim3(nblk(n, 256)), dim3(256), 0, s, n, dst, src, a);
    return hipGetLastError();
}
hipError_t launch_newton_update_f32(int64_t n, double *x, const double *fnorm, const float *u,
                                    hipStream_t s)
{
    hipLaunchKernelGGL(k_newton_update_f32, dim3(nblk(n, 256)), dim3(256), 0, s, n, x, fnorm, u);
    return hipGetLastError();
}
hipError_t launch_newton_update_f64(int64_t n, double *x, const double *fnorm, const double *u,
                                    hipStream_t s)
{
    hipLaunchKernelGGL(k_newton_update_f64, dim3(nblk(n, 256)), dim3(256), 0, s, n, x, fnorm, u);
    return hipGetLastError();
}
hipError_t launch_axpy_f32(int64_t n, float *y, const float *x, float a, hipStream_t s)
{
    hipLaunchKernelGGL(k_axpy_f32, dim3(nblk(n, 256)), dim3(256), 0, s, n, y, x, a);
    return hipGetLastError();
}
hipError_t launch_vcopy_f32(int64_t n, float *dst, const float *src, hipStream_t s)
{
    hipLaunchKernelGGL(k_vcopy_f32, dim3(nblk(n, 256)), dim3(256), 0, s, n, dst, src);
    return hipGetLastError();
}
hipError_t launch_f32_to_f64(int64_t n, const float *src, double *dst, hipStream_t s)
{
    hipLaunchKernelGGL(k_f32_to_f64, dim3(nblk(n, 256)), dim3(256), 0, s, n, src, dst);
    return hipGetLastError();
}
hipError_t launch_f64_to_f32(int64_t n, const double *src, float *dst, hipStream_t s)
{
    hipLaunchKernelGGL(k_f64_to_f32, dim3(nblk(n, 256)), dim3(256), 0, s, n, src, dst);
    return hipGetLastError();
}


// ---------------------------------------------------------- batched launchers
hipError_t launch_b_fill_x0(const BDesc *d, const BState *st, int nslots, hipStream_t s)
{
    hipLaunchKernelGGL(k_b_fill_x0, dim3(nslots), dim3(256), 0, s, d, st, nslots);
    return hipGetLastError();
}
hipError_t launch_b_residual(const BDesc *d, BState *st, int nslots, int mask, int grid,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_b_residual, dim3(grid), dim3(256), 0, s, d, st, nslots, mask);
    return hipGetLastError();
}
hipError_t launch_b_newton_check(const BDesc *d, BState *st, int nslots, int mask, BParams p,
                                 hipStream_t s)
{
    hipLaunchKernelGGL(k_b_newton_check, dim3(nslots), dim3(256), 0, s, d, st, nslots, mask, p);
    return hipGetLastError();
}
hipError_t launch_b_jac(int prec, const BDesc *d, BState *st, int nslots, float tl, int grid,
                        hipStream_t s)
{
    switch (prec) {
    case N3P_FP16: hipLaunchKernelGGL(k_b_jac<f16>, dim3(grid), dim3(256), 0, s, d, st, nslots, tl); break;
    case N3P_BF16: hipLaunchKernelGGL(k_b_jac<bf16>, dim3(grid), dim3(256), 0, s, d, st, nslots, tl); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
hipError_t launch_b_ir_init(const BDesc *d, BState *st, int nslots, BParams p, hipStream_t s)
{
    hipLaunchKernelGGL(k_b_ir_init, dim3(nslots), dim3(256), 0, s, d, st, nslots, p);
    return hipGetLastError();
}
hipError_t launch_b_ir_check(const BDesc *d, BState *st, int nslots, BParams p, hipStream_t s)
{
    hipLaunchKernelGGL(k_b_ir_check, dim3(nslots), dim3(256), 0, s, d, st, nslots, p);
    return hipGetLastError();
}
hipError_t launch_b_ir_final(const BDesc *d, BState *st, int nslots, BParams p, hipStream_t s)
{
    hipLaunchKernelGGL(k_b_ir_final, dim3(nslots), dim3(256), 0, s, d, st, nslots, p);
    return hipGetLastError();
}

}  // namespace n3p
