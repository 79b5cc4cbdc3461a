// k_solve.hip -- the preconditioner-vector product U^{-1} L^{-1} P r
// (Section 2.2) and the single-precision residual r = b - A u.
//
// Triangular solves: one persistent launch per solve.  Row blocks of BS rows
// are taken in dependency order through an atomic ticket (a block only waits
// on blocks with smaller tickets, which are already running, so the waits
// always end).  Block i accumulates the contributions of finished blocks as
// they are published, then substitutes its diagonal block in one wavefront
// and publishes its piece of the solution with a per-block flag holding the
// launch's epoch (no flag reset between launches).  Factors are read in their
// storage precision and promoted in registers (interprecision transfer on
// the fly, Section 2.3).  Every wait is bounded; an expired wait raises
// FLAG_TIMEOUT and the block proceeds so that the grid always drains.
#include <algorithm>

#include "n3p_internal.hpp"

namespace n3p {

constexpr int SPIN_LIMIT = 1 << 24;

__device__ __forceinline__ bool wait_epoch(int *f, uint32_t epoch, int *flags)
{
    int spins = 0;
    while ((uint32_t)__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins > SPIN_LIMIT) {
            set_flag(&flags[FLAG_TIMEOUT], 1);
            return false;
        }
    }
    return true;
}

template <typename V> __device__ __forceinline__ V shfl_v(V v, int src) { return __shfl(v, src); }

// ---------------------------------------------------------------- lower
// y = L^{-1} (P b): L unit lower (below the diagonal of LU), perm[i] = the
// original row placed at position i (null = identity).
template <typename T, typename V, int BS>
__global__ __launch_bounds__(256) void k_trsv_lower(int64_t n, const T *__restrict__ LU, int64_t lda,
                                                    const int32_t *__restrict__ perm,
                                                    const V *__restrict__ b, V *__restrict__ y,
                                                    int *__restrict__ sync, uint32_t epoch,
                                                    int *__restrict__ flags)
{
    __shared__ int s_blk;
    __shared__ V ysh[BS];
    __shared__ V part[4][BS];
    const int tid = threadIdx.x;
    if (tid == 0) s_blk = __hip_atomic_fetch_add(&sync[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int blk = s_blk;
    const int64_t r0 = (int64_t)blk * BS;
    const int r = tid % BS, g = tid / BS;
    const int64_t row = r0 + r;
    const bool rv = row < n;
    V acc = 0;
    for (int jb = 0; jb < blk; ++jb) {
        if (tid == 0) wait_epoch(&sync[1 + jb], epoch, flags);
        __syncthreads();
        __hip_atomic_load(&sync[1 + jb], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        if (tid < BS) ysh[tid] = __hip_atomic_load(&y[(int64_t)jb * BS + tid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        if (rv) {
            const T *lp = LU + row + (int64_t)jb * BS * lda;
#pragma unroll 4
            for (int c = g; c < BS; c += 4) acc += (V)to_f32(lp[(int64_t)c * lda]) * ysh[c];
        }
        __syncthreads();
    }
    part[g][r] = acc;
    __syncthreads();
    if (tid < 64) {
        // one wavefront: lane r owns row r0 + r (BS == 64)
        V z = 0;
        if (rv) {
            const int64_t src = perm ? (int64_t)perm[row] : row;
            z = b[src] - (part[0][r] + part[1][r] + part[2][r] + part[3][r]);
        }
        V ld[BS];
#pragma unroll
        for (int c = 0; c < BS; ++c) {
            const int64_t col = r0 + c;
            ld[c] = (rv && col < n && c < r) ? (V)to_f32(LU[row + col * lda]) : (V)0;
        }
#pragma unroll
        for (int c = 0; c < BS; ++c) {
            const V yc = shfl_v(z, c);
            if (r > c) z -= ld[c] * yc;
        }
        if (rv) __hip_atomic_store(&y[row], z, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (tid == 0) __hip_atomic_store(&sync[1 + blk], (int)epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ---------------------------------------------------------------- upper
// x = S U^{-1} y with S = diag(colscale) (null = identity).  Blocks run from
// the last to the first; xs holds the unscaled solution other blocks read.
template <typename T, typename V, int BS>
__global__ __launch_bounds__(256) void k_trsv_upper(int64_t n, const T *__restrict__ LU, int64_t lda,
                                                    const V *__restrict__ yin,
                                                    const float *__restrict__ colscale,
                                                    V *__restrict__ x, V *__restrict__ xs,
                                                    int *__restrict__ sync, uint32_t epoch,
                                                    int *__restrict__ flags)
{
    __shared__ int s_blk;
    __shared__ V xsh[BS];
    __shared__ V part[4][BS];
    const int tid = threadIdx.x;
    const int nb = (int)((n + BS - 1) / BS);
    if (tid == 0) s_blk = nb - 1 - __hip_atomic_fetch_add(&sync[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int blk = s_blk;
    const int64_t r0 = (int64_t)blk * BS;
    const int r = tid % BS, g = tid / BS;
    const int64_t row = r0 + r;
    const bool rv = row < n;
    V acc = 0;
    for (int jb = nb - 1; jb > blk; --jb) {
        if (tid == 0) wait_epoch(&sync[1 + jb], epoch, flags);
        __syncthreads();
        __hip_atomic_load(&sync[1 + jb], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        if (tid < BS) {
            const int64_t ix = (int64_t)jb * BS + tid;
            xsh[tid] = ix < n ? __hip_atomic_load(&xs[ix], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : (V)0;
        }
        __syncthreads();
        if (rv) {
            const int64_t c0 = (int64_t)jb * BS;
            const int cmax = (int)std::min<int64_t>(BS, n - c0);
            const T *up = LU + row + c0 * lda;
#pragma unroll 4
            for (int c = g; c < cmax; c += 4) acc += (V)to_f32(up[(int64_t)c * lda]) * xsh[c];
        }
        __syncthreads();
    }
    part[g][r] = acc;
    __syncthreads();
    if (tid < 64) {
        V z = rv ? yin[row] - (part[0][r] + part[1][r] + part[2][r] + part[3][r]) : (V)0;
        V ud[BS];
#pragma unroll
        for (int c = 0; c < BS; ++c) {
            const int64_t col = r0 + c;
            ud[c] = (rv && col < n && c >= r) ? (V)to_f32(LU[row + col * lda]) : (V)0;
        }
        const V dii = rv ? ud[0] : (V)1;  // placeholder, replaced below
        (void)dii;
        V diag = (V)1;
#pragma unroll
        for (int c = 0; c < BS; ++c)
            if (c == r && rv) diag = ud[c];
#pragma unroll
        for (int c = BS - 1; c >= 0; --c) {
            if (r == c) z = z / diag;
            const V xc = shfl_v(z, c);
            if (r < c) z -= ud[c] * xc;
        }
        if (rv) {
            __hip_atomic_store(&xs[row], z, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            x[row] = colscale ? z * (V)colscale[row] : z;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (tid == 0) __hip_atomic_store(&sync[1 + blk], (int)epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ void k_zero_ticket(int *sync) { sync[0] = 0; }

size_t trsv_sync_ints(int64_t n) { return (size_t)(2 + (n + TRSV_BS - 1) / TRSV_BS); }

template <typename T, typename V>
static hipError_t trsv_lower_t(int64_t n, const void *LU, int64_t lda, const int32_t *perm,
                               const V *b, V *y, int *sync, uint32_t epoch, int *flags,
                               hipStream_t s)
{
    const unsigned nb = (unsigned)((n + TRSV_BS - 1) / TRSV_BS);
    hipLaunchKernelGGL(k_zero_ticket, dim3(1), dim3(1), 0, s, sync);
    hipLaunchKernelGGL((k_trsv_lower<T, V, TRSV_BS>), dim3(nb), dim3(256), 0, s, n, (const T *)LU,
                       lda, perm, b, y, sync, epoch, flags);
    return hipGetLastError();
}

template <typename T, typename V>
static hipError_t trsv_upper_t(int64_t n, const void *LU, int64_t lda, const V *y,
                               const float *colscale, V *x, V *xs, int *sync, uint32_t epoch,
                               int *flags, hipStream_t s)
{
    const unsigned nb = (unsigned)((n + TRSV_BS - 1) / TRSV_BS);
    hipLaunchKernelGGL(k_zero_ticket, dim3(1), dim3(1), 0, s, sync);
    hipLaunchKernelGGL((k_trsv_upper<T, V, TRSV_BS>), dim3(nb), dim3(256), 0, s, n, (const T *)LU,
                       lda, y, colscale, x, xs, sync, epoch, flags);
    return hipGetLastError();
}

hipError_t launch_trsv_lower(int prec, int64_t n, const void *LU, int64_t lda, const int32_t *perm,
                             const float *b, float *y, int *sync, uint32_t epoch, int *flags,
                             hipStream_t s)
{
    switch (prec) {
    case N3P_FP16: return trsv_lower_t<f16, float>(n, LU, lda, perm, b, y, sync, epoch, flags, s);
    case N3P_BF16: return trsv_lower_t<bf16, float>(n, LU, lda, perm, b, y, sync, epoch, flags, s);
    case N3P_FP32: return trsv_lower_t<float, float>(n, LU, lda, perm, b, y, sync, epoch, flags, s);
    case N3P_FP64: return trsv_lower_t<double, float>(n, LU, lda, perm, b, y, sync, epoch, flags, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_trsv_upper(int prec, int64_t n, const void *LU, int64_t lda, const float *y,
                             const float *colscale, float *x, float *yscratch, int *sync,
                             uint32_t epoch, int *flags, hipStream_t s)
{
    switch (prec) {
    case N3P_FP16: return trsv_upper_t<f16, float>(n, LU, lda, y, colscale, x, yscratch, sync, epoch, flags, s);
    case N3P_BF16: return trsv_upper_t<bf16, float>(n, LU, lda, y, colscale, x, yscratch, sync, epoch, flags, s);
    case N3P_FP32: return trsv_upper_t<float, float>(n, LU, lda, y, colscale, x, yscratch, sync, epoch, flags, s);
    case N3P_FP64: return trsv_upper_t<double, float>(n, LU, lda, y, colscale, x, yscratch, sync, epoch, flags, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_trsv_lower_f64(int64_t n, const double *LU, int64_t lda, const int32_t *perm,
                                 const double *b, double *y, int *sync, uint32_t epoch, int *flags,
                                 hipStream_t s)
{
    return trsv_lower_t<double, double>(n, LU, lda, perm, b, y, sync, epoch, flags, s);
}

hipError_t launch_trsv_upper_f64(int64_t n, const double *LU, int64_t lda, const double *y,
                                 double *x, double *yscratch, int *sync, uint32_t epoch, int *flags,
                                 hipStream_t s)
{
    return trsv_upper_t<double, double>(n, LU, lda, y, nullptr, x, yscratch, sync, epoch, flags, s);
}

// ---------------------------------------------------------------- matvec
// Partial sums of A u over column chunks (FP64 accumulation of FP32 data),
// then a fixed-order reduction: r = b - sum (b may be null: r = sum).
constexpr int MV_ROWS = 256, MV_CH = 256;

__global__ __launch_bounds__(256) void k_gemv_f32_part(int64_t n, const float *__restrict__ A,
                                                       int64_t lda, const float *__restrict__ u,
                                                       double *__restrict__ part)
{
    __shared__ float ush[MV_CH];
    const int64_t j0 = (int64_t)blockIdx.y * MV_CH;
    const int64_t jn = std::min<int64_t>(MV_CH, n - j0);
    if (threadIdx.x < jn) ush[threadIdx.x] = u[j0 + threadIdx.x];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * MV_ROWS + threadIdx.x;
    if (i >= n) return;
    const float *ap = A + i + j0 * lda;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int64_t c = 0;
    for (; c + 4 <= jn; c += 4) {
        s0 += (double)ap[(c + 0) * lda] * (double)ush[c + 0];
        s1 += (double)ap[(c + 1) * lda] * (double)ush[c + 1];
        s2 += (double)ap[(c + 2) * lda] * (double)ush[c + 2];
        s3 += (double)ap[(c + 3) * lda] * (double)ush[c + 3];
    }
    for (; c < jn; ++c) s0 += (double)ap[c * lda] * (double)ush[c];
    part[(int64_t)blockIdx.y * n + i] = (s0 + s1) + (s2 + s3);
}

__global__ void k_gemv_finish(int64_t n, int nch, const double *__restrict__ part,
                              const float *__restrict__ b, float *__restrict__ r)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int c = 0; c < nch; ++c) s += part[(int64_t)c * n + i];
    r[i] = b ? (float)((double)b[i] - s) : (float)s;
}

hipError_t launch_gemv_resid(int64_t n, const float *A, int64_t lda, const float *u, const float *b,
                             float *r, double *part, hipStream_t s)
{
    const int nch = (int)((n + MV_CH - 1) / MV_CH);
    hipLaunchKernelGGL(k_gemv_f32_part, dim3((unsigned)((n + MV_ROWS - 1) / MV_ROWS), nch),
                       dim3(256), 0, s, n, A, lda, u, part);
    hipLaunchKernelGGL(k_gemv_finish, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, nch,
                       (const double *)part, b, r);
    return hipGetLastError();
}

hipError_t launch_gemv_f32(int64_t n, const float *A, int64_t lda, const float *v, float *y,
                           double *part, hipStream_t s)
{
    return launch_gemv_resid(n, A, lda, v, nullptr, y, part, s);
}

// ----------------------------------------------------------------- GMRES
// Modified Gram-Schmidt on one workgroup: for i = 0..j, h_i = <V_i, w>,
// w -= h_i V_i (sequentially, as MGS prescribes); h_{j+1} = ||w||,
// V_{j+1} = w / h_{j+1}.  Dots accumulate in FP64.
__device__ double block_sum_1024(double v, double *sh)
{
    const int t = threadIdx.x;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((t & 63) == 0) sh[t >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (t == 0) {
        for (int w = 0; w < 16; ++w) s += sh[w];
        sh[16] = s;
    }
    __syncthreads();
    s = sh[16];
    __syncthreads();
    return s;
}

__global__ __launch_bounds__(1024) void k_mgs(int64_t n, float *__restrict__ V, int64_t ldv, int j,
                                              float *__restrict__ w, double *__restrict__ Hcol)
{
    __shared__ double sh[17];
    const int t = threadIdx.x;
    for (int i = 0; i <= j; ++i) {
        const float *vi = V + (int64_t)i * ldv;
        double d = 0.0;
        for (int64_t k = t; k < n; k += 1024) d += (double)vi[k] * (double)w[k];
        const double h = block_sum_1024(d, sh);
        const float hf = (float)h;
        for (int64_t k = t; k < n; k += 1024) w[k] -= hf * vi[k];
        if (t == 0) Hcol[i] = h;
        __syncthreads();
    }
    double q = 0.0;
    for (int64_t k = t; k < n; k += 1024) q += (double)w[k] * (double)w[k];
    const double hn = sqrt(block_sum_1024(q, sh));
    if (t == 0) Hcol[j + 1] = hn;
    float *vn = V + (int64_t)(j + 1) * ldv;
    const float inv = hn > 0.0 ? (float)(1.0 / hn) : 0.0f;
    for (int64_t k = t; k < n; k += 1024) vn[k] = w[k] * inv;
}

__global__ void k_krylov_update(int64_t n, const float *__restrict__ V, int64_t ldv, int k,
                                const double *__restrict__ y, float *__restrict__ d)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int q = 0; q < k; ++q) s += (double)V[(int64_t)q * ldv + i] * y[q];
    d[i] = (float)((double)d[i] + s);
}

hipError_t launch_mgs(int64_t n, float *V, int64_t ldv, int j, float *w, double *Hcol, hipStream_t s)
{
    hipLaunchKernelGGL(k_mgs, dim3(1), dim3(1024), 0, s, n, V, ldv, j, w, Hcol);
    return hipGetLastError();
}

hipError_t launch_krylov_update(int64_t n, const float *V, int64_t ldv, int k, const double *y,
                                float *d, hipStream_t s)
{
    hipLaunchKernelGGL(k_krylov_update, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, V,
                       ldv, k, y, d);
    return hipGetLastError();
}

}  // namespace n3p
