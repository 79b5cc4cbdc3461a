// n3p_internal.hpp -- shared declarations of the gfx950 HIP implementation.
//
// Storage conventions (all kernels):
//   * matrices are column-major; the factorisation works on an Np x Np copy
//     with Np = n rounded up to a multiple of NB_PAD, padded with the
//     identity (the padded LU is the LU of J plus an identity block);
//   * "LT" is the L panel of the current outer block stored row-major
//     (K-contiguous) so that both operands of the Schur-complement GEMM feed
//     the matrix cores with contiguous K;
//   * "flags" is a small int array in the workspace:
//       [0] speculation failed (a pivot would have been interchanged)
//       [1] non-finite value produced
//       [2] first exactly-zero pivot (k+1), 0 if none
//       [3] device wait expired (bounded spins)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "n3p.h"

namespace n3p {

constexpr int NB_OUT = 1024;  // outer block: K of the big Schur-complement GEMM
constexpr int NB_PAD = 512;   // factorisation sizes are padded to a multiple of this
constexpr int NB_LEAF = 64;   // leaf panel width
constexpr int NB_MID = 256;   // middle level: leaves' rank-64 updates stay inside it
constexpr int TRSV_BS = 64;   // row block of the triangular solves
// the pivoting path keeps one row per thread in at most PIVOT_MAX_WG
// workgroups of 256 threads, all resident at once
constexpr int PIVOT_MAX_WG = 128;
constexpr int64_t PIVOT_MAX_NP = (int64_t)PIVOT_MAX_WG * 256;
constexpr int FLAG_FAIL = 0, FLAG_NONFINITE = 1, FLAG_ZEROPIV = 2, FLAG_TIMEOUT = 3;
constexpr int NFLAGS = 16;

typedef _Float16 f16;
typedef __bf16 bf16;

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// compute type of the factorisation arithmetic for a storage type
template <typename T> struct compute_of { typedef float type; };
template <> struct compute_of<double> { typedef double type; };

template <typename T> __device__ __forceinline__ T to_store(float v) { return (T)v; }
template <> __device__ __forceinline__ double to_store<double>(float v) { return (double)v; }
template <typename T> __device__ __forceinline__ T to_store_d(double v) { return (T)(float)v; }
template <> __device__ __forceinline__ double to_store_d<double>(double v) { return v; }

__device__ __forceinline__ float to_f32(f16 v) { return (float)v; }
__device__ __forceinline__ float to_f32(bf16 v) { return (float)v; }
__device__ __forceinline__ float to_f32(float v) { return v; }
__device__ __forceinline__ double to_f32(double v) { return v; }

__device__ __forceinline__ int ld_flag(const int *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void set_flag(int *p, int v)
{
    __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Block-uniform read of a device flag: thread 0 reads, the value is broadcast
// through LDS, so every thread of the block takes the same early-exit branch
// (a per-thread read could split a block around a barrier).
__device__ __forceinline__ int block_flag(const int *p)
{
    __shared__ int s_flag;
    if (threadIdx.x == 0) s_flag = ld_flag(p);
    __syncthreads();
    const int v = s_flag;
    __syncthreads();
    return v;
}

// Cross-lane broadcasts on the VALU path (no LDS round trip).
// lane_bcast: value held by lane `src` of the wavefront (src wave-uniform).
__device__ __forceinline__ float lane_bcast(float v, int src)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ __forceinline__ double lane_bcast(double v, int src)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// quad_bcast<K>: value held by lane K of each group of four lanes (DPP quad_perm).
template <int K> __device__ __forceinline__ float quad_bcast(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), K * 0x55, 0xF, 0xF, false));
}
template <int K> __device__ __forceinline__ double quad_bcast(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), K * 0x55, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), K * 0x55, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

inline size_t elem_size(int prec)
{
    switch (prec) {
    case N3P_FP16: case N3P_BF16: return 2;
    case N3P_FP32: return 4;
    case N3P_FP64: return 8;
    default: return 0;
    }
}

// ---------------------------------------------------------------- launchers
// (defined in the .hip files; all enqueue on `s` and return hipError_t)

// problem kernels
hipError_t launch_hinv(int64_t n, double *h, hipStream_t s);  // h[k] = 1/(k+1), k < 2n-1
hipError_t launch_heq_residual(int64_t n, double c, const double *x, const double *h, double *F,
                               double *D, hipStream_t s);
hipError_t launch_heq_jacobian(int64_t n, double c, const double *D, const double *h, float *J,
                               int64_t ldj, hipStream_t s);
// rowq: optional n-double scratch for the Jacobian's row factors (ignored
// for the FP64 factorisation, which keeps the division form)
hipError_t launch_heq_jac_round(int prec, int64_t n, int64_t Np, double c, const double *D,
                                const double *h, float *J, int64_t ldj, void *Ah, int64_t ldh,
                                float *colscale, float tl, int *flags, double *rowq, hipStream_t s);
hipError_t launch_dense_tanh_residual(int64_t n, const double *A, int64_t lda, const double *b,
                                      const double *x, double *F, double *part, hipStream_t s);
hipError_t launch_dense_tanh_jacobian(int64_t n, const double *A, int64_t lda, const double *x,
                                      float *J, int64_t ldj, hipStream_t s);
hipError_t launch_dense_tanh_jacobian_f64(int64_t n, int64_t Np, const double *A, int64_t lda,
                                          const double *x, float *J, int64_t ldj, double *Ah,
                                          int64_t ldh, hipStream_t s);
// J (FP32, n x n) -> padded Np x Np copy in prec, column scales (may be null)
hipError_t launch_round_scale(int prec, int64_t n, int64_t Np, const float *J, int64_t ldj,
                              void *Ah, int64_t ldh, float *colscale, float target_log2,
                              int *flags, hipStream_t s);
// copy a caller matrix (n x n, lda) in prec into the padded Np x Np buffer and back
hipError_t launch_pad_copy_in(int prec, int64_t n, int64_t Np, const void *A, int64_t lda,
                              void *Ap, hipStream_t s);
hipError_t launch_pad_copy_out(int prec, int64_t n, int64_t Np, const void *Ap, void *A,
                               int64_t lda, hipStream_t s);
hipError_t launch_copy_bytes(void *dst, const void *src, size_t bytes, hipStream_t s);

// reductions and vector kernels
hipError_t launch_nrm2_f64(int64_t n, const double *x, double *part, double *out, hipStream_t s);
hipError_t launch_nrm2_f32(int64_t n, const float *x, double *part, double *out, hipStream_t s);
hipError_t launch_fill_i32(int *p, int v, int64_t n, hipStream_t s);
// GPU-timeline timestamp (100 MHz real-time counter ticks) into *p
hipError_t launch_stamp(uint64_t *p, hipStream_t s);
constexpr double STAMP_MS_PER_TICK = 1e-5;
hipError_t launch_fill_f32(float *p, float v, int64_t n, hipStream_t s);
hipError_t launch_iota_i32(int32_t *p, int64_t n, hipStream_t s);
// b = -F / ||F|| (FP64 in, FP32 out, padded tail zeroed up to np)
hipError_t launch_rhs_unit(int64_t n, int64_t np, const double *F, const double *fnorm, float *b,
                           hipStream_t s);
hipError_t launch_rhs_unit_f64(int64_t n, int64_t np, const double *F, const double *fnorm,
                               double *b, hipStream_t s);
// dst = a * src
hipError_t launch_scal_copy_f32(int64_t n, float *dst, const float *src, double a, hipStream_t s);
// x += ||F|| * u  (u FP32 or FP64)
hipError_t launch_newton_update_f32(int64_t n, double *x, const double *fnorm, const float *u,
                                    hipStream_t s);
hipError_t launch_newton_update_f64(int64_t n, double *x, const double *fnorm, const double *u,
                                    hipStream_t s);
hipError_t launch_axpy_f32(int64_t n, float *y, const float *x, float a, hipStream_t s);
hipError_t launch_vcopy_f32(int64_t n, float *dst, const float *src, hipStream_t s);
hipError_t launch_f32_to_f64(int64_t n, const float *src, double *dst, hipStream_t s);
hipError_t launch_f64_to_f32(int64_t n, const double *src, float *dst, hipStream_t s);

// factorisation kernels
hipError_t launch_leaf_spec(int prec, int64_t Np, int64_t c0, void *A, int64_t lda, void *LT,
                            int64_t k0, int *flags, hipStream_t s);
hipError_t launch_gemm_pair(int prec, int64_t M1, int64_t N1, const void *At1, int64_t ldat1,
                            const void *B1, int64_t ldb1, void *C1, int64_t ldc1, int64_t M2,
                            int64_t N2, const void *At2, int64_t ldat2, const void *B2,
                            int64_t ldb2, void *C2, int64_t ldc2, int64_t K, int *flags,
                            hipStream_t s);
hipError_t launch_gemm_sub(int prec, int64_t M, int64_t N, int64_t K, const void *At,
                           int64_t ldat, const void *B, int64_t ldb, void *C, int64_t ldc,
                           int *flags, bool check_abort, hipStream_t s);
// no-interchange factorisation of one outer block (FP16 / BF16): the
// diagonal square (k_top) and the two triangular solves beside it (k_trsm);
// top_pub_words / top_inv_floats size their publication area and the
// inverses' side buffer
size_t top_pub_words();
size_t top_inv_floats();
hipError_t launch_top(int prec, int64_t k0, int W, void *A, int64_t lda, void *LT, uint64_t *pub,
                      float *inv, int *flags, uint32_t tag0, hipStream_t s);
// the next block's square (k_top) fused with the rest of this block's
// trailing update C[M x N] -= At^T B and C2[M2 x N2] -= At2^T B2 (256x256
// tiles; M, N, M2, N2 multiples of 256; M2 = 0 for one region; same K, ldat,
// ldb, ldc)
hipError_t launch_top_gemm(int prec, int64_t k0, int W, void *A, int64_t lda, void *LT,
                           uint64_t *pub, float *inv, int *flags, uint32_t tag0, int64_t M,
                           int64_t N, int64_t K, const void *At, int64_t ldat, const void *B,
                           int64_t ldb, void *C, int64_t ldc, int64_t M2, int64_t N2,
                           const void *At2, const void *B2, void *C2, hipStream_t s);
hipError_t launch_trsm(int prec, int64_t Np, int64_t k0, int W, void *A, int64_t lda, void *LT,
                       const float *inv, int *flags, hipStream_t s);
// pivoting path: exchange area size (bytes), its reset, the cooperative leaf
// panel, the row moves of its interchanges, the LT rebuild of an outer block
size_t pivot_xch_bytes(int prec, int64_t Np);
hipError_t launch_pivot_reset(int prec, int64_t Np, void *xch, hipStream_t s);
hipError_t launch_pivot_coop(int prec, int64_t Np, int64_t c0, int64_t k0, void *A, int64_t lda,
                             int32_t *ipiv, void *LT, void *xch, int *flags, hipStream_t s);
hipError_t launch_gather_u12(int prec, int64_t Np, int64_t c0, int64_t k0, int64_t kend, void *A,
                             int64_t lda, const void *xch, int *flags, hipStream_t s);
hipError_t launch_gather_block(int prec, int64_t Np, int64_t k0, int64_t kend, void *A,
                               int64_t lda, const void *xch, hipStream_t s);
hipError_t launch_lt_rebuild(int prec, int64_t Np, int64_t r0, int64_t k0, int64_t ncol,
                             const void *A, int64_t lda, void *LT, hipStream_t s);
hipError_t launch_u12(int prec, int64_t c0, int64_t col0, int64_t col1, void *A, int64_t lda,
                      int *flags, hipStream_t s);
hipError_t launch_check_factor_finite(int prec, int64_t Np, const void *A, int64_t lda,
                                      int *flags, hipStream_t s);

// measurement helper: the matrix-core rate (not a step of the method)
hipError_t launch_mfma_rate(int prec, int blocks, int iters, float *out, double *flops,
                            hipStream_t s);

// triangular solves and matvec
// round_out = 1: each solution entry rounded to the factor type as it is formed
hipError_t launch_trsv_lower(int prec, int64_t n, const void *LU, int64_t lda, const int32_t *perm,
                             const float *b, float *y, int *sync, uint32_t epoch, int *flags,
                             hipStream_t s, int round_out = 0);
hipError_t launch_trsv_upper(int prec, int64_t n, const void *LU, int64_t lda, const float *y,
                             const float *colscale, float *x, int *sync, uint32_t epoch, int *flags,
                             hipStream_t s, int round_out = 0);
// out = in * a rounded to the factor type of prec (held as FP32)
hipError_t launch_scale_round(int prec, int64_t n, const float *in, float a, float *out, hipStream_t s);
hipError_t launch_trsv_lower_f64(int64_t n, const double *LU, int64_t lda, const int32_t *perm,
                                 const double *b, double *y, int *sync, uint32_t epoch,
                                 int *flags, hipStream_t s);
hipError_t launch_trsv_upper_f64(int64_t n, const double *LU, int64_t lda, const double *y,
                                 double *x, int *sync, uint32_t epoch, int *flags, hipStream_t s);
hipError_t launch_gemv_resid(int64_t n, const float *A, int64_t lda, const float *u,
                             const float *b, float *r, double *part, hipStream_t s);
// the same r = b - A u with the partial sums in the library's fixed scratch
// (n <= N3P_GEMV_NOALLOC_MAX_N); allocates nothing
hipError_t launch_gemv_resid_noalloc(int64_t n, const float *A, int64_t lda, const float *u,
                                     const float *b, float *r, hipStream_t s);
// y = A v (FP32 out) for GMRES
hipError_t launch_gemv_f32(int64_t n, const float *A, int64_t lda, const float *v, float *y,
                           double *part, hipStream_t s);
// modified Gram-Schmidt step: w against V[0..j], H column out, V[j+1] = w/h
hipError_t launch_mgs(int64_t n, float *V, int64_t ldv, int j, float *w, double *Hcol,
                      hipStream_t s);
// d += V[0..k) y
hipError_t launch_krylov_update(int64_t n, const float *V, int64_t ldv, int k, const double *y,
                                float *d, hipStream_t s);

size_t trsv_sync_ints(int64_t n);


// ------------------------------------------------ FFT form of the H-equation
int fft_length(int64_t n);  // power of two >= 2n - 1 (0 if n > 32768)
hipError_t launch_hk_setup(int64_t n, int L, double2 *tw, double2 *H, double2 *t1, double2 *t2,
                           hipStream_t s);
hipError_t launch_hk_residual(int64_t n, int L, double c, const double *x, const double2 *tw,
                              const double2 *H, double2 *t1, double2 *t2, double2 *W, double *F,
                              double *D, hipStream_t s);
// out = b - J v (b non-null) or J v, rows n .. np-1 of out set to 0
hipError_t launch_hk_jv(int64_t n, int64_t np, int L, double c, const double *D, const float *v,
                        const float *b, float *out, const double2 *tw, const double2 *H,
                        double2 *t1, double2 *t2, double2 *W, hipStream_t s);

// ============================================================ batched engine
// Many independent H-equation solves advance together, one Newton step per
// round: every kernel below walks a table of slots.  BDesc is written by the
// host when a request is admitted; BState is written only by the kernels and
// read back by the host after each step.  A slot's arithmetic never depends on
// which other slots are present (no reductions across slots), so a request's
// result is the same alone and in any mix.
constexpr int B_LEAF = NB_LEAF;      // leaf width and padding granule (64)
constexpr int B_MAX_NP = 4096;       // largest padded size of a batched solve
constexpr int B_SOLVE_THREADS = 1024;

constexpr int B_MAX_SLOTS = 256;

enum BPhase { BP_FREE = 0, BP_FRESH = 1, BP_RUN = 2, BP_DONE = 3 };

// Work items of a batched launch: slot s contributes cnt(s) items.  Every
// workgroup builds the same prefix table in LDS (off[0 .. nslots]) and walks
// items blockIdx.x, blockIdx.x + gridDim.x, ...  b_find returns the slot of an
// item (the largest s with off[s] <= item, which skips empty slots).
template <typename Cnt>
__device__ __forceinline__ int b_offsets(int nslots, int *off, Cnt cnt)
{
    for (int t = threadIdx.x; t < nslots; t += blockDim.x) off[t + 1] = cnt(t);
    __syncthreads();
    if (threadIdx.x == 0) {
        off[0] = 0;
        for (int i = 0; i < nslots; ++i) off[i + 1] += off[i];
    }
    __syncthreads();
    return off[nslots];
}
__device__ __forceinline__ int b_find(const int *off, int nslots, int item)
{
    int lo = 0, hi = nslots - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

struct BDesc {
    int64_t n, Np;
    double c;
    int prec;            // N3P_FP16 or N3P_BF16
    int pad_;
    void *A;             // factor buffer, Np x Np column-major (ld Np), identity padding
    void *LT;            // L of the current leaf, transposed: row i at LT + 64 i
    void *DG;            // 2 x 64 x 64 factored diagonal blocks
    float *J;            // n x n FP32 Jacobian, ld n
    float *colscale;     // Np
    double *x, *F, *D, *h;          // n, n, n, 2n
    float *b, *u, *uprev, *r, *y;   // Np each
    int *flags;          // NFLAGS
};

struct BState {
    int phase, status, its, factor;
    int ir_on, sweeps, ir_failed, pad_;
    double f0, fn, tau, nb, rn;
    double rel[N3P_MAX_HIST];        // ||F_k|| / ||F_0||
    int lin[N3P_MAX_HIST];           // IR sweeps at step k+1
};

struct BParams {                     // per-engine constants
    double tau_r, tau_a, eta;
    int maxit, max_sweeps;
    float target_log2;
    int pad_;
};

// launchers (grid sizes are the engine's, from its tuning table)
hipError_t launch_b_residual(const BDesc *d, BState *st, int nslots, int phase_mask, int grid,
                             hipStream_t s);
hipError_t launch_b_newton_check(const BDesc *d, BState *st, int nslots, int phase_mask,
                                 BParams p, hipStream_t s);
hipError_t launch_b_jac(int prec, const BDesc *d, BState *st, int nslots, float tl, int grid,
                        hipStream_t s);
hipError_t launch_b_leaf(int prec, const BDesc *d, const BState *st, int nslots, int leaf,
                         int grid, hipStream_t s);
hipError_t launch_b_gemm(int prec, const BDesc *d, const BState *st, int nslots, int leaf,
                         int kc, int grid, hipStream_t s);
hipError_t launch_b_ir_init(const BDesc *d, BState *st, int nslots, BParams p, hipStream_t s);
hipError_t launch_b_solve(int prec, const BDesc *d, const BState *st, int nslots,
                          hipStream_t s);
hipError_t launch_b_gemv(const BDesc *d, const BState *st, int nslots, int grid, hipStream_t s);
hipError_t launch_b_ir_check(const BDesc *d, BState *st, int nslots, BParams p, hipStream_t s);
hipError_t launch_b_ir_final(const BDesc *d, BState *st, int nslots, BParams p, hipStream_t s);
hipError_t launch_b_fill_x0(const BDesc *d, const BState *st, int nslots, hipStream_t s);

}  // namespace n3p
