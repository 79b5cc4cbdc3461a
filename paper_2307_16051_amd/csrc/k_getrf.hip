// k_getrf.hip -- blocked right-looking LU with partial pivoting for gfx950.
//
// The factorisation (Gaussian elimination, Section 1.3; the half-precision
// factorisation J_h = L U of Section 2) runs on the padded Np x Np copy:
//
//   for each outer block of NB_OUT columns (1024; sizes padded to 512):
//     for each leaf of NB_LEAF columns inside it:
//       leaf kernel   -- factor the leaf, form L21 and the U row block
//       inner GEMMs   -- update the rest of the outer block (K = NB_LEAF)
//     outer GEMM      -- Schur complement of the trailing matrix (K = NB_OUT)
//
// Pivoting: the leaf kernel first tries the diagonal as pivot and verifies,
// column by column, that every candidate below it is smaller in magnitude by
// a margin (|a_ij| <= (1 - 2^-8) |a_jj|).  When that holds for every column,
// partial pivoting (largest magnitude, ties to the lowest row) selects the
// diagonal at every step, so the no-interchange factorisation IS the
// partial-pivoting one.  If any column fails the test, a flag aborts the
// remaining kernels and the host re-runs the factorisation with explicit
// pivot searches and row interchanges (k_pivot.hip).  Near-ties
// always take the explicit path, so rounding differences cannot change a
// pivot decision.
//
// The Schur-complement GEMMs use the matrix cores: FP16/BF16 inputs with FP32
// accumulation (v_mfma_f32_32x32x16_{f16,bf16}), rounded to the storage type
// once per GEMM; FP32 and FP64 use v_mfma_{f32,f64}_16x16x4.
#include <algorithm>

#include "n3p_gemm.hpp"

namespace n3p {

// oct_bcast<K>: value held by lane K of each group of eight lanes.  A quad
// broadcast gives every quad its own lane K % 4; the quad of the octet that
// does not hold lane K then takes it from its neighbour quad by a row shift of
// four lanes, written only to that quad's banks.
template <int K> __device__ __forceinline__ int oct_bcast_i(int v)
{
    const int qb = __builtin_amdgcn_mov_dpp(v, (K & 3) * 0x55, 0xF, 0xF, false);
    if (K < 4) return __builtin_amdgcn_update_dpp(qb, qb, 0x114, 0xF, 0xA, false);  // row_shr:4
    return __builtin_amdgcn_update_dpp(qb, qb, 0x104, 0xF, 0x5, false);             // row_shl:4
}
template <int K> __device__ __forceinline__ float oct_bcast(float v)
{
    return __int_as_float(oct_bcast_i<K>(__float_as_int(v)));
}
template <int K> __device__ __forceinline__ double oct_bcast(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = oct_bcast_i<K>((int)(b & 0xffffffffLL));
    const int hi = oct_bcast_i<K>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// recip: 1/v.  FP32: hardware reciprocal estimate refined by one Newton-Raphson
// step (r + r(1 - v r)), within an ulp of the rounded quotient; FP64: division.
__device__ __forceinline__ float recip(float v)
{
    const float r = __builtin_amdgcn_rcpf(v);
    return fmaf(fmaf(-v, r, 1.0f), r, r);
}
__device__ __forceinline__ double recip(double v) { return 1.0 / v; }

// =========================================================== leaf (no-swap)
// Tile b < nrt: 64 rows of L21 below the leaf; nrt <= b < nrt + nct: 64
// columns of the U row block to the right of the leaf (when the leaf is the
// last one, a single tile only stores the diagonal block).  Every workgroup
// first factors the 64x64 diagonal block itself (identical arithmetic in
// every workgroup), so none waits for another.  The factored diagonal block
// goes to DG (a side buffer): workgroups still reading the unfactored block
// from A must not see it change; with DG null (allowed only when the leaf has
// no tiles) it goes straight to A.  DGprev (if non-null) is the previous
// leaf's diagonal block, copied into A by tile 0 (nothing else touches that
// region now).  L21 is also written transposed to LT (row i at
// LT + i * ldlt + ltcol, K contiguous) for the Schur update.
//
// Every column step is a short dependent chain, so the work stays on the
// VALU path: the diagonal LU is blocked by 8-column strips held one row per
// lane (readlane broadcasts, one barrier per strip); the triangular solves
// use eight lanes per row or column (DPP broadcasts, no barrier).  Column
// loops run in groups whose index is a runtime loop while the steps inside
// are unrolled; per-lane register arrays rotate after each group so every
// register index stays static.
constexpr int LEAF_THREADS = 512;

template <typename T>
__device__ __forceinline__ void leaf_body(int bid, int64_t Np, int64_t c0, T *__restrict__ A,
                                          int64_t lda, T *__restrict__ LT, int64_t ldlt,
                                          int64_t ltcol, int nrt, int nct, T *__restrict__ DG,
                                          const T *__restrict__ DGprev, int64_t cprev,
                                          int *__restrict__ flags)
{
    typedef typename compute_of<T>::type CT;
    constexpr int L = NB_LEAF;
    constexpr int LP = L + 5;  // staging row stride: column chunks conflict-free, octet accesses 2-way
    constexpr int NT = LEAF_THREADS;
    // diagonal block; odd row stride, so the column accesses (lane = row)
    // of the strips hit 64 different banks
    __shared__ __attribute__((aligned(16))) CT Dm[L][L + 1];
    // Per column group kc of the tile solves: Ui[kc][kq][g][c] =
    // U[8kc+kq][8(kc+c)+g] and Li[kc][kq][g][u] = L[8(kc+u)+g][8kc+kq] where
    // kc + c <= 7 and that index exceeds the row (column) 8kc+kq, else 0 -- so
    // a lane's 8 coefficients of one step are contiguous and 16-byte aligned.
    __shared__ __attribute__((aligned(16))) CT Ui[L * L];
    __shared__ __attribute__((aligned(16))) CT Li[L * L];
    __shared__ __attribute__((aligned(16))) CT Sg[L][LP];       // staging of one tile
    __shared__ CT rdiag[L];
    __shared__ int sfail;
    if (block_flag(&flags[FLAG_FAIL])) return;
    const int t = threadIdx.x;
    if (bid == 0 && DGprev) {
        for (int e = t; e < L * L; e += NT) {
            const int i = e % L, j = e / L;
            A[(cprev + i) + (cprev + j) * lda] = DGprev[i + j * L];
        }
    }
    if (t == 0) sfail = 0;
    constexpr int CH = 16 / (int)sizeof(T);  // elements per 16-byte chunk
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    union Chunk { u32x4 v; T e[CH]; };
    for (int e = t; e < L * L / CH; e += NT) {  // diagonal block, column chunks
        const int i0 = (e % (L / CH)) * CH, j = e / (L / CH);
        Chunk ch;
        ch.v = *(const u32x4 *)(A + (c0 + i0) + (c0 + j) * lda);
#pragma unroll
        for (int u = 0; u < CH; ++u) Dm[i0 + u][j] = (CT)to_f32(ch.e[u]);
    }
    // this workgroup's tile (64 rows of L21 or 64 columns of U12), loaded now
    // into registers so the loads overlap the diagonal factorisation
    constexpr int NPRE = L * L / CH / NT;
    const T *tsrc = nullptr;
    if (bid < nrt) tsrc = A + (c0 + L + (int64_t)bid * L) + c0 * lda;
    else if (bid - nrt < nct) tsrc = A + c0 + (c0 + L + (int64_t)(bid - nrt) * L) * lda;
    u32x4 pre[NPRE];
    if (tsrc) {
#pragma unroll
        for (int k = 0; k < NPRE; ++k) {
            const int e = t + k * NT, i0 = (e % (L / CH)) * CH, j = e / (L / CH);
            pre[k] = *(const u32x4 *)(tsrc + i0 + j * lda);
        }
    }
    __syncthreads();
    const CT margin = (CT)(1.0 - 1.0 / 256.0);
    // ---- diagonal block, no interchange, with the partial-pivoting check.
    // Blocked by 8-column strips: wave w keeps columns 8w .. 8w+7 of all 64
    // rows in registers (lane = row).  For panel p, wave p factors its strip
    // (pivot row entries by readlane, no barrier inside the panel) and stores
    // it; after one barrier every later wave applies the panel to its own
    // strip: row k of the strip is final when step k starts, so it is read
    // by readlane and the multipliers of the panel come from LDS.
    {
        const int w = t / 64, r = t % 64;
        CT x[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) x[c] = Dm[r][8 * w + c];
        bool fail = false;
        for (int p = 0; p < 8; ++p) {
            if (w == p) {
#pragma unroll
                for (int kk = 0; kk < 8; ++kk) {
                    const int k = 8 * p + kk;
                    // branch-free (selects, no exec-mask branches): this is the
                    // leaf's serial chain
                    const CT piv = lane_bcast(x[kk], k);
                    const CT rp = recip(piv);
                    const bool below = r > k;
                    const CT lx = x[kk] * rp;
                    fail |= !(fabs(piv) > (CT)0) || (below && !(fabs(x[kk]) <= margin * fabs(piv)));
                    const CT l = below ? lx : (CT)0;
                    x[kk] = below ? lx : x[kk];
#pragma unroll
                    for (int c = kk + 1; c < 8; ++c) x[c] -= l * lane_bcast(x[c], k);
                }
#pragma unroll
                for (int c = 0; c < 8; ++c) Dm[r][8 * p + c] = x[c];
            }
            __syncthreads();
            if (w > p) {
                CT l[8];
#pragma unroll
                for (int kk = 0; kk < 8; ++kk) l[kk] = r > 8 * p + kk ? Dm[r][8 * p + kk] : (CT)0;
#pragma unroll
                for (int kk = 0; kk < 8; ++kk)
#pragma unroll
                    for (int c = 0; c < 8; ++c) x[c] -= l[kk] * lane_bcast(x[c], 8 * p + kk);
            }
        }
        if (fail) sfail = 1;
    }
    __syncthreads();
    if (sfail) {  // block-uniform: settled before the barrier
        if (t == 0) set_flag(&flags[FLAG_FAIL], 1);
        return;
    }
    for (int e = t; e < L * L; e += NT) {
        const int c = e % 8, g = (e / 8) % 8, kq = (e / 64) % 8, kc = e / 512;
        const int k = 8 * kc + kq, j = 8 * (kc + c) + g;
        const bool in = kc + c <= 7 && j > k;
        Ui[e] = in ? Dm[k][j] : (CT)0;
        Li[e] = in ? Dm[j][k] : (CT)0;
    }
    if (t < L) rdiag[t] = (CT)1 / Dm[t][t];
    if (bid == 0) {
        for (int e = t; e < L * L; e += NT) {
            const int i = e % L, j = e / L;
            const T v = to_store_d<T>((double)Dm[i][j]);
            if (DG) DG[i + j * L] = v;
            else A[(c0 + i) + (c0 + j) * lda] = v;
        }
    }
    __syncthreads();
    const int g = t % 8, w8 = t / 8;  // lane-in-octet, octet index (row or column)
    bool bad = false, fail = false;
    if (bid < nrt) {
        // ---- L21 rows [R0, R0+64): l U11 = a.  Octet w8 owns row R0 + w8;
        // lane g holds columns 8(c + kc) + g of the current group kc.  At step
        // k the owner lane (g = k % 8, slot 0) holds the Schur complement entry
        // partial pivoting would compare: it checks it against the pivot,
        // scales it and broadcasts it to its octet.
        const int64_t R0 = c0 + L + (int64_t)bid * L;
#pragma unroll
        for (int k = 0; k < NPRE; ++k) {  // the prefetched column chunks
            const int e = t + k * NT, i0 = (e % (L / CH)) * CH, j = e / (L / CH);
            Chunk ch;
            ch.v = pre[k];
#pragma unroll
            for (int u = 0; u < CH; ++u) Sg[i0 + u][j] = (CT)to_f32(ch.e[u]);
        }
        __syncthreads();
        CT x[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) x[c] = Sg[w8][8 * c + g];
        for (int kc = 0; kc < 8; ++kc) {
            CT u[8][8];
#pragma unroll
            for (int kq = 0; kq < 8; ++kq)
#pragma unroll
                for (int c = 0; c < 8; ++c) u[kq][c] = Ui[((kc * 8 + kq) * 8 + g) * 8 + c];
            // this lane owns column 8kc + g: its pivot bound and reciprocal
            const CT lim = margin * fabs(Dm[8 * kc + g][8 * kc + g]);
            const CT rd = rdiag[8 * kc + g];
#pragma unroll
            for (int kq = 0; kq < 8; ++kq) {
                const bool own = g == kq;  // branch-free, as in the diagonal chain
                fail |= own && !(fabs(x[0]) <= lim);
                x[0] = own ? x[0] * rd : x[0];
                CT xk;
                switch (kq) {
                case 0: xk = oct_bcast<0>(x[0]); break;
                case 1: xk = oct_bcast<1>(x[0]); break;
                case 2: xk = oct_bcast<2>(x[0]); break;
                case 3: xk = oct_bcast<3>(x[0]); break;
                case 4: xk = oct_bcast<4>(x[0]); break;
                case 5: xk = oct_bcast<5>(x[0]); break;
                case 6: xk = oct_bcast<6>(x[0]); break;
                default: xk = oct_bcast<7>(x[0]); break;
                }
#pragma unroll
                for (int c = 0; c < 8; ++c) x[c] -= xk * u[kq][c];
            }
            Sg[w8][8 * kc + g] = x[0];
#pragma unroll
            for (int c = 0; c < 7; ++c) x[c] = x[c + 1];
            x[7] = 0;
        }
        __syncthreads();
        for (int e = t; e < L * L / CH; e += NT) {  // A: column chunks
            const int i0 = (e % (L / CH)) * CH, j = e / (L / CH);
            Chunk ch;
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                ch.e[u] = to_store_d<T>((double)Sg[i0 + u][j]);
                bad |= !isfinite(to_f32(ch.e[u]));  // the stored value
            }
            *(u32x4 *)(A + (R0 + i0) + (c0 + j) * lda) = ch.v;
        }
        for (int e = t; e < L * L / CH; e += NT) {  // LT: row chunks (K contiguous)
            const int i = e / (L / CH), j0 = (e % (L / CH)) * CH;
            Chunk ch;
#pragma unroll
            for (int u = 0; u < CH; ++u) ch.e[u] = to_store_d<T>((double)Sg[i][j0 + u]);
            *(u32x4 *)(LT + (R0 + i) * ldlt + ltcol + j0) = ch.v;
        }
        if (fail) set_flag(&flags[FLAG_FAIL], 1);
    } else if (bid - nrt < nct) {
        // ---- U12 columns [C0, C0+64): forward substitution with the unit
        // lower L11.  Octet w8 owns column C0 + w8; lane g holds rows
        // 8(u + ku) + g of the current group ku.
        const int64_t C0 = c0 + L + (int64_t)(bid - nrt) * L;
#pragma unroll
        for (int k = 0; k < NPRE; ++k) {  // the prefetched column chunks
            const int e = t + k * NT, i0 = (e % (L / CH)) * CH, j = e / (L / CH);
            Chunk ch;
            ch.v = pre[k];
#pragma unroll
            for (int u = 0; u < CH; ++u) Sg[i0 + u][j] = (CT)to_f32(ch.e[u]);
        }
        __syncthreads();
        CT y[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) y[u] = Sg[8 * u + g][w8];
        for (int ku = 0; ku < 8; ++ku) {
            CT lv[8][8];
#pragma unroll
            for (int kq = 0; kq < 8; ++kq)
#pragma unroll
                for (int u = 0; u < 8; ++u) lv[kq][u] = Li[((ku * 8 + kq) * 8 + g) * 8 + u];
#pragma unroll
            for (int kq = 0; kq < 8; ++kq) {
                CT yk;
                switch (kq) {
                case 0: yk = oct_bcast<0>(y[0]); break;
                case 1: yk = oct_bcast<1>(y[0]); break;
                case 2: yk = oct_bcast<2>(y[0]); break;
                case 3: yk = oct_bcast<3>(y[0]); break;
                case 4: yk = oct_bcast<4>(y[0]); break;
                case 5: yk = oct_bcast<5>(y[0]); break;
                case 6: yk = oct_bcast<6>(y[0]); break;
                default: yk = oct_bcast<7>(y[0]); break;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) y[u] -= lv[kq][u] * yk;
            }
            Sg[8 * ku + g][w8] = y[0];
#pragma unroll
            for (int u = 0; u < 7; ++u) y[u] = y[u + 1];
            y[7] = 0;
        }
        __syncthreads();
        for (int e = t; e < L * L / CH; e += NT) {
            const int i0 = (e % (L / CH)) * CH, j = e / (L / CH);
            Chunk ch;
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                ch.e[u] = to_store_d<T>((double)Sg[i0 + u][j]);
                bad |= !isfinite(to_f32(ch.e[u]));  // the stored value
            }
            *(u32x4 *)(A + (c0 + i0) + (C0 + j) * lda) = ch.v;
        }
    }
    if (bad) set_flag(&flags[FLAG_NONFINITE], 1);
}

template <typename T>
__global__ __launch_bounds__(LEAF_THREADS) void k_leaf_spec(int64_t Np, int64_t c0, T *__restrict__ A,
                                                            int64_t lda, T *__restrict__ LT, int64_t k0,
                                                            int nrt, int nct, T *__restrict__ DG,
                                                            const T *__restrict__ DGprev, int64_t cprev,
                                                            int *__restrict__ flags)
{
    leaf_body<T>(blockIdx.x, Np, c0, A, lda, LT, NB_OUT, c0 - k0, nrt, nct, DG, DGprev, cprev, flags);
}

// copy a 64x64 diagonal block from DG into A (the last leaf's block)
template <typename T>
__global__ __launch_bounds__(256) void k_put_diag(int64_t c0, T *__restrict__ A, int64_t lda,
                                                  const T *__restrict__ DG, const int *flags)
{
    if (ld_flag(&flags[FLAG_FAIL])) return;
    for (int e = threadIdx.x; e < NB_LEAF * NB_LEAF; e += 256) {
        const int i = e % NB_LEAF, j = e / NB_LEAF;
        A[(c0 + i) + (c0 + j) * lda] = DG[i + j * NB_LEAF];
    }
}

// The FP16/BF16 Schur tile (gemm16_tile) and its XCD-aware tile order are in n3p_gemm.hpp.

template <typename T, int TM, int TN, int WGM, int WGN, int KC>
__global__ __launch_bounds__(WGM *WGN * 64) void k_gemm16(int M, int N, int K,
                                                          const T *__restrict__ At, int64_t ldat,
                                                          const T *__restrict__ B, int64_t ldb,
                                                          T *__restrict__ C, int64_t ldc,
                                                          int *__restrict__ flags, int check_abort)
{
    if (check_abort && block_flag(&flags[FLAG_FAIL])) return;
    const int ntm = M / TM, ntn = N / TN;
    int tm, tn;
    grouped_tile(xcd_tile(blockIdx.x, ntm * ntn), ntm, ntn, tm, tn);
    __shared__ __attribute__((aligned(16))) T lds[gemm16_lds_elems<TM, TN, KC>()];
    gemm16_tile<T, TM, TN, WGM, WGN, KC>(tm * TM, tn * TN, K, At, ldat, B, ldb, C, ldc, flags, lds);
}

// Two independent updates with the same K in one launch (tiles of the first,
// then of the second): after a leaf, the rest of its panel (below) and the
// row block right of the panel write disjoint parts of C and only read L and U.
struct GemmProb {
    int M, N;
    const void *At;
    int64_t ldat;
    const void *B;
    int64_t ldb;
    void *C;
    int64_t ldc;
};

template <typename T, int TM, int TN, int WGM, int WGN, int KC>
__global__ __launch_bounds__(WGM *WGN * 64) void k_gemm16_pair(GemmProb p1, GemmProb p2, int K,
                                                               int *__restrict__ flags)
{
    if (block_flag(&flags[FLAG_FAIL])) return;
    const int nt1 = (p1.M / TM) * (p1.N / TN), nt2 = (p2.M / TM) * (p2.N / TN);
    int tile = xcd_tile(blockIdx.x, nt1 + nt2);
    const GemmProb &p = tile < nt1 ? p1 : p2;
    if (tile >= nt1) tile -= nt1;
    int tm, tn;
    grouped_tile(tile, p.M / TM, p.N / TN, tm, tn);
    __shared__ __attribute__((aligned(16))) T lds[gemm16_lds_elems<TM, TN, KC>()];
    gemm16_tile<T, TM, TN, WGM, WGN, KC>(tm * TM, tn * TN, K, (const T *)p.At, p.ldat, (const T *)p.B,
                                         p.ldb, (T *)p.C, p.ldc, flags, lds);
}

// ========================================== Schur GEMM, FP32/FP64 matrix cores
template <typename T> struct mfma16x4;
// Output layout of the 16x16 fragment: lane l holds column l & 15; register q
// holds row 4 (l >> 4) + q for the FP32 instruction and row (l >> 4) + 4 q for
// the FP64 one (checked on gfx950 with an in-bounds probe).
template <> struct mfma16x4<float> {
    typedef f32x4 acc_t;
    static __device__ __forceinline__ int row(int lane, int q) { return 4 * (lane >> 4) + q; }
    static __device__ __forceinline__ acc_t op(float a, float b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <> struct mfma16x4<double> {
    typedef f64x4 acc_t;
    static __device__ __forceinline__ int row(int lane, int q) { return (lane >> 4) + 4 * q; }
    static __device__ __forceinline__ acc_t op(double a, double b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

// 64x64 block tile, 4 waves of 32x32 (2x2 fragments of 16x16), KC = 16.
template <typename T>
__global__ __launch_bounds__(256) void k_gemm_mfma4(int M, int N, int K, const T *__restrict__ At,
                                                    int64_t ldat, const T *__restrict__ B,
                                                    int64_t ldb, T *__restrict__ C, int64_t ldc,
                                                    int *__restrict__ flags, int check_abort)
{
    typedef typename mfma16x4<T>::acc_t acc_t;
    constexpr int TM = 64, TN = 64, KC = 16;
    __shared__ T As[KC][TM + 4];
    __shared__ T Bs[KC][TN + 4];
    if (check_abort && block_flag(&flags[FLAG_FAIL])) return;
    const int ntm = M / TM, ntn = N / TN, nt = ntm * ntn;
    int tile = blockIdx.x;
    if ((nt & 7) == 0) tile = (blockIdx.x & 7) * (nt >> 3) + (blockIdx.x >> 3);
    const int row0 = (tile % ntm) * TM, col0 = (tile / ntm) * TN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    acc_t acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[a][b][q] = 0;
    // loader: thread -> (row r = tid/4, k quad kq = (tid%4)*4)
    const int lrow = tid >> 2, lkq = (tid & 3) * 4;
    for (int kk = 0; kk < K; kk += KC) {
        T va[4], vb[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            va[q] = At[(int64_t)(row0 + lrow) * ldat + kk + lkq + q];
            vb[q] = B[(int64_t)(col0 + lrow) * ldb + kk + lkq + q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            As[lkq + q][lrow] = va[q];
            Bs[lkq + q][lrow] = vb[q];
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < KC; ks += 4) {
            const int kr = ks + (lane >> 4), ci = lane & 15;
#pragma unroll
            for (int fm = 0; fm < 2; ++fm) {
                const T a = As[kr][wm * 32 + fm * 16 + ci];
#pragma unroll
                for (int fn = 0; fn < 2; ++fn) {
                    const T b = Bs[kr][wn * 32 + fn * 16 + ci];
                    acc[fm][fn] = mfma16x4<T>::op(a, b, acc[fm][fn]);
                }
            }
        }
    }
    bool bad = false;
#pragma unroll
    for (int fm = 0; fm < 2; ++fm)
#pragma unroll
        for (int fn = 0; fn < 2; ++fn) {
            const int col = col0 + wn * 32 + fn * 16 + (lane & 15);
            const int rb0 = row0 + wm * 32 + fm * 16;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                T *p = C + (int64_t)col * ldc + rb0 + mfma16x4<T>::row(lane, q);
                const T v = *p - acc[fm][fn][q];
                bad |= !isfinite((double)v);
                *p = v;
            }
        }
    if (bad) set_flag(&flags[FLAG_NONFINITE], 1);
}

template <typename T>
__global__ __launch_bounds__(256) void k_check_finite(int64_t Np, const T *__restrict__ A,
                                                      int64_t lda, int *__restrict__ flags)
{
    const int64_t j = blockIdx.x;
    bool bad = false;
    for (int64_t i = threadIdx.x; i < Np; i += 256) bad |= !isfinite((double)to_f32(A[i + j * lda]));
    if (bad) set_flag(&flags[FLAG_NONFINITE], 1);
}

// ================================================================ launchers
template <typename T>
static hipError_t leaf_spec_t(int64_t Np, int64_t c0, void *A, int64_t lda, void *LT, int64_t k0,
                              void *DG, const void *DGprev, int64_t cprev, int *flags,
                              hipStream_t s)
{
    const int64_t below = Np - c0 - NB_LEAF;  // a multiple of NB_LEAF
    const int nrt = (int)(below / NB_LEAF);
    const int nct = nrt;
    const unsigned grid = (unsigned)std::max(1, nrt + nct);
    hipLaunchKernelGGL(k_leaf_spec<T>, dim3(grid), dim3(LEAF_THREADS), 0, s, Np, c0, (T *)A, lda,
                       (T *)LT, k0, nrt, nct, (T *)DG, (const T *)DGprev, cprev, flags);
    return hipGetLastError();
}

hipError_t launch_leaf_spec2(int prec, int64_t Np, int64_t c0, void *A, int64_t lda, void *LT,
                             int64_t k0, void *DG, const void *DGprev, int64_t cprev, int *flags,
                             hipStream_t s)
{
    switch (prec) {
    case N3P_FP16: return leaf_spec_t<f16>(Np, c0, A, lda, LT, k0, DG, DGprev, cprev, flags, s);
    case N3P_BF16: return leaf_spec_t<bf16>(Np, c0, A, lda, LT, k0, DG, DGprev, cprev, flags, s);
    case N3P_FP32: return leaf_spec_t<float>(Np, c0, A, lda, LT, k0, DG, DGprev, cprev, flags, s);
    case N3P_FP64: return leaf_spec_t<double>(Np, c0, A, lda, LT, k0, DG, DGprev, cprev, flags, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_put_diag(int prec, int64_t c0, void *A, int64_t lda, const void *DG,
                           const int *flags, hipStream_t s)
{
    switch (prec) {
    case N3P_FP16: hipLaunchKernelGGL(k_put_diag<f16>, dim3(1), dim3(256), 0, s, c0, (f16 *)A, lda, (const f16 *)DG, flags); break;
    case N3P_BF16: hipLaunchKernelGGL(k_put_diag<bf16>, dim3(1), dim3(256), 0, s, c0, (bf16 *)A, lda, (const bf16 *)DG, flags); break;
    case N3P_FP32: hipLaunchKernelGGL(k_put_diag<float>, dim3(1), dim3(256), 0, s, c0, (float *)A, lda, (const float *)DG, flags); break;
    case N3P_FP64: hipLaunchKernelGGL(k_put_diag<double>, dim3(1), dim3(256), 0, s, c0, (double *)A, lda, (const double *)DG, flags); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int TM, int TN, int WGM, int WGN, int KC>
static void gemm16_go(int64_t M, int64_t N, int64_t K, const void *At, int64_t ldat, const void *B,
                      int64_t ldb, void *C, int64_t ldc, int *flags, bool ca, hipStream_t s)
{
    const unsigned grid = (unsigned)((M / TM) * (N / TN));
    hipLaunchKernelGGL((k_gemm16<T, TM, TN, WGM, WGN, KC>), dim3(grid), dim3(WGM * WGN * 64), 0, s,
                       (int)M, (int)N, (int)K, (const T *)At, ldat, (const T *)B, ldb, (T *)C, ldc,
                       flags, (int)ca);
}

template <typename T>
static hipError_t gemm16_t(int64_t M, int64_t N, int64_t K, const void *At, int64_t ldat,
                           const void *B, int64_t ldb, void *C, int64_t ldc, int *flags, bool ca,
                           hipStream_t s)
{
    if (M % 64 || N % 64 || K % 32) return hipErrorInvalidValue;
    if (M % 256 == 0 && N % 256 == 0 && M * N >= (int64_t)256 * 256 * 128)
        gemm16_go<T, 256, 256, 2, 4, 32>(M, N, K, At, ldat, B, ldb, C, ldc, flags, ca, s);
    else if (M % 128 == 0 && N % 128 == 0 && M * N >= (int64_t)128 * 128 * 128)
        gemm16_go<T, 128, 128, 2, 2, 32>(M, N, K, At, ldat, B, ldb, C, ldc, flags, ca, s);
    else
        gemm16_go<T, 64, 64, 2, 2, 32>(M, N, K, At, ldat, B, ldb, C, ldc, flags, ca, s);
    return hipGetLastError();
}

template <typename T>
static hipError_t gemm4_t(int64_t M, int64_t N, int64_t K, const void *At, int64_t ldat,
                          const void *B, int64_t ldb, void *C, int64_t ldc, int *flags, bool ca,
                          hipStream_t s)
{
    if (M % 64 || N % 64 || K % 16) return hipErrorInvalidValue;
    const unsigned grid = (unsigned)((M / 64) * (N / 64));
    hipLaunchKernelGGL(k_gemm_mfma4<T>, dim3(grid), dim3(256), 0, s, (int)M, (int)N, (int)K,
                       (const T *)At, ldat, (const T *)B, ldb, (T *)C, ldc, flags, (int)ca);
    return hipGetLastError();
}

hipError_t launch_gemm_sub(int prec, int64_t M, int64_t N, int64_t K, const void *At, int64_t ldat,
                           const void *B, int64_t ldb, void *C, int64_t ldc, int *flags,
                           bool check_abort, hipStream_t s)
{
    if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
    switch (prec) {
    case N3P_FP16: return gemm16_t<f16>(M, N, K, At, ldat, B, ldb, C, ldc, flags, check_abort, s);
    case N3P_BF16: return gemm16_t<bf16>(M, N, K, At, ldat, B, ldb, C, ldc, flags, check_abort, s);
    case N3P_FP32: return gemm4_t<float>(M, N, K, At, ldat, B, ldb, C, ldc, flags, check_abort, s);
    case N3P_FP64: return gemm4_t<double>(M, N, K, At, ldat, B, ldb, C, ldc, flags, check_abort, s);
    }
    return hipErrorInvalidValue;
}

template <typename T>
static hipError_t gemm16_pair_t(GemmProb a, GemmProb b, int K, int *flags, hipStream_t s)
{
    auto fits = [](const GemmProb &q, int t) { return q.M % t == 0 && q.N % t == 0; };
    if (fits(a, 128) && fits(b, 128)) {
        const unsigned g = (unsigned)((a.M / 128) * (a.N / 128) + (b.M / 128) * (b.N / 128));
        hipLaunchKernelGGL((k_gemm16_pair<T, 128, 128, 2, 2, 32>), dim3(g), dim3(256), 0, s, a, b, K, flags);
    } else {
        const unsigned g = (unsigned)((a.M / 64) * (a.N / 64) + (b.M / 64) * (b.N / 64));
        hipLaunchKernelGGL((k_gemm16_pair<T, 64, 64, 2, 2, 32>), dim3(g), dim3(256), 0, s, a, b, K, flags);
    }
    return hipGetLastError();
}

// C1 -= At1^T B1 and C2 -= At2^T B2 (same K) in one launch; FP16/BF16 only,
// every M, N a multiple of 64 and K of 32.  An empty problem is allowed.
hipError_t launch_gemm_pair(int prec, int64_t M1, int64_t N1, const void *At1, int64_t ldat1,
                            const void *B1, int64_t ldb1, void *C1, int64_t ldc1, int64_t M2,
                            int64_t N2, const void *At2, int64_t ldat2, const void *B2,
                            int64_t ldb2, void *C2, int64_t ldc2, int64_t K, int *flags,
                            hipStream_t s)
{
    if (M1 % 64 || N1 % 64 || M2 % 64 || N2 % 64 || K % 32 || K <= 0) return hipErrorInvalidValue;
    GemmProb a{(int)M1, (int)N1, At1, ldat1, B1, ldb1, C1, ldc1};
    GemmProb b{(int)M2, (int)N2, At2, ldat2, B2, ldb2, C2, ldc2};
    if (M1 <= 0 || N1 <= 0) { a.M = 0; a.N = 64; }
    if (M2 <= 0 || N2 <= 0) { b.M = 0; b.N = 64; }
    if (a.M == 0 && b.M == 0) return hipSuccess;
    switch (prec) {
    case N3P_FP16: return gemm16_pair_t<f16>(a, b, (int)K, flags, s);
    case N3P_BF16: return gemm16_pair_t<bf16>(a, b, (int)K, flags, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_check_factor_finite(int prec, int64_t Np, const void *A, int64_t lda, int *flags,
                                      hipStream_t s)
{
    switch (prec) {
    case N3P_FP16: hipLaunchKernelGGL(k_check_finite<f16>, dim3((unsigned)Np), dim3(256), 0, s, Np, (const f16 *)A, lda, flags); break;
    case N3P_BF16: hipLaunchKernelGGL(k_check_finite<bf16>, dim3((unsigned)Np), dim3(256), 0, s, Np, (const bf16 *)A, lda, flags); break;
    case N3P_FP32: hipLaunchKernelGGL(k_check_finite<float>, dim3((unsigned)Np), dim3(256), 0, s, Np, (const float *)A, lda, flags); break;
    case N3P_FP64: hipLaunchKernelGGL(k_check_finite<double>, dim3((unsigned)Np), dim3(256), 0, s, Np, (const double *)A, lda, flags); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}


// ====================================================== batched engine kernels
// Leaf `leaf` (columns 64 leaf .. +64) of every slot that factors this step:
// the same leaf body as the single factorisation, with L21 kept transposed in
// the slot's LT (ld 64) for the rank-64 update that follows.  A slot's last
// leaf has no tiles and writes its diagonal block straight into A.
template <typename T>
__global__ __launch_bounds__(LEAF_THREADS) void k_b_leaf(const BDesc *__restrict__ d,
                                                         const BState *__restrict__ st, int nslots,
                                                         int leaf)
{
    __shared__ int off[B_MAX_SLOTS + 1];
    const int64_t c0 = (int64_t)leaf * NB_LEAF;
    const int total = b_offsets(nslots, off, [&](int s) {
        if (st[s].phase != BP_RUN || !st[s].factor || d[s].Np <= c0) return 0;
        const int nrt = (int)((d[s].Np - c0 - NB_LEAF) / NB_LEAF);
        return nrt > 0 ? 2 * nrt : 1;
    });
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int s = b_find(off, nslots, item);
        const BDesc &q = d[s];
        const int nrt = (int)((q.Np - c0 - NB_LEAF) / NB_LEAF);
        T *DGs = (T *)q.DG;
        T *DG = nrt > 0 ? DGs + (leaf % 2) * NB_LEAF * NB_LEAF : nullptr;
        const T *DGprev = leaf > 0 ? DGs + ((leaf - 1) % 2) * NB_LEAF * NB_LEAF : nullptr;
        leaf_body<T>(item - off[s], q.Np, c0, (T *)q.A, q.Np, (T *)q.LT, NB_LEAF, 0, nrt, nrt, DG,
                     DGprev, c0 - NB_LEAF, q.flags);
        __syncthreads();
    }
}

// Rank-64 Schur update after leaf `leaf`: A22 -= L21 U12 for every slot that
// factors this step, in TM x TM tiles (TM = 64: every trailing size is a
// multiple of 64).
template <typename T, int KC>
__global__ __launch_bounds__(256) void k_b_gemm(const BDesc *__restrict__ d,
                                                const BState *__restrict__ st, int nslots, int leaf)
{
    constexpr int TM = 64;
    __shared__ int off[B_MAX_SLOTS + 1];
    __shared__ __attribute__((aligned(16))) T lds[gemm16_lds_elems<TM, TM, KC>()];
    const int64_t c0 = (int64_t)leaf * NB_LEAF, c1 = c0 + NB_LEAF;
    const int total = b_offsets(nslots, off, [&](int s) {
        if (st[s].phase != BP_RUN || !st[s].factor || d[s].Np <= c1) return 0;
        const int m = (int)((d[s].Np - c1) / TM);
        return m * m;
    });
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int s = b_find(off, nslots, item);
        const BDesc &q = d[s];
        if (ld_flag(&q.flags[FLAG_FAIL])) continue;  // abandoned: needs interchanges
        const int m = (int)((q.Np - c1) / TM), local = item - off[s];
        const int tm = local % m, tn = local / m;
        T *A = (T *)q.A;
        const int64_t Np = q.Np;
        gemm16_tile<T, TM, TM, 2, 2, KC>(tm * TM, tn * TM, NB_LEAF, (const T *)q.LT + c1 * NB_LEAF,
                                         NB_LEAF, A + c0 + c1 * Np, Np, A + c1 + c1 * Np, Np,
                                         q.flags, lds);
        __syncthreads();
    }
}

hipError_t launch_b_leaf(int prec, const BDesc *d, const BState *st, int nslots, int leaf,
                         int grid, hipStream_t s)
{
    switch (prec) {
    case N3P_FP16: hipLaunchKernelGGL(k_b_leaf<f16>, dim3(grid), dim3(LEAF_THREADS), 0, s, d, st, nslots, leaf); break;
    case N3P_BF16: hipLaunchKernelGGL(k_b_leaf<bf16>, dim3(grid), dim3(LEAF_THREADS), 0, s, d, st, nslots, leaf); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_b_gemm(int prec, const BDesc *d, const BState *st, int nslots, int leaf,
                         int kc, int grid, hipStream_t s)
{
    if (prec == N3P_FP16) {
        if (kc == 64) hipLaunchKernelGGL((k_b_gemm<f16, 64>), dim3(grid), dim3(256), 0, s, d, st, nslots, leaf);
        else hipLaunchKernelGGL((k_b_gemm<f16, 32>), dim3(grid), dim3(256), 0, s, d, st, nslots, leaf);
    } else if (prec == N3P_BF16) {
        if (kc == 64) hipLaunchKernelGGL((k_b_gemm<bf16, 64>), dim3(grid), dim3(256), 0, s, d, st, nslots, leaf);
        else hipLaunchKernelGGL((k_b_gemm<bf16, 32>), dim3(grid), dim3(256), 0, s, d, st, nslots, leaf);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace n3p
