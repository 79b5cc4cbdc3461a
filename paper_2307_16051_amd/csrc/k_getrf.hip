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
// pivot searches and row interchanges (k_pivot_coop / k_row_gather).  Near-ties
// always take the explicit path, so rounding differences cannot change a
// pivot decision.
//
// The Schur-complement GEMMs use the matrix cores: FP16/BF16 inputs with FP32
// accumulation (v_mfma_f32_32x32x16_{f16,bf16}), rounded to the storage type
// once per GEMM; FP32 and FP64 use v_mfma_{f32,f64}_16x16x4.
#include <algorithm>

#include "n3p_internal.hpp"

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
    constexpr int LP = L + 4;
    constexpr int NT = LEAF_THREADS;
    __shared__ __attribute__((aligned(16))) CT Dm[L][LP];       // diagonal block
    // Ui[k][g][c] = U[k][8c+g], Li[k][g][u] = L[8u+g][k] where that index
    // exceeds k, else 0; flat with 8 trailing entries so reads for register
    // slots past index 63 stay in the array (those slots are dead).
    __shared__ __attribute__((aligned(16))) CT Ui[L * L + 8];
    __shared__ __attribute__((aligned(16))) CT Li[L * L + 8];
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
                    const CT piv = lane_bcast(x[kk], k);
                    if (!(fabs(piv) > (CT)0)) fail = true;
                    const CT rp = recip(piv);
                    CT l = 0;
                    if (r > k) {
                        if (!(fabs(x[kk]) <= margin * fabs(piv))) fail = true;
                        l = x[kk] * rp;
                        x[kk] = l;
                    }
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
    for (int e = t; e < L * L + 8; e += NT) {
        const int k = e / L, m = e % L;
        const int g = m / 8, c = m % 8, j = 8 * c + g;
        const bool in = e < L * L && j > k;
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
                for (int c = 0; c < 8; ++c) u[kq][c] = Ui[(8 * kc + kq) * L + g * 8 + kc + c];
            // this lane owns column 8kc + g: its pivot bound and reciprocal
            const CT lim = margin * fabs(Dm[8 * kc + g][8 * kc + g]);
            const CT rd = rdiag[8 * kc + g];
#pragma unroll
            for (int kq = 0; kq < 8; ++kq) {
                if (g == kq) {
                    if (!(fabs(x[0]) <= lim)) fail = true;
                    x[0] *= rd;
                }
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
                for (int u = 0; u < 8; ++u) lv[kq][u] = Li[(8 * ku + kq) * L + g * 8 + ku + u];
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

// ============================================= Schur GEMM, FP16/BF16 matrix cores
// C[M x N] -= At^T B, where At holds A row-major (row i at At + i*ldat, K
// contiguous) and B is column-major (column j at B + j*ldb, K contiguous).
// Block tile TM x TN, WGM x WGN waves, K staged through LDS in KC chunks,
// double-buffered.  Each wave owns (TM/WGM) x (TN/WGN) as 32x32 fragments.
template <typename T> struct mfma32;
template <> struct mfma32<f16> {
    typedef h8 vec;
    static __device__ __forceinline__ f32x16 op(vec a, vec b, f32x16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};
template <> struct mfma32<bf16> {
    typedef b8 vec;
    static __device__ __forceinline__ f32x16 op(vec a, vec b, f32x16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};

template <typename T, int TM, int TN, int WGM, int WGN, int KC>
__device__ __forceinline__ void gemm16_tile(int row0, int col0, int K, const T *__restrict__ At,
                                            int64_t ldat, const T *__restrict__ B, int64_t ldb,
                                            T *__restrict__ C, int64_t ldc, int *__restrict__ flags)
{
    typedef typename mfma32<T>::vec vec;
    constexpr int NT = WGM * WGN * 64;
    constexpr int WM = TM / WGM, WN = TN / WGN, FM = WM / 32, FN = WN / 32;
    constexpr int KP = KC + 8;          // padded LDS row (elements): 16-byte skew
    constexpr int CPR = KC / 8;         // 16-byte chunks per row
    constexpr int ACH = TM * CPR / NT;  // A chunks per thread per stage
    constexpr int BCH = TN * CPR / NT;
    static_assert(ACH * NT == TM * CPR && BCH * NT == TN * CPR, "tile/thread mismatch");
    __shared__ __attribute__((aligned(16))) T As[2][TM * KP];
    __shared__ __attribute__((aligned(16))) T Bs[2][TN * KP];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WGM, wn = wave / WGM;

    f32x16 acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[a][b][q] = 0.0f;

    // staging registers as native vectors (a union-based vector type would be
    // kept in scratch or LDS by the compiler)
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    u32x4 ra[ACH], rb[BCH];
#define N3P_GLOAD(kk_)                                                                        \
    do {                                                                                      \
        _Pragma("unroll") for (int c = 0; c < ACH; ++c) {                                     \
            const int ch = tid + c * NT, r = ch / CPR, seg = ch % CPR;                        \
            ra[c] = *(const u32x4 *)(At + (int64_t)(row0 + r) * ldat + (kk_) + seg * 8);      \
        }                                                                                     \
        _Pragma("unroll") for (int c = 0; c < BCH; ++c) {                                     \
            const int ch = tid + c * NT, r = ch / CPR, seg = ch % CPR;                        \
            rb[c] = *(const u32x4 *)(B + (int64_t)(col0 + r) * ldb + (kk_) + seg * 8);        \
        }                                                                                     \
    } while (0)
#define N3P_SSTORE(buf_)                                                                      \
    do {                                                                                      \
        _Pragma("unroll") for (int c = 0; c < ACH; ++c) {                                     \
            const int ch = tid + c * NT, r = ch / CPR, seg = ch % CPR;                        \
            *(u32x4 *)(&As[(buf_)][r * KP + seg * 8]) = ra[c];                                \
        }                                                                                     \
        _Pragma("unroll") for (int c = 0; c < BCH; ++c) {                                     \
            const int ch = tid + c * NT, r = ch / CPR, seg = ch % CPR;                        \
            *(u32x4 *)(&Bs[(buf_)][r * KP + seg * 8]) = rb[c];                                \
        }                                                                                     \
    } while (0)

    N3P_GLOAD(0);
    N3P_SSTORE(0);
    __syncthreads();
    int buf = 0;
    const int lr = lane & 31, lk = (lane >> 5) * 8;
    for (int kk = 0; kk < K; kk += KC) {
        const bool more = kk + KC < K;
        if (more) N3P_GLOAD(kk + KC);
#pragma unroll
        for (int ks = 0; ks < KC; ks += 16) {
            vec a[FM], b[FN];
#pragma unroll
            for (int fm = 0; fm < FM; ++fm)
                a[fm] = *(const vec *)(&As[buf][(wm * WM + fm * 32 + lr) * KP + ks + lk]);
#pragma unroll
            for (int fn = 0; fn < FN; ++fn)
                b[fn] = *(const vec *)(&Bs[buf][(wn * WN + fn * 32 + lr) * KP + ks + lk]);
#pragma unroll
            for (int fm = 0; fm < FM; ++fm)
#pragma unroll
                for (int fn = 0; fn < FN; ++fn) acc[fm][fn] = mfma32<T>::op(a[fm], b[fn], acc[fm][fn]);
        }
        if (more) N3P_SSTORE(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
#undef N3P_GLOAD
#undef N3P_SSTORE

    // epilogue: lane holds column (lane & 31) and rows 8g + 4(lane >> 5) + q
    typedef T t4 __attribute__((ext_vector_type(4)));
    bool bad = false;
#pragma unroll
    for (int fm = 0; fm < FM; ++fm)
#pragma unroll
        for (int fn = 0; fn < FN; ++fn) {
            const int col = col0 + wn * WN + fn * 32 + lr;
            const int rb0 = row0 + wm * WM + fm * 32 + (lane >> 5) * 4;
            T *cp = C + (int64_t)col * ldc;
#pragma unroll
            for (int gq = 0; gq < 4; ++gq) {
                t4 *p = (t4 *)(cp + rb0 + gq * 8);
                t4 cv = *p;
                t4 o;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float v = (float)cv[q] - acc[fm][fn][gq * 4 + q];
                    o[q] = (T)v;
                    bad |= !isfinite((float)o[q]);
                }
                *p = o;
            }
        }
    if (bad) set_flag(&flags[FLAG_NONFINITE], 1);
}

template <typename T, int TM, int TN, int WGM, int WGN, int KC>
__global__ __launch_bounds__(WGM *WGN * 64) void k_gemm16(int M, int N, int K,
                                                          const T *__restrict__ At, int64_t ldat,
                                                          const T *__restrict__ B, int64_t ldb,
                                                          T *__restrict__ C, int64_t ldc,
                                                          int *__restrict__ flags, int check_abort)
{
    if (check_abort && block_flag(&flags[FLAG_FAIL])) return;
    const int ntm = M / TM, ntn = N / TN, nt = ntm * ntn;
    const int bid = blockIdx.x;
    // XCD-aware order: workgroups are dispatched round-robin over the 8 XCDs;
    // give each XCD a contiguous run of tiles, and order that run in groups
    // of GM row tiles so the tiles an XCD's CUs hold at once share a few A
    // row blocks and B column blocks in its L2.
    // workgroup bid runs on XCD bid % 8; XCD x owns tiles [start_x, start_x + count_x)
    const int xcd = bid & 7, q8 = nt >> 3, r8 = nt & 7;
    const int tile = xcd * q8 + (xcd < r8 ? xcd : r8) + (bid >> 3);
    constexpr int GM = 8;
    const int per_group = GM * ntn, group = tile / per_group, first_m = group * GM;
    const int gsize = ntm - first_m < GM ? ntm - first_m : GM;
    const int in_group = tile - group * per_group;
    const int tm = first_m + in_group % gsize, tn = in_group / gsize;
    gemm16_tile<T, TM, TN, WGM, WGN, KC>(tm * TM, tn * TN, K, At, ldat, B, ldb, C, ldc, flags);
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
    const int nt1 = (p1.M / TM) * (p1.N / TN);
    int tile = blockIdx.x;
    const GemmProb &p = tile < nt1 ? p1 : p2;
    if (tile >= nt1) tile -= nt1;
    const int ntm = p.M / TM;
    const int tm = tile % ntm, tn = tile / ntm;
    gemm16_tile<T, TM, TN, WGM, WGN, KC>(tm * TM, tn * TN, K, (const T *)p.At, p.ldat, (const T *)p.B,
                                         p.ldb, (T *)p.C, p.ldc, flags);
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

// ============================================ pivoting path (explicit search)
// Partial pivoting (largest magnitude, ties to the lowest row) of one 64-column
// leaf over rows [c0, Np), spread over P workgroups that each hold a
// contiguous block of rows in registers (FP32 arithmetic, FP64 for FP64
// storage).  Per column every workgroup reduces its own candidate and
// publishes it -- row index, magnitude and the whole 64-value row -- as
// tag-stamped 64-bit words (tag = global column + 1), written and polled with
// agent-scope atomic accesses, so no cache-wide fence is needed.  Every
// wavefront then reads all P candidates and takes the same decision from the
// same words: no grid-wide barrier, one round trip for the candidates and one
// for the winning row per column.  Slots alternate with the column parity; a
// workgroup publishes column k + 2 only after every workgroup has published
// column k + 1, which each does only after it has finished reading column k.
//
// P <= 128 workgroups (512 threads, 256 for FP64) fill one CU each on an
// otherwise idle device, so all are resident together.  Every wait is bounded regardless: an
// expired wait raises FLAG_TIMEOUT and the wavefront stops waiting, so the grid
// always drains (the factors are then invalid and the caller reports the
// timeout).
//
// Columns are processed in 8 groups of 8.  The register row is rotated by 8
// slots after each group, so the current group's columns always sit in slots
// 0..7 (compile-time register indices): in group g, slot s holds panel column
// (s + 8 g) mod 64 and slots >= 64 - 8 g hold finished columns.
constexpr int PC_SPIN_LIMIT = 1 << 20;  // polls of ~1 us: a wait that long has failed

template <typename CT> struct pc_cfg;
// rows per thread, words per value, threads per workgroup (FP64 rows need the
// whole register file: one wavefront per SIMD)
template <> struct pc_cfg<float> { static constexpr int R = 1, W = 1, TH = 512; };
template <> struct pc_cfg<double> { static constexpr int R = 1, W = 2, TH = 256; };

__device__ __forceinline__ void put_word(uint64_t *w, uint32_t tag, uint32_t payload)
{
    __hip_atomic_store(w, ((uint64_t)tag << 32) | payload, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void put_val(uint64_t *w, uint32_t tag, float v)
{
    put_word(w, tag, __float_as_uint(v));
}
__device__ __forceinline__ void put_val(uint64_t *w, uint32_t tag, double v)
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    put_word(w, tag, (uint32_t)b);
    put_word(w + 1, tag, (uint32_t)(b >> 32));
}
template <typename CT> __device__ __forceinline__ CT val_of(const uint64_t *w);
template <> __device__ __forceinline__ float val_of<float>(const uint64_t *w)
{
    return __uint_as_float((uint32_t)w[0]);
}
template <> __device__ __forceinline__ double val_of<double>(const uint64_t *w)
{
    return __longlong_as_double((long long)(((uint64_t)(uint32_t)w[1] << 32) | (uint32_t)w[0]));
}

// Poll NW consecutive words per lane (lanes with `have`) until every word of
// the wavefront carries `tag`; bounded.
template <int NW>
__device__ __forceinline__ void poll_words(const uint64_t *p, bool have, uint32_t tag,
                                           uint64_t (&w)[NW], bool &dead, int *flags)
{
    int spins = 0;
    for (;;) {
        bool ok = true;
        if (have) {
#pragma unroll
            for (int h = 0; h < NW; ++h) {
                w[h] = __hip_atomic_load(p + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok &= (uint32_t)(w[h] >> 32) == tag;
            }
        }
        if (__all(ok) || dead) return;
        __builtin_amdgcn_s_sleep(1);
        if (++spins > PC_SPIN_LIMIT) {
            set_flag(&flags[FLAG_TIMEOUT], 1);
            dead = true;
            return;
        }
    }
}

template <typename CT>
__device__ __forceinline__ bool better(CT a, int ia, CT b, int ib)
{
    return a > b || (a == b && ia < ib);
}

// 16-byte vectors of the storage types (row stores into LT)
template <typename T> struct vec16;
template <> struct vec16<f16> { typedef h8 type; };
template <> struct vec16<bf16> { typedef b8 type; };
template <> struct vec16<float> { typedef f32x4 type; };
template <> struct vec16<double> { typedef double type __attribute__((ext_vector_type(2))); };

// Exchange area (64-bit words, zeroed once per factorisation):
//   cand [2][pmax][4]  : row index, magnitude (1 or 2 words)
//   rows [2][pmax][64W]: the candidate rows, in register-slot order (every
//                        workgroup is in the same column group when it reads)
//   rowk [2][64W]      : row k before the interchange, slot order
//   then int list[1 + 2*128]: count, (dest, src) row pairs of the leaf's
//   interchanges composed into one permutation.
// State of one thread of the panel kernel; step<KK>(g) is column 8 g + KK.
template <typename T, typename CT>
struct PcState {
    static constexpr int R = pc_cfg<CT>::R, W = pc_cfg<CT>::W, TH = pc_cfg<CT>::TH, L = NB_LEAF;
    static constexpr int NWV = TH / 64;
    static constexpr int RW = TH * R;  // rows per workgroup
    static constexpr int NONE = 0x7fffffff;
    CT v[R][L];
    int rowi[R];
    bool dead, nonfin;
    int tid, lane, wv, P, wg, m, pmax;
    int64_t c0;
    uint64_t *cand, *rows, *rowk;
    int *flags;
    CT (*red_v)[NWV];
    int (*red_i)[NWV];
    CT (*crow)[NWV][L];  // [parity][wavefront]: the wavefront's candidate row
    CT (*krow_l)[L];     // [parity]: row k (workgroup 0)
    int *pivs;

    template <int KK> __device__ __forceinline__ void step(int g)
    {
        const int k = 8 * g + KK, lim = L - 8 * g;
        const int par = k & 1;
        const uint32_t tag = (uint32_t)(c0 + k + 1);
        // --- this workgroup's candidate
        CT best = (CT)-1;
        int bi = NONE;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (rowi[r] >= k && rowi[r] < m) {
                CT a = fabs(v[r][KK]);
                if (a != a) { nonfin = true; a = (CT)0; }
                if (better(a, rowi[r], best, bi)) { best = a; bi = rowi[r]; }
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const CT ob = __shfl_xor(best, off);
            const int oi = __shfl_xor(bi, off);
            if (better(ob, oi, best, bi)) { best = ob; bi = oi; }
        }
        // the wavefront's candidate row (and row k) staged in LDS by its owner,
        // so that one wavefront publishes it with a single 64-lane store
        if (bi != NONE && tid == (bi - wg * RW) % TH) {
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (r == (bi - wg * RW) / TH)
#pragma unroll
                    for (int s = 0; s < L; ++s) crow[par][wv][s] = v[r][s];
        }
        if (wg == 0 && tid == k) {
#pragma unroll
            for (int s = 0; s < L; ++s) krow_l[par][s] = v[0][s];
        }
        if (lane == 0) { red_v[par][wv] = best; red_i[par][wv] = bi; }
        __syncthreads();
        best = red_v[par][0];
        bi = red_i[par][0];
        int bwv = 0;
#pragma unroll
        for (int w = 1; w < NWV; ++w)
            if (better(red_v[par][w], red_i[par][w], best, bi)) { best = red_v[par][w]; bi = red_i[par][w]; bwv = w; }
        // --- publish: the candidate first, then its row; (workgroup 0) row k
        if (wv == 0 && bi != NONE) {
            if (lane == 0) {
                uint64_t *cw = cand + ((size_t)par * pmax + wg) * 4;
                put_word(cw, tag, (uint32_t)bi);
                put_val(cw + 1, tag, best);
            }
            put_val(rows + ((size_t)par * pmax + wg) * L * W + lane * W, tag, crow[par][bwv][lane]);
        }
        if (wg == 0 && wv == NWV - 1) put_val(rowk + (size_t)par * L * W + lane * W, tag, krow_l[par][lane]);
        // --- every wavefront: the pivot row p from all P (<= 128) candidates
        int p = k;
        {
            CT cv = (CT)-1;
            int ci = NONE;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int q = lane + 64 * h;
                if (h == 1 && P <= 64) break;
                uint64_t cw[W + 1];
                const bool have = q < P;
                poll_words<W + 1>(cand + ((size_t)par * pmax + (have ? q : 0)) * 4, have, tag, cw, dead, flags);
                if (have) {
                    const int qi = (int)(uint32_t)cw[0];
                    const CT qv = val_of<CT>(cw + 1);
                    if (better(qv, qi, cv, ci)) { cv = qv; ci = qi; }
                }
            }
            for (int off = 32; off > 0; off >>= 1) {
                const CT ob = __shfl_xor(cv, off);
                const int oi = __shfl_xor(ci, off);
                if (better(ob, oi, cv, ci)) { cv = ob; ci = oi; }
            }
            if (!dead && ci >= k && ci < m) p = ci;
        }
        const int pw = p / RW;  // workgroup holding row p
        CT prow, krow = (CT)0;  // lane s: slot s of the pivot row / of row k
        {
            uint64_t w[W];
            poll_words<W>(rows + ((size_t)par * pmax + pw) * L * W + lane * W, true, tag, w, dead, flags);
            prow = val_of<CT>(w);
        }
        const int pin = p - pw * RW;
        const bool holds_p = p != k && pw == wg && (pin % TH) / 64 == wv;
        if (holds_p) {
            uint64_t w[W];
            poll_words<W>(rowk + (size_t)par * L * W + lane * W, true, tag, w, dead, flags);
            krow = val_of<CT>(w);
        }
        if (wg == 0 && tid == 0) pivs[k] = p;
        // --- interchange rows k and p (only the wavefronts holding them)
        if ((wg == 0 && wv == 0) || holds_p) {
            bool isk[R], isp[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                isk[r] = rowi[r] == k;
                isp[r] = holds_p && rowi[r] == p;
            }
#pragma unroll
            for (int s = 0; s < L; ++s) {
                const CT ps = lane_bcast(prow, s);
                const CT ks = holds_p ? lane_bcast(krow, s) : (CT)0;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (isk[r]) v[r][s] = ps;
                    if (isp[r]) v[r][s] = ks;
                }
            }
        }
        // --- multipliers and the rank-1 update of the unfinished columns
        const CT pk = lane_bcast(prow, KK);
        if (pk == (CT)0 && wg == 0 && tid == 0) atomicCAS(&flags[FLAG_ZEROPIV], 0, (int)(c0 + k + 1));
        bool upd[R];
        CT l[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            upd[r] = pk != (CT)0 && rowi[r] > k && rowi[r] < m;
            l[r] = upd[r] ? v[r][KK] / pk : (CT)0;
            if (upd[r]) v[r][KK] = l[r];
        }
#pragma unroll
        for (int s = KK + 1; s < L; ++s) {
            if (s < lim) {
                const CT ps = lane_bcast(prow, s);
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (upd[r]) v[r][s] -= l[r] * ps;
            }
        }
    }

    // rotate by 8 slots: the next group's columns move to slots 0..7
    __device__ __forceinline__ void rotate()
    {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            CT t8[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) t8[q] = v[r][q];
#pragma unroll
            for (int s = 0; s < L - 8; ++s) v[r][s] = v[r][s + 8];
#pragma unroll
            for (int q = 0; q < 8; ++q) v[r][L - 8 + q] = t8[q];
        }
    }
};

template <typename T, typename CT>
__global__ __launch_bounds__(pc_cfg<CT>::TH) void k_pivot_coop(int64_t Np, int64_t c0, int64_t k0,
                                                           T *__restrict__ A, int64_t lda,
                                                           int32_t *__restrict__ ipiv,
                                                           T *__restrict__ LT,
                                                           uint64_t *__restrict__ xch, int pmax,
                                                           int *__restrict__ flags)
{
    typedef PcState<T, CT> S;
    constexpr int R = S::R, W = S::W, L = NB_LEAF, RW = S::RW;
    __shared__ CT red_v[2][S::NWV];
    __shared__ int red_i[2][S::NWV];
    __shared__ CT crow[2][S::NWV][L];
    __shared__ CT krow_l[2][L];
    __shared__ int pivs[L];
    if (block_flag(&flags[FLAG_TIMEOUT])) return;
    S st;
    st.tid = threadIdx.x;
    st.lane = st.tid & 63;
    st.wv = st.tid >> 6;
    st.P = (int)gridDim.x;
    st.wg = (int)blockIdx.x;
    st.m = (int)(Np - c0);
    st.pmax = pmax;
    st.c0 = c0;
    st.cand = xch;
    st.rows = xch + (size_t)8 * pmax;
    st.rowk = st.rows + (size_t)2 * pmax * L * W;
    st.flags = flags;
    st.red_v = red_v;
    st.red_i = red_i;
    st.crow = crow;
    st.krow_l = krow_l;
    st.pivs = pivs;
    st.dead = false;
    st.nonfin = false;
    int *list = (int *)(st.rowk + 2 * L * W);
    const int tid = st.tid, lane = st.lane, wv = st.wv, wg = st.wg, m = st.m;

#pragma unroll
    for (int r = 0; r < R; ++r) {
        st.rowi[r] = wg * RW + r * S::TH + tid;
#pragma unroll
        for (int j = 0; j < L; ++j) st.v[r][j] = (CT)0;
        if (st.rowi[r] < m) {
            const T *src = A + (c0 + st.rowi[r]) + c0 * lda;
#pragma unroll
            for (int j = 0; j < L; ++j) st.v[r][j] = (CT)to_f32(src[j * lda]);
        }
    }

    for (int g = 0; g < L / 8; ++g) {
        st.template step<0>(g);
        st.template step<1>(g);
        st.template step<2>(g);
        st.template step<3>(g);
        st.template step<4>(g);
        st.template step<5>(g);
        st.template step<6>(g);
        st.template step<7>(g);
        st.rotate();
    }
    if (st.nonfin) set_flag(&flags[FLAG_NONFINITE], 1);

    // --- the factored panel into A; rows below the leaf also into LT (K contiguous)
    typedef typename vec16<T>::type V16;
    constexpr int VE = 16 / sizeof(T);
    bool bad = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (st.rowi[r] >= m) continue;
        T *dst = A + (c0 + st.rowi[r]) + c0 * lda;
        T *lt = LT + (c0 + st.rowi[r]) * (int64_t)NB_OUT + (c0 - k0);
        const bool below = st.rowi[r] >= L;
#pragma unroll
        for (int q = 0; q < L / VE; ++q) {
            V16 pk16;
#pragma unroll
            for (int e = 0; e < VE; ++e) {
                const T x = to_store_d<T>((double)st.v[r][q * VE + e]);
                bad |= !isfinite(to_f32(x));  // the stored value (FP16 overflows above 65504)
                dst[(q * VE + e) * lda] = x;
                pk16[e] = x;
            }
            if (below) *(V16 *)(lt + q * VE) = pk16;
        }
    }
    if (bad) set_flag(&flags[FLAG_NONFINITE], 1);

    // --- workgroup 0: ipiv, and the 64 interchanges composed into one list of
    // (dest, src) row moves: entry e < 64 is panel row e (lane e, val_lo); rows
    // >= 64 that take part get entries 64 + i (lane i, key_hi/val_hi).
    __syncthreads();
    if (wg == 0 && wv == 0) {
        int val_lo = lane, key_hi = -1, val_hi = -1, nh = 0;
        for (int t = 0; t < L; ++t) {
            const int p = pivs[t];
            if (p == t) continue;
            int e = p;
            if (p >= L) {
                const unsigned long long b = __ballot(key_hi == p);
                if (b) {
                    e = L + (int)__builtin_ctzll(b);
                } else {
                    e = L + nh;
                    if (lane == nh) { key_hi = p; val_hi = p; }
                    ++nh;
                }
            }
            const int vt = __builtin_amdgcn_readlane(val_lo, t);
            const int ve = e < L ? __builtin_amdgcn_readlane(val_lo, e) : __builtin_amdgcn_readlane(val_hi, e - L);
            if (lane == t) val_lo = ve;
            if (e < L) {
                if (lane == e) val_lo = vt;
            } else if (lane == e - L) {
                val_hi = vt;
            }
        }
        const bool m0 = val_lo != lane, m1 = lane < nh && val_hi != key_hi;
        const unsigned long long b0 = __ballot(m0), b1 = __ballot(m1);
        const int n0 = __popcll(b0);
        if (m0) {
            const int i = __builtin_amdgcn_mbcnt_hi((unsigned)(b0 >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)b0, 0));
            list[1 + 2 * i] = (int)c0 + lane;
            list[2 + 2 * i] = (int)c0 + val_lo;
        }
        if (m1) {
            const int i = n0 + __builtin_amdgcn_mbcnt_hi((unsigned)(b1 >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)b1, 0));
            list[1 + 2 * i] = (int)c0 + key_hi;
            list[2 + 2 * i] = (int)c0 + val_hi;
        }
        if (lane == 0) list[0] = n0 + __popcll(b1);
        ipiv[c0 + lane] = (int32_t)(c0 + pivs[lane]);
    }
}

// A leaf's interchanges on every column outside the leaf: new[dest] = old[src]
// for the listed (dest, src) pairs (at most 128).  Two columns per 256-thread
// workgroup, one pair per thread; every read completes before any write.
template <typename T>
__global__ __launch_bounds__(256) void k_row_gather(T *__restrict__ A, int64_t lda,
                                                    const int *__restrict__ list, int64_t c0,
                                                    int64_t ncol)
{
    const int64_t q = (int64_t)blockIdx.x * 2 + (threadIdx.x >> 7);
    const int e = threadIdx.x & 127;
    const int n = list[0];
    const bool act = q < ncol && e < n;
    const int64_t col = q < c0 ? q : q + NB_LEAF;
    T *cp = A + col * lda;
    T x = (T)0.0f;
    if (act) x = cp[list[2 + 2 * e]];
    __syncthreads();
    if (act) cp[list[1 + 2 * e]] = x;
}

// LT rows [r0, Np) for the outer block starting at column k0: the block's L
// columns transposed (K contiguous), read from A after all of the block's
// interchanges.  64 x 64 tiles through LDS; grid (rows / 64, columns / 64).
template <typename T>
__global__ __launch_bounds__(256) void k_lt_rebuild(const T *__restrict__ A, int64_t lda,
                                                    T *__restrict__ LT, int64_t r0, int64_t k0)
{
    __shared__ T tile[64][65];
    const int64_t rb = r0 + (int64_t)blockIdx.x * 64;
    const int jb = blockIdx.y * 64;
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int e = t + 256 * q, i = e & 63, j = e >> 6;
        tile[j][i] = A[(rb + i) + (k0 + jb + j) * lda];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int e = t + 256 * q, j = e & 63, i = e >> 6;
        LT[(rb + i) * (int64_t)NB_OUT + jb + j] = tile[j][i];
    }
}

// U row block of a factored leaf: rows [c0, c0+64) x columns [col0, col1),
// forward substitution with the unit lower L11 taken from A.
template <typename T>
__global__ __launch_bounds__(256) void k_u12(int64_t col0, int64_t col1, int64_t c0,
                                             T *__restrict__ A, int64_t lda,
                                             int *__restrict__ flags)
{
    typedef typename compute_of<T>::type CT;
    constexpr int L = NB_LEAF;
    __shared__ CT Dm[L][L + 1];
    const int t = threadIdx.x;
    for (int e = t; e < L * L; e += 256) {
        const int i = e % L, j = e / L;
        Dm[i][j] = (CT)to_f32(A[(c0 + i) + (c0 + j) * lda]);
    }
    __syncthreads();
    const int64_t jc = col0 + (int64_t)blockIdx.x * 256 + t;
    if (jc >= col1) return;
    T *col = A + jc * lda + c0;
    CT y[L];
#pragma unroll
    for (int k = 0; k < L; ++k) y[k] = (CT)to_f32(col[k]);
#pragma unroll
    for (int k = 1; k < L; ++k) {
        CT s = y[k];
#pragma unroll
        for (int m = 0; m < k; ++m) s -= Dm[k][m] * y[m];
        y[k] = s;
    }
    bool bad = false;
#pragma unroll
    for (int k = 0; k < L; ++k) {
        const T v = to_store_d<T>((double)y[k]);
        if (!isfinite(to_f32(v))) bad = true;
        col[k] = v;
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

static int pc_rows_per_wg(int prec) { return prec == N3P_FP64 ? pc_cfg<double>::TH : pc_cfg<float>::TH; }

static int64_t pc_pmax(int prec, int64_t Np)
{
    return (Np + pc_rows_per_wg(prec) - 1) / pc_rows_per_wg(prec);
}

size_t pivot_xch_bytes(int prec, int64_t Np)
{
    const int64_t pmax = pc_pmax(prec, Np), W = prec == N3P_FP64 ? 2 : 1;
    const int64_t words = 8 * pmax + 2 * pmax * NB_LEAF * W + 2 * NB_LEAF * W;
    return (size_t)words * 8 + (size_t)(1 + 4 * NB_LEAF) * 4;
}

hipError_t launch_pivot_reset(int prec, int64_t Np, void *xch, hipStream_t s)
{
    return launch_fill_i32((int *)xch, 0, (int64_t)(pivot_xch_bytes(prec, Np) / 4), s);
}

template <typename T, typename CT>
static hipError_t pivot_coop_t(int64_t Np, int64_t c0, int64_t k0, void *A, int64_t lda,
                               int32_t *ipiv, void *LT, void *xch, int pmax, int P, int *flags,
                               hipStream_t s)
{
    hipLaunchKernelGGL((k_pivot_coop<T, CT>), dim3(P), dim3(pc_cfg<CT>::TH), 0, s, Np, c0, k0, (T *)A,
                       lda, ipiv, (T *)LT, (uint64_t *)xch, pmax, flags);
    return hipGetLastError();
}

hipError_t launch_pivot_coop(int prec, int64_t Np, int64_t c0, int64_t k0, void *A, int64_t lda,
                             int32_t *ipiv, void *LT, void *xch, int *flags, hipStream_t s)
{
    const int64_t rw = pc_rows_per_wg(prec), m = Np - c0;
    const int64_t P = (m + rw - 1) / rw, pmax = pc_pmax(prec, Np);
    if (m < NB_LEAF || m % NB_LEAF || P > 128) return hipErrorInvalidValue;
    switch (prec) {
    case N3P_FP16: return pivot_coop_t<f16, float>(Np, c0, k0, A, lda, ipiv, LT, xch, (int)pmax, (int)P, flags, s);
    case N3P_BF16: return pivot_coop_t<bf16, float>(Np, c0, k0, A, lda, ipiv, LT, xch, (int)pmax, (int)P, flags, s);
    case N3P_FP32: return pivot_coop_t<float, float>(Np, c0, k0, A, lda, ipiv, LT, xch, (int)pmax, (int)P, flags, s);
    case N3P_FP64: return pivot_coop_t<double, double>(Np, c0, k0, A, lda, ipiv, LT, xch, (int)pmax, (int)P, flags, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_row_gather(int prec, int64_t Np, int64_t c0, void *A, int64_t lda,
                             const void *xch, hipStream_t s)
{
    const int64_t pmax = pc_pmax(prec, Np), W = prec == N3P_FP64 ? 2 : 1;
    const int *list = (const int *)((const uint64_t *)xch + 8 * pmax + 2 * pmax * NB_LEAF * W +
                                    2 * NB_LEAF * W);
    const int64_t ncol = Np - NB_LEAF;
    if (ncol <= 0) return hipSuccess;
    const unsigned grid = (unsigned)((ncol + 1) / 2);
    switch (prec) {
    case N3P_FP16: hipLaunchKernelGGL(k_row_gather<f16>, dim3(grid), dim3(256), 0, s, (f16 *)A, lda, list, c0, ncol); break;
    case N3P_BF16: hipLaunchKernelGGL(k_row_gather<bf16>, dim3(grid), dim3(256), 0, s, (bf16 *)A, lda, list, c0, ncol); break;
    case N3P_FP32: hipLaunchKernelGGL(k_row_gather<float>, dim3(grid), dim3(256), 0, s, (float *)A, lda, list, c0, ncol); break;
    case N3P_FP64: hipLaunchKernelGGL(k_row_gather<double>, dim3(grid), dim3(256), 0, s, (double *)A, lda, list, c0, ncol); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_lt_rebuild(int prec, int64_t Np, int64_t r0, int64_t k0, int64_t ncol,
                             const void *A, int64_t lda, void *LT, hipStream_t s)
{
    if (r0 >= Np || ncol <= 0) return hipSuccess;
    if ((Np - r0) % 64 || ncol % 64 || ncol > NB_OUT) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((Np - r0) / 64), (unsigned)(ncol / 64));
    switch (prec) {
    case N3P_FP16: hipLaunchKernelGGL(k_lt_rebuild<f16>, grid, dim3(256), 0, s, (const f16 *)A, lda, (f16 *)LT, r0, k0); break;
    case N3P_BF16: hipLaunchKernelGGL(k_lt_rebuild<bf16>, grid, dim3(256), 0, s, (const bf16 *)A, lda, (bf16 *)LT, r0, k0); break;
    case N3P_FP32: hipLaunchKernelGGL(k_lt_rebuild<float>, grid, dim3(256), 0, s, (const float *)A, lda, (float *)LT, r0, k0); break;
    case N3P_FP64: hipLaunchKernelGGL(k_lt_rebuild<double>, grid, dim3(256), 0, s, (const double *)A, lda, (double *)LT, r0, k0); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_u12(int prec, int64_t c0, int64_t col0, int64_t col1, void *A, int64_t lda,
                      int *flags, hipStream_t s)
{
    const int64_t ncol = col1 - col0;
    if (ncol <= 0) return hipSuccess;
    const unsigned grid = (unsigned)((ncol + 255) / 256);
    switch (prec) {
    case N3P_FP16: hipLaunchKernelGGL(k_u12<f16>, dim3(grid), dim3(256), 0, s, col0, col1, c0, (f16 *)A, lda, flags); break;
    case N3P_BF16: hipLaunchKernelGGL(k_u12<bf16>, dim3(grid), dim3(256), 0, s, col0, col1, c0, (bf16 *)A, lda, flags); break;
    case N3P_FP32: hipLaunchKernelGGL(k_u12<float>, dim3(grid), dim3(256), 0, s, col0, col1, c0, (float *)A, lda, flags); break;
    case N3P_FP64: hipLaunchKernelGGL(k_u12<double>, dim3(grid), dim3(256), 0, s, col0, col1, c0, (double *)A, lda, flags); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
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
                                         q.flags);
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
