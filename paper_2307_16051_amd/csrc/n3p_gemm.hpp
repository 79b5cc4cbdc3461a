// n3p_gemm.hpp -- the FP16/BF16 matrix-core Schur-complement tile (C -= L U)
// shared by the factorisation kernels (k_getrf.hip, k_panel.hip), and the
// XCD-aware tile order of its launches.
#pragma once

#include "n3p_internal.hpp"

namespace n3p {

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

// LDS elements of one tile: two stages of the A and B operand blocks
template <int TM, int TN, int KC> constexpr int gemm16_lds_elems() { return 2 * (TM + TN) * (KC + 8); }

template <typename T, int TM, int TN, int WGM, int WGN, int KC>
__device__ __forceinline__ void gemm16_tile(int row0, int col0, int K, const T *__restrict__ At,
                                            int64_t ldat, const T *__restrict__ B, int64_t ldb,
                                            T *__restrict__ C, int64_t ldc, int *__restrict__ flags,
                                            T *__restrict__ lds)
{
    typedef typename mfma32<T>::vec vec;
    constexpr int NT = WGM * WGN * 64;
    constexpr int WM = TM / WGM, WN = TN / WGN, FM = WM / 32, FN = WN / 32;
    constexpr int KP = KC + 8;          // padded LDS row (elements): 16-byte skew
    constexpr int CPR = KC / 8;         // 16-byte chunks per row
    constexpr int ACH = TM * CPR / NT;  // A chunks per thread per stage
    constexpr int BCH = TN * CPR / NT;
    static_assert(ACH * NT == TM * CPR && BCH * NT == TN * CPR, "tile/thread mismatch");
    // LDS from the caller: gemm16_lds_elems<TM, TN, KC>() elements, 16-byte aligned
    T (*As)[TM * KP] = (T (*)[TM * KP])lds;
    T (*Bs)[TN * KP] = (T (*)[TN * KP])(lds + 2 * TM * KP);

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

    // epilogue: lane holds column (lane & 31) and rows 8g + 4(lane >> 5) + q.
    // Every C load of the wave is issued before the first store, so the
    // read-modify-write costs one memory round trip, not one per fragment
    // (the compiler cannot move a load past a store to the same array).
    typedef T t4 __attribute__((ext_vector_type(4)));
    t4 cv[FM][FN][4];
#pragma unroll
    for (int fm = 0; fm < FM; ++fm)
#pragma unroll
        for (int fn = 0; fn < FN; ++fn) {
            const T *cp = C + (int64_t)(col0 + wn * WN + fn * 32 + lr) * ldc + row0 + wm * WM +
                          fm * 32 + (lane >> 5) * 4;
#pragma unroll
            for (int gq = 0; gq < 4; ++gq) cv[fm][fn][gq] = *(const t4 *)(cp + gq * 8);
        }
    bool bad = false;
#pragma unroll
    for (int fm = 0; fm < FM; ++fm)
#pragma unroll
        for (int fn = 0; fn < FN; ++fn) {
            T *cp = C + (int64_t)(col0 + wn * WN + fn * 32 + lr) * ldc + row0 + wm * WM + fm * 32 +
                    (lane >> 5) * 4;
#pragma unroll
            for (int gq = 0; gq < 4; ++gq) {
                t4 o;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float v = (float)cv[fm][fn][gq][q] - acc[fm][fn][gq * 4 + q];
                    o[q] = (T)v;
                    bad |= !isfinite((float)o[q]);
                }
                *(t4 *)(cp + gq * 8) = o;
            }
        }
    if (bad) set_flag(&flags[FLAG_NONFINITE], 1);
}

// XCD-aware tile order: workgroups are dispatched round-robin over the 8
// XCDs (workgroup bid runs on XCD bid % 8), so give each XCD a contiguous run
// of the tile sequence: XCD x owns tiles [start_x, start_x + count_x).  A
// bijection for any tile count.
__device__ __forceinline__ int xcd_tile(int bid, int nt)
{
    const int xcd = bid & 7, q8 = nt >> 3, r8 = nt & 7;
    return xcd * q8 + (xcd < r8 ? xcd : r8) + (bid >> 3);
}
// Tile sequence -> (row tile, column tile) in groups of GM row tiles, so the
// tiles an XCD's CUs hold at once share a few A row blocks and B column
// blocks in its L2.
__device__ __forceinline__ void grouped_tile(int tile, int ntm, int ntn, int &tm, int &tn)
{
    constexpr int GM = 8;
    const int per_group = GM * ntn, group = tile / per_group, first_m = group * GM;
    const int gsize = ntm - first_m < GM ? ntm - first_m : GM;
    const int in_group = tile - group * per_group;
    tm = first_m + in_group % gsize;
    tn = in_group / gsize;
}

}  // namespace n3p
