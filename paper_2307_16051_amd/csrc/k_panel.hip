// k_panel.hip -- the no-interchange factorisation of one outer block (up to
// 1024 columns) for FP16 / BF16 storage: Gaussian elimination (Section 1.3)
// on the half-precision copy of the Jacobian (Section 2), checked on the fly
// against partial pivoting as in k_getrf.hip (every Schur-complement entry
// below a pivot must satisfy |a_ik| <= (1 - 2^-8) |a_kk|, i.e. every
// multiplier |l_ik| <= 1 - 2^-8; a failure sets FLAG_FAIL and the host
// factors again with explicit pivoting).
//
// For the outer block with columns [k0, k0 + W):
//   k_top   factors its W x W diagonal square A11 = L11 U11.  One workgroup
//           per 64-row tile, holding the tile's W columns in LDS.  Leaf l
//           (columns 64 l .. 64 l + 63) is factored by workgroup l, which
//           also inverts its triangular factors and forms the leaf's U row
//           block; the workgroups below take their L tile X U^{-1} and their
//           rank-64 update from what it publishes.  Everything a leaf passes
//           on travels as 64-bit words stamped with the leaf's tag (no flag
//           round trip, no cache-wide fence).
//   k_trsm  L21 = A21 U11^{-1} for the 64-row tiles below the square
//           (left-looking over the leaves) and U12 = L11^{-1} A12 for the
//           64-column slabs to its right (block forward substitution).
// The trailing update A22 -= L21 U12 (K = W) is the matrix-core GEMM of
// k_getrf.hip.
//
// Products run on the matrix cores (v_mfma_f32_32x32x16_{f16,bf16}, FP32
// accumulation).  A product with a triangular inverse splits the FP32 inverse
// (scaled by a power of two) into a high and a low half-precision part, and
// an FP32 right-hand side likewise, so it carries about 16-22 bits before the
// result is rounded once to the storage type -- the accuracy of the FP32
// substitution it replaces, not that of half precision.
#include <algorithm>

#include "n3p_gemm.hpp"

namespace n3p {

namespace {

constexpr int PT = 64;               // leaf width and tile height
constexpr int TOP_THREADS = 512;     // eight wavefronts
constexpr int TRSM_THREADS = 512;    // eight wavefronts
constexpr int PSPIN = 1 << 22;       // bounded polls (~0.1 s): a wait that long has failed

// publication words of one leaf (64-bit: tag << 32 | two storage values).
// A 64x64 block published as a matrix-core operand (rows m, depth k) takes
// 2048 words: the pair (k, k + 1) of row m = 32 fm + l32 with
// k = 16 ks + 8 h + 2 e is word op_word(fm, ks, h, l32, e), so the four words
// a lane reads per 16-deep step are adjacent and a wavefront's read of one
// step is 2 KB contiguous.
constexpr int PUB_UINV = 0;          // (U^{-1} * 2^s)^T: high parts, then low parts at + 2048
constexpr int PUB_SCALE = 4096;      // s (four copies)
constexpr int PUB_U12 = 4160;        // + 2048 b: U(leaf, b)^T, the leaf's U rows in block column b
constexpr int PUB_LEAF = PUB_U12 + 16 * 2048;
__host__ __device__ constexpr int op_word(int fm, int ks, int h, int l32, int e)
{
    return (((fm * 4 + ks) * 2 + h) * 32 + l32) * 4 + e;
}
// side buffer for k_trsm (storage type): per leaf the scaled high and low
// parts of (U^{-1})^T and of L^{-1} as matrix-core operands (the pair of word
// op_word(...) at elements 2 op_word(...), + 1); after the 16 leaves, two int
// exponents per leaf (s of U^{-1}, s of L^{-1})
constexpr int IH_UHI = 0, IH_ULO = 4096, IH_LHI = 8192, IH_LLO = 12288, IH_LEAF = 16384;
constexpr int IH_EXP = 16 * IH_LEAF;  // element offset of the exponents (as int pairs)
// then copies of the square's off-diagonal blocks in matrix-core operand
// order, for k_trsm: block (r, b) at OP_U + (16 r + b) * 4096 holds U(r, b)^T
// (b > r) and at OP_L + (16 r + b) * 4096 L(r, b) (b < r); element p of
// lane (h, l32) of 16-deep step ks of row half fm is at
// ((4 fm + ks) * 64 + 32 h + l32) * 8 + p, so one wavefront's operand load
// is 1 KB contiguous
constexpr int OP_U = IH_EXP + 128;
constexpr int OP_L = OP_U + 256 * 4096;
constexpr int IH_TOTAL = OP_L + 256 * 4096;

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// 32x32x16 matrix-core step.  Operands: lane l holds row (A) / column (B)
// l & 31 and the 8 consecutive K values 8 (l >> 5) .. +7 of the 16-deep step;
// result: lane l holds column l & 31, rows 8 g + 4 (l >> 5) + q in acc[4 g + q].
template <typename T> struct pmma;
template <> struct pmma<f16> {
    typedef h8 vec;
    static __device__ __forceinline__ f32x16 op(vec a, vec b, f32x16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};
template <> struct pmma<bf16> {
    typedef b8 vec;
    static __device__ __forceinline__ f32x16 op(vec a, vec b, f32x16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};

template <typename T> __device__ __forceinline__ uint32_t bits(T v)
{
    return (uint32_t)__builtin_bit_cast(unsigned short, v);
}
template <typename T> __device__ __forceinline__ T from_bits(uint32_t b)
{
    return __builtin_bit_cast(T, (unsigned short)(b & 0xffffu));
}
template <typename T> __device__ __forceinline__ uint32_t pack2(T a, T b)
{
    return bits(a) | (bits(b) << 16);
}
template <typename T> __device__ __forceinline__ typename pmma<T>::vec as_vec(u32x4 v)
{
    return __builtin_bit_cast(typename pmma<T>::vec, v);
}
// 1/v: hardware reciprocal estimate refined by one Newton-Raphson step (within
// an ulp of the rounded quotient; the pivots of the leaf chain)
__device__ __forceinline__ float rcp_nr(float v)
{
    const float r = __builtin_amdgcn_rcpf(v);
    return fmaf(fmaf(-v, r, 1.0f), r, r);
}
__device__ __forceinline__ f32x16 zero16()
{
    f32x16 z;
#pragma unroll
    for (int q = 0; q < 16; ++q) z[q] = 0.0f;
    return z;
}

// high / low storage-precision parts of 8 FP32 values (v ~ hi + lo)
template <typename T>
__device__ __forceinline__ void split8(const float (&v)[8], typename pmma<T>::vec &hi,
                                       typename pmma<T>::vec &lo)
{
    u32x4 a, b;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const T h0 = (T)v[2 * p], h1 = (T)v[2 * p + 1];
        const T l0 = (T)(v[2 * p] - to_f32(h0)), l1 = (T)(v[2 * p + 1] - to_f32(h1));
        a[p] = pack2(h0, h1);
        b[p] = pack2(l0, l1);
    }
    hi = as_vec<T>(a);
    lo = as_vec<T>(b);
}

// power-of-two exponent s with max * 2^s in [2^13, 2^14) (0 for a zero max)
__device__ __forceinline__ int scale_exp(float mx)
{
    if (!(mx > 0.0f) || !isfinite(mx)) return 0;
    int e;
    frexpf(mx, &e);
    return 14 - e;
}

// Element (i, c) of a tile with rows of W values held row-major in LDS.  The
// 16-byte chunks of row i are permuted by XOR with i & 7, so 8 consecutive
// rows of one column, and one column chunk of 32 consecutive rows, spread
// over the banks.  Chunks stay 16-byte aligned.
__device__ __forceinline__ int tix(int i, int c, int W)
{
    return i * W + ((((c >> 3) ^ (i & 7)) << 3) | (c & 7));
}

__device__ __forceinline__ uint64_t tload(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void tstore(uint64_t *p, uint32_t tag, uint32_t v)
{
    __hip_atomic_store(p, ((uint64_t)tag << 32) | v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// NG groups of 4 consecutive words per lane (group g at base + g * stride):
// poll until every word of the wavefront carries `tag` (bounded; an expired
// wait raises FLAG_TIMEOUT and returns whatever was read).
template <int NG>
__device__ __forceinline__ void tissue4(const uint64_t *base, int stride, uint64_t (&v)[NG][4])
{
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
        for (int e = 0; e < 4; ++e) v[g][e] = tload(base + g * stride + e);
}
// the wait of tfetch4 on words already issued by tissue4
template <int NG>
__device__ __forceinline__ void twait4(uint64_t (&v)[NG][4], const uint64_t *base, int stride,
                                       uint32_t tag, uint32_t (&out)[NG][4], int *flags)
{
    int spins = 0;
    for (;;) {
        bool ok = true;
#pragma unroll
        for (int g = 0; g < NG; ++g)
#pragma unroll
            for (int e = 0; e < 4; ++e) ok &= (uint32_t)(v[g][e] >> 32) == tag;
        if (__all(ok)) break;
        if (++spins > PSPIN) {
            set_flag(&flags[FLAG_TIMEOUT], 1);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
#pragma unroll
        for (int g = 0; g < NG; ++g)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if ((uint32_t)(v[g][e] >> 32) != tag) v[g][e] = tload(base + g * stride + e);
    }
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
        for (int e = 0; e < 4; ++e) out[g][e] = (uint32_t)v[g][e];
}
template <int NG>
__device__ __forceinline__ void tfetch4(const uint64_t *base, int stride, uint32_t tag,
                                        uint32_t (&out)[NG][4], int *flags)
{
    uint64_t v[NG][4];
    tissue4<NG>(base, stride, v);
    twait4<NG>(v, base, stride, tag, out, flags);
}

template <typename T> __device__ __forceinline__ u32x4 to_u4(const uint32_t (&w)[4])
{
    u32x4 v;
    v[0] = w[0];
    v[1] = w[1];
    v[2] = w[2];
    v[3] = w[3];
    return v;
}

// Max over a wavefront (every lane active) with DPP row operations: two quad
// swaps, then the half-row and row mirrors leave each 16-lane row's max in
// all of its lanes; the four rows are combined through lane reads.  (Max is
// exact, so the order of the comparisons does not change the result.)
__device__ __forceinline__ float dpp_f(float v, int ctrl_sel)
{
    const int b = __float_as_int(v);
    int r;
    switch (ctrl_sel) {
    case 0: r = __builtin_amdgcn_update_dpp(b, b, 0xB1, 0xF, 0xF, false); break;   // quad_perm [1,0,3,2]
    case 1: r = __builtin_amdgcn_update_dpp(b, b, 0x4E, 0xF, 0xF, false); break;   // quad_perm [2,3,0,1]
    case 2: r = __builtin_amdgcn_update_dpp(b, b, 0x141, 0xF, 0xF, false); break;  // row_half_mirror
    default: r = __builtin_amdgcn_update_dpp(b, b, 0x140, 0xF, 0xF, false); break; // row_mirror
    }
    return __int_as_float(r);
}
__device__ __forceinline__ float wave_max(float v)
{
    v = fmaxf(v, dpp_f(v, 0));
    v = fmaxf(v, dpp_f(v, 1));
    v = fmaxf(v, dpp_f(v, 2));
    v = fmaxf(v, dpp_f(v, 3));
    const float a = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    const float b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
    const float c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    const float d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
    return fmaxf(fmaxf(a, b), fmaxf(c, d));
}

// max over a block of NW wavefronts
template <int NW>
__device__ __forceinline__ float block_max(float v, float *red)
{
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    float m = red[0];
#pragma unroll
    for (int i = 1; i < NW; ++i) m = fmaxf(m, red[i]);
    __syncthreads();
    return m;
}

// max over a block of NW wavefronts of two values at once
template <int NW>
__device__ __forceinline__ float2 block_max2(float2 v, float2 *red)
{
    v.x = wave_max(v.x);
    v.y = wave_max(v.y);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    float2 m = red[0];
#pragma unroll
    for (int i = 1; i < NW; ++i) {
        m.x = fmaxf(m.x, red[i].x);
        m.y = fmaxf(m.y, red[i].y);
    }
    __syncthreads();
    return m;
}

typedef float DmRow[PT + 1];

// Inverses of the eight diagonal 8x8 blocks of U and of L, in place: wave J,
// lanes 0..7 the columns of U_JJ^{-1} (back substitution), lanes 8..15 those
// of L_JJ^{-1} (forward substitution, unit diagonal).  The block's entries
// are read into registers first, so the reads issue together instead of one
// per step of the dependent chain.
__device__ __forceinline__ void inv_diag8(DmRow *Dm, int J, int lane)
{
    const int c = lane & 7, b = 8 * J;
    float xd[8];
    if (lane < 8) {
        float u[8][8];
#pragma unroll
        for (int rr = 0; rr < 8; ++rr)
#pragma unroll
            for (int m = rr; m < 8; ++m) u[rr][m] = Dm[b + rr][b + m];
#pragma unroll
        for (int rr = 7; rr >= 0; --rr) {
            float v = rr == c ? 1.0f : 0.0f;
#pragma unroll
            for (int m = rr + 1; m < 8; ++m) v -= u[rr][m] * xd[m];
            xd[rr] = v * rcp_nr(u[rr][rr]);
        }
    } else if (lane < 16) {
        float l[8][8];
#pragma unroll
        for (int rr = 1; rr < 8; ++rr)
#pragma unroll
            for (int m = 0; m < rr; ++m) l[rr][m] = Dm[b + rr][b + m];
#pragma unroll
        for (int rr = 0; rr < 8; ++rr) {
            float v = rr == c ? 1.0f : 0.0f;
#pragma unroll
            for (int m = 0; m < rr; ++m) v -= l[rr][m] * xd[m];
            xd[rr] = v;
        }
    }
    __syncthreads();
    if (lane < 8) {
#pragma unroll
        for (int rr = 0; rr < 8; ++rr)
            if (rr <= c) Dm[b + rr][b + c] = xd[rr];
    } else if (lane < 16) {
#pragma unroll
        for (int rr = 0; rr < 8; ++rr)
            if (rr > c) Dm[b + rr][b + c] = xd[rr];
    }
}

// Doubling 8 -> 16 on the VALU: pairs p = 0, 16, 32, 48; thread t takes
// entry (i, c) of pair q of the U (t < 256) or L (t >= 256) triangle.
__device__ __forceinline__ void inv_double8(DmRow *Dm, float *Ts, int t)
{
    const int tri = t >> 8, q = (t >> 6) & 3, i = (t >> 3) & 7, c = t & 7, p = 16 * q;
    // each phase reads its 16 operands first, then sums in order
    float ra[8], rb[8];
    float v = 0.0f;
    if (tri == 0) {  // T = U12 X22 (X22 upper)
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            rb[m] = Dm[p + 8 + m][p + 8 + c];
            ra[m] = Dm[p + i][p + 8 + m];
        }
#pragma unroll
        for (int m = 0; m < 8; ++m) v += ra[m] * (m <= c ? rb[m] : 0.0f);
    } else {         // T = L21 X11 (X11 unit lower)
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            rb[m] = Dm[p + m][p + c];
            ra[m] = Dm[p + 8 + i][p + m];
        }
#pragma unroll
        for (int m = 0; m < 8; ++m) v += ra[m] * (m > c ? rb[m] : (m == c ? 1.0f : 0.0f));
    }
    Ts[t] = v;
    __syncthreads();
    const float *T = Ts + (t & ~63);  // this pair's T, row-major 8x8
    v = 0.0f;
    if (tri == 0) {  // X12 = -X11 T (X11 upper)
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            ra[m] = Dm[p + i][p + m];
            rb[m] = T[m * 8 + c];
        }
#pragma unroll
        for (int m = 0; m < 8; ++m) v += (m >= i ? ra[m] : 0.0f) * rb[m];
    } else {         // X21 = -X22 T (X22 unit lower)
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            ra[m] = Dm[p + 8 + i][p + 8 + m];
            rb[m] = T[m * 8 + c];
        }
#pragma unroll
        for (int m = 0; m < 8; ++m) v += (m < i ? ra[m] : (m == i ? 1.0f : 0.0f)) * rb[m];
    }
    __syncthreads();
    if (tri == 0) Dm[p + i][p + 8 + c] = -v;
    else Dm[p + 8 + i][p + c] = -v;
    __syncthreads();
}

// 16x16 tile of A B (K = k_len, a multiple of 4) on the FP32 matrix cores
// (v_mfma_f32_16x16x4f32): lane l supplies A[l & 15][k + (l >> 4)] and
// B[k + (l >> 4)][l & 15] for each 4-deep step; the result acc[q] is the entry
// (4 (l >> 4) + q, l & 15).
template <int KL, typename FA, typename FB>
__device__ __forceinline__ f32x4 mm16f32(FA fa, FB fb, int lane)
{
    f32x4 acc;
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = 0.0f;
    const int ci = lane & 15, kq = lane >> 4;
    // every operand read first, then the products in order
    float av[KL / 4], bv[KL / 4];
#pragma unroll
    for (int s = 0; s < KL / 4; ++s) {
        av[s] = fa(ci, 4 * s + kq);
        bv[s] = fb(4 * s + kq, ci);
    }
#pragma unroll
    for (int s = 0; s < KL / 4; ++s) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s], bv[s], acc, 0, 0, 0);
    return acc;
}

// Doubling BS -> 2 BS (BS = 16 or 32) on the matrix cores.  Work items:
// (triangle, pair, 16x16 output tile); BS = 16: 2 pairs x 1 tile per
// triangle, BS = 32: 1 pair x 4 tiles per triangle -- four items per
// triangle, one per wave (waves 0..3 U, 4..7 L).
template <int BS>
__device__ __forceinline__ void inv_double_mfma(DmRow *Dm, float *Ts, int w, int lane)
{
    constexpr int NT = BS / 16;                 // output tiles per side
    constexpr int NPAIR = PT / (2 * BS);        // pairs per triangle
    const int tri = w >> 2, item = w & 3;
    const int q = item / (NT * NT), ti = (item / NT) % NT, tc = item % NT;
    const bool on = q < NPAIR;                  // BS = 16: items 2, 3 have no pair
    const int p = 2 * BS * (on ? q : 0);
    float *T = Ts + tri * 1024 + (on ? q : 0) * BS * BS;   // row-major BS x BS
    const int ci = lane & 15, kq = lane >> 4;
    f32x4 acc;
    if (!on) {
    } else if (tri == 0) {  // T = U12 X22, X22 upper
        acc = mm16f32<BS>([&](int i, int m) { return Dm[p + 16 * ti + i][p + BS + m]; },
                          [&](int m, int c) {
                              const int cc = 16 * tc + c;
                              const float x = Dm[p + BS + m][p + BS + cc];
                              return m <= cc ? x : 0.0f;
                          },
                          lane);
    } else {         // T = L21 X11, X11 unit lower
        acc = mm16f32<BS>([&](int i, int m) { return Dm[p + BS + 16 * ti + i][p + m]; },
                          [&](int m, int c) {
                              const int cc = 16 * tc + c;
                              const float x = Dm[p + m][p + cc];
                              return m > cc ? x : (m == cc ? 1.0f : 0.0f);
                          },
                          lane);
    }
    if (on) {
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) T[(16 * ti + 4 * kq + qq) * BS + 16 * tc + ci] = acc[qq];
    }
    __syncthreads();
    if (!on) {
    } else if (tri == 0) {  // X12 = -X11 T, X11 upper
        acc = mm16f32<BS>([&](int i, int m) {
                              const int ii = 16 * ti + i;
                              const float x = Dm[p + ii][p + m];
                              return m >= ii ? x : 0.0f;
                          },
                          [&](int m, int c) { return T[m * BS + 16 * tc + c]; }, lane);
    } else {         // X21 = -X22 T, X22 unit lower
        acc = mm16f32<BS>([&](int i, int m) {
                              const int ii = 16 * ti + i;
                              const float x = Dm[p + BS + ii][p + BS + m];
                              return m < ii ? x : (m == ii ? 1.0f : 0.0f);
                          },
                          [&](int m, int c) { return T[m * BS + 16 * tc + c]; }, lane);
    }
    __syncthreads();
    if (on) {
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
            const int ii = 16 * ti + 4 * kq + qq, cc = 16 * tc + ci;
            if (tri == 0) Dm[p + ii][p + BS + cc] = -acc[qq];
            else Dm[p + BS + ii][p + cc] = -acc[qq];
        }
    }
    __syncthreads();
}

struct TopArgs {
    int64_t k0;      // first row and column of the diagonal square
    int W;           // its size (multiple of 64, <= 1024)
    void *A;         // factor matrix, column-major
    int64_t lda;
    void *LT;        // L rows, row-major, ld NB_OUT (column index relative to k0)
    uint64_t *pub;   // PUB_LEAF words per leaf
    void *inv;       // side buffer: the inverses for k_trsm
    int *flags;
    uint32_t tag0;   // leaf l publishes with tag0 + l (tags never repeat within a factorisation)
};

// ======================================================================= k_top
// LDS of the square's workgroup: the row tile, the diagonal block (FP32),
// the inversion scratch and two small reduction areas.
constexpr int TOP_TILE_BYTES = PT * NB_OUT * 2;
constexpr int TOP_DM_BYTES = PT * (PT + 1) * 4;
constexpr int TOP_TS_BYTES = 2048 * 4;
constexpr int TOP_LDS_BYTES = TOP_TILE_BYTES + TOP_DM_BYTES + TOP_TS_BYTES + 64 + 16;

// Workgroup r of the diagonal square (see the file comment).  lds: at least
// TOP_LDS_BYTES, 16-byte aligned.
template <typename T>
__device__ __forceinline__ void top_body(const TopArgs &a, int r, char *lds)
{
    typedef typename pmma<T>::vec vec;
    T *tile = (T *)lds;
    DmRow *Dm = (DmRow *)(lds + TOP_TILE_BYTES);
    float *Ts = (float *)(lds + TOP_TILE_BYTES + TOP_DM_BYTES);
    float2 *red2 = (float2 *)(lds + TOP_TILE_BYTES + TOP_DM_BYTES + TOP_TS_BYTES);
    int &sfail = *(int *)(lds + TOP_TILE_BYTES + TOP_DM_BYTES + TOP_TS_BYTES + 64);
    if (block_flag(&a.flags[FLAG_FAIL])) return;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, h = lane >> 5, l32 = lane & 31;
    const int W = a.W, nl = W / PT;
    T *A = (T *)a.A;
    const int64_t lda = a.lda, k0 = a.k0, row0 = k0 + (int64_t)r * PT;
    int *flags = a.flags;
    const float margin = 1.0f - 1.0f / 256.0f;

    // ---- the row tile: rows row0 .. row0 + 63, columns k0 .. k0 + W - 1
    for (int e = t; e < W * 8; e += TOP_THREADS) {
        const int c = e >> 3, rc = e & 7;
        const u32x4 v = *(const u32x4 *)(A + (row0 + rc * 8) + (k0 + c) * lda);
#pragma unroll
        for (int q = 0; q < 8; ++q) tile[tix(rc * 8 + q, c, W)] = from_bits<T>(v[q >> 1] >> (16 * (q & 1)));
    }
    if (t == 0) sfail = 0;
    __syncthreads();

    bool bad = false;
    uint64_t pre[4][4];  // words requested ahead (see below)
    // L tile of leaf l: L^T = (U^{-1})^T X^T on waves 0..3 (fm: leaf columns,
    // fn: tile rows), from the published scaled U^{-1} halves.
    auto l21 = [&](int l) {
        const uint64_t *pl = a.pub + (size_t)l * PUB_LEAF;
        const uint32_t tag = a.tag0 + (uint32_t)l;
        f32x16 acc = zero16();
        float sc = 1.0f;
        const int fm = w & 1, fn = (w >> 1) & 1, i = 32 * fn + l32;
        if (w < 4) {
            uint32_t uh[4][4], ul[4][4], se[1][4];
            // all three requested before the first wait: one memory round
            // trip once the leaf has published, not three
            uint64_t vh[4][4], vl[4][4], vs[1][4];
            const uint64_t *ph = pl + PUB_UINV + op_word(fm, 0, h, l32, 0);
            tissue4<4>(ph, op_word(0, 1, 0, 0, 0), vh);
            tissue4<4>(ph + 2048, op_word(0, 1, 0, 0, 0), vl);
            tissue4<1>(pl + PUB_SCALE, 0, vs);
            twait4<4>(vh, ph, op_word(0, 1, 0, 0, 0), tag, uh, flags);
            twait4<4>(vl, ph + 2048, op_word(0, 1, 0, 0, 0), tag, ul, flags);
            twait4<1>(vs, pl + PUB_SCALE, 0, tag, se, flags);
            sc = ldexpf(1.0f, -(int)se[0][0]);
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const vec b = as_vec<T>(*(const u32x4 *)&tile[tix(i, 64 * l + 16 * ks + 8 * h, W)]);
                acc = pmma<T>::op(as_vec<T>(to_u4<T>(uh[ks])), b, acc);
                acc = pmma<T>::op(as_vec<T>(to_u4<T>(ul[ks])), b, acc);
            }
        }
        __syncthreads();  // every read of X done before L overwrites it
        if (w < 4) {
            bool f = false;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                T o[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float v = acc[4 * g + q] * sc;
                    f |= !(fabsf(v) <= margin);
                    o[q] = (T)v;
                }
                u32x2 st;
                st[0] = pack2(o[0], o[1]);
                st[1] = pack2(o[2], o[3]);
                *(u32x2 *)&tile[tix(i, 64 * l + 32 * fm + 8 * g + 4 * h, W)] = st;
            }
            if (f) set_flag(&flags[FLAG_FAIL], 1);
        }
        __syncthreads();
    };
    // Update of 32 columns (half hf) of block column b, both row halves of
    // the tile, by leaves l0 .. l1 - 1 at once: C^T -= sum_l U(l, b)^T L(r, l)^T
    // (one rounding), U(l, b) from leaf l's words.
    // use_pre: leaf l0's words are already issued into pre (tissue4)
    auto upd_range = [&](int l0, int l1, int b, int hf, bool use_pre) {
        const int wofs = PUB_U12 + b * 2048 + op_word(hf, 0, h, l32, 0);
        constexpr int wstr = op_word(0, 1, 0, 0, 0);
        f32x16 acc[2] = {zero16(), zero16()};
        // the next leaf's words are requested before this leaf's products,
        // so a run of leaves costs about one memory round trip each, not two
        uint64_t vn[4][4];
        if (!(use_pre && l1 > l0)) {
            if (l0 < l1) tissue4<4>(a.pub + (size_t)l0 * PUB_LEAF + wofs, wstr, vn);
        }
        for (int l = l0; l < l1; ++l) {
            uint32_t uw[4][4];
            if (use_pre && l == l0)
                twait4<4>(pre, a.pub + (size_t)l * PUB_LEAF + wofs, wstr, a.tag0 + (uint32_t)l, uw, flags);
            else
                twait4<4>(vn, a.pub + (size_t)l * PUB_LEAF + wofs, wstr, a.tag0 + (uint32_t)l, uw, flags);
            if (l + 1 < l1) tissue4<4>(a.pub + (size_t)(l + 1) * PUB_LEAF + wofs, wstr, vn);
#pragma unroll
            for (int fn = 0; fn < 2; ++fn) {
                const int i = 32 * fn + l32;
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    const vec lb = as_vec<T>(*(const u32x4 *)&tile[tix(i, 64 * l + 16 * ks + 8 * h, W)]);
                    acc[fn] = pmma<T>::op(as_vec<T>(to_u4<T>(uw[ks])), lb, acc[fn]);
                }
            }
        }
#pragma unroll
        for (int fn = 0; fn < 2; ++fn) {
            const int i = 32 * fn + l32;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                u32x2 *p = (u32x2 *)&tile[tix(i, 64 * b + 32 * hf + 8 * g + 4 * h, W)];
                const u32x2 cv = *p;
                T o[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    o[q] = (T)(to_f32(from_bits<T>(cv[q >> 1] >> (16 * (q & 1)))) - acc[fn][4 * g + q]);
                    bad |= !isfinite(to_f32(o[q]));
                }
                u32x2 st;
                st[0] = pack2(o[0], o[1]);
                st[1] = pack2(o[2], o[3]);
                *p = st;
            }
        }
    };
    // upd_range for one leaf and one row half fn of the tile (the same sums
    // in the same order), so that four waves share a block
    auto upd_half = [&](int l, int b, int hf, int fn) {
        uint32_t uw[4][4];
        tfetch4<4>(a.pub + (size_t)l * PUB_LEAF + PUB_U12 + b * 2048 + op_word(hf, 0, h, l32, 0),
                   op_word(0, 1, 0, 0, 0), a.tag0 + (uint32_t)l, uw, flags);
        const int i = 32 * fn + l32;
        f32x16 acc = zero16();
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const vec lb = as_vec<T>(*(const u32x4 *)&tile[tix(i, 64 * l + 16 * ks + 8 * h, W)]);
            acc = pmma<T>::op(as_vec<T>(to_u4<T>(uw[ks])), lb, acc);
        }
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            u32x2 *p = (u32x2 *)&tile[tix(i, 64 * b + 32 * hf + 8 * g + 4 * h, W)];
            const u32x2 cv = *p;
            T o[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                o[q] = (T)(to_f32(from_bits<T>(cv[q >> 1] >> (16 * (q & 1)))) - acc[4 * g + q]);
                bad |= !isfinite(to_f32(o[q]));
            }
            u32x2 st;
            st[0] = pack2(o[0], o[1]);
            st[1] = pack2(o[2], o[3]);
            *p = st;
        }
    };
    // the update by leaf l of block columns b0 .. b1, spread over the waves
    // (four units per block: column half hf, row half fn)
    auto update = [&](int l, int b0, int b1) {
        for (int u = w; u < 4 * (b1 - b0 + 1); u += 8) upd_half(l, b0 + (u >> 2), (u >> 1) & 1, u & 1);
    };

    // ---- the leaves above this tile: L tile, then the rank-64 update of the
    // blocks up to r + 1 only (the last leaf, r - 1: of the diagonal block
    // only).  Blocks further right take all their updates at once just
    // before their U rows are formed, so this workgroup never waits for the
    // U rows a leaf forms last.
    for (int l = 0; l < r; ++l) {
        l21(l);
        update(l, l + 1, l + 1 < r ? std::min(r + 1, nl - 1) : r);
        __syncthreads();
    }

    // the words of U(r - 1, r + 1), half w, that waves 0 and 1 apply to
    // block r + 1 right after the inversion (requested before the inversion)
    const bool have_pre = r > 0 && r + 1 < nl && w < 2;

    // ---- leaf r: factor the diagonal block (columns 64 r .. 64 r + 63) with
    // the partial-pivoting check.  Wave w keeps columns 8 w .. 8 w + 7 of all
    // 64 rows (lane = row); the owner of strip p factors it with readlane
    // broadcasts, and after one barrier every later wave applies it.
    {
        float x[8];
        {
            const u32x4 v = *(const u32x4 *)&tile[tix(lane, 64 * r + 8 * w, W)];
#pragma unroll
            for (int c = 0; c < 8; ++c) x[c] = to_f32(from_bits<T>(v[c >> 1] >> (16 * (c & 1))));
        }
        bool fail = false;
        for (int p = 0; p < 8; ++p) {
            if (w == p) {
#pragma unroll
                for (int kk = 0; kk < 8; ++kk) {
                    const int k = 8 * p + kk;
                    const float piv = lane_bcast(x[kk], k);
                    const float rp = rcp_nr(piv);
                    const bool below = lane > k;
                    fail |= !(fabsf(piv) > 0.0f) || (below && !(fabsf(x[kk]) <= margin * fabsf(piv)));
                    const float lx = x[kk] * rp;
                    const float lv = below ? lx : 0.0f;
                    x[kk] = below ? lx : x[kk];
                    // all broadcasts first, then the updates: independent
                    // readlanes issue back to back instead of alternating
                    // with the FMAs that consume them
                    float ub[8];
#pragma unroll
                    for (int c = kk + 1; c < 8; ++c) ub[c] = lane_bcast(x[c], k);
#pragma unroll
                    for (int c = kk + 1; c < 8; ++c) x[c] -= lv * ub[c];
                }
#pragma unroll
                for (int c = 0; c < 8; ++c) Dm[lane][8 * p + c] = x[c];
            }
            __syncthreads();
            if (w > p) {
                float lv[8];
#pragma unroll
                for (int kk = 0; kk < 8; ++kk) lv[kk] = lane > 8 * p + kk ? Dm[lane][8 * p + kk] : 0.0f;
#pragma unroll
                for (int kk = 0; kk < 8; ++kk) {
                    float ub[8];
#pragma unroll
                    for (int c = 0; c < 8; ++c) ub[c] = lane_bcast(x[c], 8 * p + kk);
#pragma unroll
                    for (int c = 0; c < 8; ++c) x[c] -= lv[kk] * ub[c];
                }
            }
        }
        if (fail) sfail = 1;
    }
    __syncthreads();
    if (t == 0 && sfail) set_flag(&flags[FLAG_FAIL], 1);
    // factored block into the tile (its final values)
    {
        const int i = t >> 3, cc = (t & 7) * 8;
        T o[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            o[q] = (T)Dm[i][cc + q];
            bad |= !isfinite(to_f32(o[q]));
        }
        u32x4 st;
#pragma unroll
        for (int p = 0; p < 4; ++p) st[p] = pack2(o[2 * p], o[2 * p + 1]);
        *(u32x4 *)&tile[tix(i, 64 * r + cc, W)] = st;
    }

    // ---- triangular inverses in place in Dm: U^{-1} on and above the
    // diagonal, L^{-1} (unit diagonal) below it.  Diagonal 8x8 blocks first,
    // then three doublings (8 -> 16 -> 32 -> 64): for a pair of inverted
    // diagonal blocks X11, X22 and the block U12 (L21) between them,
    // X12 = -X11 (U12 X22) and X21 = -X22 (L21 X11).
    // U(r - 1, r + 1) requested now: leaf r - 1 forms it after handing over
    // U(r - 1, r), so a request before the diagonal factorisation could
    // still find the words unpublished and the wait after the inversion
    // would pay a whole round trip; requested here, the words are back with
    // the right tag by then and their latency is off the chain
    if (have_pre)
        tissue4<4>(a.pub + (size_t)(r - 1) * PUB_LEAF + PUB_U12 + (r + 1) * 2048 + op_word(w, 0, h, l32, 0),
                   op_word(0, 1, 0, 0, 0), pre);
    inv_diag8(Dm, w, lane);
    __syncthreads();
    inv_double8(Dm, Ts, t);
    inv_double_mfma<16>(Dm, Ts, w, lane);
    inv_double_mfma<32>(Dm, Ts, w, lane);
    // scale exponents of the two inverses for the split into halves
    int su, sl;
    {
        float mu = 0.0f, ml = 1.0f;
        static_assert(PT * PT % TOP_THREADS == 0, "whole rounds");
#pragma unroll
        for (int k = 0; k < PT * PT / TOP_THREADS; ++k) {
            const int e = t + k * TOP_THREADS, i = e >> 6, j = e & 63;
            const float v = fabsf(Dm[i][j]);
            if (i <= j) mu = fmaxf(mu, v);
            else ml = fmaxf(ml, v);
        }
        float2 m2 = block_max2<TOP_THREADS / 64>(make_float2(mu, ml), red2);
        su = scale_exp(m2.x);
        sl = scale_exp(m2.y);
    }
    // ---- what leaf r passes on.  U(r, r + 1) first, since the next leaf's
    // workgroup waits for it: waves 0 and 1 form it with the scaled halves of
    // L^{-1} in registers, while waves 2..7 publish (U^{-1})^T (scaled
    // halves; row j of the operand is column j of U^{-1}) and write the same
    // words to the side buffer.  Then L^{-1} replaces Dm in LDS as the A
    // operand of the remaining U row blocks.
    T *iv = (T *)a.inv + (size_t)r * IH_LEAF;
    const float ful = ldexpf(1.0f, -sl);
    // U rows of leaf r in block columns b > r: U12 = L^{-1} T_b.  Unit
    // (b, fn): 32 columns of block b, both row halves.  A operand opa(fm, ks,
    // lo): the high (lo = 0) or low part of L^{-1} (rows 32 fm + l32) scaled
    // by 2^sl; B operand: 8 consecutive tile rows of one column.
    auto u12 = [&](int b, int fn, auto opa) {
        const uint32_t tag = a.tag0 + (uint32_t)r;
        uint64_t *pw = a.pub + (size_t)r * PUB_LEAF + PUB_U12 + b * 2048;
        const int c = 64 * b + 32 * fn + l32;
        vec tb[4];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            u32x4 v;
#pragma unroll
            for (int p = 0; p < 4; ++p)
                v[p] = pack2(tile[tix(16 * ks + 8 * h + 2 * p, c, W)], tile[tix(16 * ks + 8 * h + 2 * p + 1, c, W)]);
            tb[ks] = as_vec<T>(v);
        }
#pragma unroll
        for (int fm = 0; fm < 2; ++fm) {
            f32x16 acc = zero16();
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                acc = pmma<T>::op(opa(fm, ks, 0), tb[ks], acc);
                acc = pmma<T>::op(opa(fm, ks, 1), tb[ks], acc);
            }
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                T o[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    o[q] = (T)(acc[4 * g + q] * ful);
                    bad |= !isfinite(to_f32(o[q]));
                    tile[tix(32 * fm + 8 * g + 4 * h + q, c, W)] = o[q];
                }
                // rows k = 32 fm + 8 g + 4 h .. + 3 of operand row 32 fn + l32
                const int wd = op_word(fn, 2 * fm + (g >> 1), g & 1, l32, 2 * h);
                tstore(pw + wd, tag, pack2(o[0], o[1]));
                tstore(pw + wd + 1, tag, pack2(o[2], o[3]));
            }
        }
    };
    // the scaled L^{-1} operand piece (fm, ks) of this lane, from Dm
    auto linv8 = [&](int fm, int ks, vec &hi, vec &lo) {
        const float fl = ldexpf(1.0f, sl);
        const int m = 32 * fm + l32;
        float v[8];
        // every entry read (the address is always in the block), then the
        // triangle selected, so the reads are not masked one by one
#pragma unroll
        for (int p = 0; p < 8; ++p) v[p] = Dm[m][16 * ks + 8 * h + p];
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            const int k = 16 * ks + 8 * h + p;
            v[p] = (k < m ? v[p] : (k == m ? 1.0f : 0.0f)) * fl;
        }
        split8<T>(v, hi, lo);
    };
    if (w < 2) {
        if (r + 1 < nl) {
            vec lah[2][4], lal[2][4];
#pragma unroll
            for (int fm = 0; fm < 2; ++fm)
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) linv8(fm, ks, lah[fm][ks], lal[fm][ks]);
            if (r > 0) upd_range(r - 1, r, r + 1, w, have_pre);
            u12(r + 1, w, [&](int fm, int ks, int lo) { return lo ? lal[fm][ks] : lah[fm][ks]; });
        }
    } else {
        const uint32_t tag = a.tag0 + (uint32_t)r;
        uint64_t *pr = a.pub + (size_t)r * PUB_LEAF;
        const float fu = ldexpf(1.0f, su);
        for (int e = t - 128; e < 2048; e += TOP_THREADS - 128) {
            // e = op_word(fm, ks, h, l32, q)
            const int q = e & 3, l32e = (e >> 2) & 31, he = (e >> 7) & 1, kse = (e >> 8) & 3, fme = e >> 10;
            const int j = 32 * fme + l32e, k = 16 * kse + 8 * he + 2 * q;
            const float v0 = k <= j ? Dm[k][j] * fu : 0.0f;
            const float v1 = k + 1 <= j ? Dm[k + 1][j] * fu : 0.0f;
            const T h0 = (T)v0, h1 = (T)v1;
            const T q0 = (T)(v0 - to_f32(h0)), q1 = (T)(v1 - to_f32(h1));
            tstore(pr + PUB_UINV + e, tag, pack2(h0, h1));
            tstore(pr + PUB_UINV + 2048 + e, tag, pack2(q0, q1));
            *(uint32_t *)(iv + IH_UHI + 2 * e) = pack2(h0, h1);
            *(uint32_t *)(iv + IH_ULO + 2 * e) = pack2(q0, q1);
        }
        if (t - 128 < 4) tstore(pr + PUB_SCALE + (t - 128), tag, (uint32_t)su);
    }
    // L^{-1} to the side buffer and into LDS in place of Dm: wave w forms
    // step ks = w & 3 of row half fm = w >> 2
    u32x4 *lop = (u32x4 *)Dm;  // [hi / lo][fm][ks][lane]
    {
        vec hi, lo;
        linv8(w >> 2, w & 3, hi, lo);
        const u32x4 uhv = __builtin_bit_cast(u32x4, hi), ulv = __builtin_bit_cast(u32x4, lo);
        *(u32x4 *)(iv + IH_LHI + (w * 64 + lane) * 8) = uhv;
        *(u32x4 *)(iv + IH_LLO + (w * 64 + lane) * 8) = ulv;
        __syncthreads();  // every read of Dm done
        lop[w * 64 + lane] = uhv;
        lop[512 + w * 64 + lane] = ulv;
        if (t == 0) {
            int *ex = (int *)((T *)a.inv + IH_EXP);
            ex[2 * r] = su;
            ex[2 * r + 1] = sl;
        }
        __syncthreads();
    }
    // the remaining U row blocks, block by block, each wave 32 columns after
    // their remaining updates (later blocks: every leaf above at once)
    auto opl = [&](int fm, int ks, int lo) { return as_vec<T>(lop[lo * 512 + (fm * 4 + ks) * 64 + lane]); };
    for (int u = w < 2 ? w + 8 : w; u < 2 * (nl - r - 1); u += 8) {
        const int b = r + 1 + (u >> 1), hf = u & 1;
        if (r > 0) upd_range(0, r, b, hf, false);
        u12(b, hf, opl);
    }
    __syncthreads();

    // ---- copies of this row tile's off-diagonal blocks in operand order for
    // k_trsm: U(r, b)^T for b > r (element (m, k) = tile(k, 64 b + m)) and
    // L(r, i) for i < r (element (m, k) = tile(m, 64 i + k))
    {
        T *op = (T *)a.inv;
        for (int e = t; e < (nl - r - 1) * 512; e += TOP_THREADS) {
            const int b = r + 1 + e / 512, q = e % 512;
            const int ln = q & 63, fk = q >> 6;
            const int m = 32 * (fk >> 2) + (ln & 31), k = 16 * (fk & 3) + 8 * (ln >> 5);
            u32x4 v;
#pragma unroll
            for (int p = 0; p < 4; ++p)
                v[p] = pack2(tile[tix(k + 2 * p, 64 * b + m, W)], tile[tix(k + 2 * p + 1, 64 * b + m, W)]);
            *(u32x4 *)(op + OP_U + (size_t)(r * 16 + b) * 4096 + q * 8) = v;
        }
        for (int e = t; e < r * 512; e += TOP_THREADS) {
            const int i = e / 512, q = e % 512;
            const int ln = q & 63, fk = q >> 6;
            const int m = 32 * (fk >> 2) + (ln & 31), k = 16 * (fk & 3) + 8 * (ln >> 5);
            *(u32x4 *)(op + OP_L + (size_t)(r * 16 + i) * 4096 + q * 8) =
                *(const u32x4 *)&tile[tix(m, 64 * i + k, W)];
        }
    }
    // ---- the finished tile to A (column-major) and LT (row-major)
    for (int e = t; e < W * 8; e += TOP_THREADS) {
        const int c = e >> 3, rc = e & 7;
        u32x4 v;
#pragma unroll
        for (int p = 0; p < 4; ++p)
            v[p] = pack2(tile[tix(rc * 8 + 2 * p, c, W)], tile[tix(rc * 8 + 2 * p + 1, c, W)]);
        *(u32x4 *)(A + (row0 + rc * 8) + (k0 + c) * lda) = v;
    }
    {
        T *LT = (T *)a.LT;
        const int cpr = W / 8;
        for (int e = t; e < PT * cpr; e += TOP_THREADS) {
            const int i = e / cpr, cc = (e % cpr) * 8;
            *(u32x4 *)(LT + (row0 + i) * NB_OUT + cc) = *(const u32x4 *)&tile[tix(i, cc, W)];
        }
    }
    if (bad) set_flag(&flags[FLAG_NONFINITE], 1);
}

template <typename T>
__global__ __launch_bounds__(TOP_THREADS) void k_top(TopArgs a)
{
    __shared__ __attribute__((aligned(16))) char lds[TOP_LDS_BYTES];
    top_body<T>(a, blockIdx.x, lds);
}

// The next block's diagonal square and the rest of this block's trailing
// update in one launch: workgroups 0 .. ntop - 1 factor the square (they are
// dispatched first, on an idle device, so they are resident together), the
// others each take one 256x256 tile of C[M x N] -= At^T B (K = the block
// width).  The two touch disjoint data: the square's columns are left of
// the update's, and the square's L rows go to the other L buffer.
struct TopGemmArgs {
    TopArgs top;
    int ntop;
    int M, N, K;
    const void *At;
    int64_t ldat;
    const void *B;
    int64_t ldb;
    void *C;
    int64_t ldc;
    // a second region with the same K and leading dimensions (M2 = 0: none)
    int M2, N2;
    const void *At2;
    const void *B2;
    void *C2;
};

template <typename T>
__global__ __launch_bounds__(TOP_THREADS) void k_top_gemm(TopGemmArgs a)
{
    __shared__ __attribute__((aligned(16))) char lds[TOP_LDS_BYTES];
    static_assert(gemm16_lds_elems<256, 256, 32>() * 2 <= TOP_LDS_BYTES, "GEMM tile LDS");
    if ((int)blockIdx.x < a.ntop) {
        top_body<T>(a.top, blockIdx.x, lds);
        return;
    }
    if (block_flag(&a.top.flags[FLAG_FAIL])) return;
    const int ntm = a.M / 256, ntn = a.N / 256, n1 = ntm * ntn;
    const int ntm2 = a.M2 / 256, ntn2 = a.N2 / 256;
    int tile = xcd_tile((int)blockIdx.x - a.ntop, n1 + ntm2 * ntn2), tm, tn;
    if (tile < n1) {
        grouped_tile(tile, ntm, ntn, tm, tn);
        gemm16_tile<T, 256, 256, 2, 4, 32>(tm * 256, tn * 256, a.K, (const T *)a.At, a.ldat,
                                           (const T *)a.B, a.ldb, (T *)a.C, a.ldc, a.top.flags, (T *)lds);
    } else {
        grouped_tile(tile - n1, ntm2, ntn2, tm, tn);
        gemm16_tile<T, 256, 256, 2, 4, 32>(tm * 256, tn * 256, a.K, (const T *)a.At2, a.ldat,
                                           (const T *)a.B2, a.ldb, (T *)a.C2, a.ldc, a.top.flags, (T *)lds);
    }
}

// ====================================================================== k_trsm
struct TrsmArgs {
    int64_t k0;
    int W;
    int nrt;          // 64-row tiles below the square (= 64-column slabs right of it)
    void *A;
    int64_t lda;
    void *LT;
    const void *inv;  // the inverses' side buffer written by k_top
    int *flags;
};

// Element (k, c) of a slab of 64 columns with columns of R values held
// column-major in LDS; chunks of 8 rows permuted by XOR with c & 7.
__device__ __forceinline__ int six(int k, int c, int R)
{
    return c * R + ((((k >> 3) ^ (c & 7)) << 3) | (k & 7));
}

// Per-workgroup state of k_trsm.  Eight wavefronts; wave w takes the 32x32
// fragment f = w & 3 ((fm, fn) = (f & 1, f >> 1)) of each 64x64 block and
// one half kh = w >> 2 of the K range of its sum.  Left-looking: block I's
// sum over the finished blocks i < I (U(i,I)^T L(:,i)^T for the rows below,
// L(I,i) U(i) for the columns right) is formed in FP32 at step I, so every
// entry is rounded to the storage type once.  The global operands of step
// I + 1's sum are requested as soon as step I's sum has consumed its
// registers, so their latency overlaps step I's diagonal-block work; waves
// 0..3 then solve the block (one fragment each).
constexpr int TRSM_PF = 2 * (NB_OUT / PT - 1);  // 16-deep K steps of the longest half sum

template <typename T> struct TrsmCtx {
    int64_t k0, lda, base;   // base: first row (role L) or column (role U) of the 64
    int W, nl, w, kh, h, l32, fm, fn;
    T *A;
    const T *LT, *inv;
    int ex[32];              // the leaves' exponents (s of U^{-1}, s of L^{-1})
    T *buf, *stg;
    float *pbuf, *red;
    bool bad, fail;
};

// the scaled high/low split of the FP32 values y (this lane's 16 fragment
// entries, waves 0..3) staged for use as a matrix-core operand; returns the
// exponent
template <typename T>
__device__ __forceinline__ int stage_split(TrsmCtx<T> &c, const float (&y)[16], bool rowmajor, int blk)
{
    float mx = 0.0f;
#pragma unroll
    for (int q = 0; q < 16; ++q) mx = fmaxf(mx, fabsf(y[q]));
    const int sy = scale_exp(block_max<8>(c.w < 4 ? mx : 0.0f, c.red));
    const float fy = ldexpf(1.0f, sy);
    if (c.w >= 4) return sy;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        T hi[4], lo[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float v = y[4 * g + q] * fy;
            hi[q] = (T)v;
            lo[q] = (T)(v - to_f32(hi[q]));
        }
        u32x2 sh, sl;
        sh[0] = pack2(hi[0], hi[1]);
        sh[1] = pack2(hi[2], hi[3]);
        sl[0] = pack2(lo[0], lo[1]);
        sl[1] = pack2(lo[2], lo[3]);
        const int k = 32 * c.fm + 8 * g + 4 * c.h;  // fragment row (block-local)
        if (rowmajor) {  // role L: entry (tile row i, leaf column k)
            const int i = 32 * c.fn + c.l32;
            *(u32x2 *)&c.buf[tix(i, 64 * blk + k, c.W)] = sh;
            *(u32x2 *)&c.stg[tix(i, k, PT)] = sl;
        } else {         // role U: entry (block row k, slab column cc)
            const int cc = 32 * c.fn + c.l32;
            *(u32x2 *)&c.buf[six(64 * blk + k, cc, c.W)] = sh;
            *(u32x2 *)&c.stg[six(k, cc, PT)] = sl;
        }
    }
    return sy;
}

// the two K halves of a fragment's sum: waves 4..7 hand theirs to waves 0..3
template <typename T>
__device__ __forceinline__ void join_halves(TrsmCtx<T> &c, f32x16 &p)
{
    const int lane = 32 * c.h + c.l32, f = c.w & 3;
    if (c.kh == 1) {
#pragma unroll
        for (int j = 0; j < 16; ++j) c.pbuf[(f * 16 + j) * 64 + lane] = p[j];
    }
    __syncthreads();
    if (c.kh == 0) {
#pragma unroll
        for (int j = 0; j < 16; ++j) p[j] += c.pbuf[(f * 16 + j) * 64 + lane];
    }
}

// ---- role L, block I: L(:, I) = (X_I - sum_{i<I} L(:, i) U(i, I)) U_II^{-1}.
// pf: this wave's A operands of block I's half sum (requested at step I - 1).
template <typename T, int I> struct StepL {
    typedef typename pmma<T>::vec vec;
    static __device__ __forceinline__ void prefetch(const TrsmCtx<T> &c, u32x4 (&pf)[TRSM_PF])
    {
        if constexpr (I >= 1 && I < 16) {
            if (I < c.nl) {
                const T *op = c.inv + OP_U + I * 4096 + (c.fm * 4 * 64 + 32 * c.h + c.l32) * 8;
#pragma unroll
                for (int s = 0; s < 2 * I; ++s) {
                    const int K = c.kh * 32 * I + 16 * s;  // block K >> 6, step (K >> 4) & 3
                    pf[s] = *(const u32x4 *)(op + (K >> 6) * 16 * 4096 + ((K >> 4) & 3) * 64 * 8);
                }
            }
        }
    }
    static __device__ __forceinline__ void run(TrsmCtx<T> &c, u32x4 (&pf)[TRSM_PF])
    {
        if (I >= c.nl) return;
        const int W = c.W, h = c.h, l32 = c.l32, fm = c.fm, fn = c.fn;
        const int i = 32 * fn + l32;
        const T *iv = c.inv + (size_t)I * IH_LEAF + (fm * 4 * 64 + 32 * h + l32) * 8;
        u32x4 uh[4], ul[4];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            uh[ks] = *(const u32x4 *)(iv + IH_UHI + ks * 64 * 8);
            ul[ks] = *(const u32x4 *)(iv + IH_ULO + ks * 64 * 8);
        }
        // this wave's half of P^T = U(<I, I)^T L(:, <I)^T
        f32x16 p = zero16();
#pragma unroll
        for (int s = 0; s < 2 * I; ++s) {
            const vec bv = as_vec<T>(*(const u32x4 *)&c.buf[tix(i, c.kh * 32 * I + 16 * s + 8 * h, W)]);
            p = pmma<T>::op(as_vec<T>(pf[s]), bv, p);
        }
        StepL<T, I + 1>::prefetch(c, pf);
        join_halves(c, p);
        // Y^T fragment: rows = leaf columns 32 fm + 8 g + 4 h + q of block I, column = tile row i
        float y[16];
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const u32x2 xv = *(const u32x2 *)&c.buf[tix(i, 64 * I + 32 * fm + 8 * g + 4 * h, W)];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                y[4 * g + q] = to_f32(from_bits<T>(xv[q >> 1] >> (16 * (q & 1)))) - p[4 * g + q];
        }
        const int sy = stage_split<T>(c, y, true, I);
        __syncthreads();
        f32x16 r = zero16();
        if (c.w < 4) {
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const vec yh = as_vec<T>(*(const u32x4 *)&c.buf[tix(i, 64 * I + 16 * ks + 8 * h, W)]);
                const vec yl = as_vec<T>(*(const u32x4 *)&c.stg[tix(i, 16 * ks + 8 * h, PT)]);
                r = pmma<T>::op(as_vec<T>(uh[ks]), yh, r);
                r = pmma<T>::op(as_vec<T>(ul[ks]), yh, r);
                r = pmma<T>::op(as_vec<T>(uh[ks]), yl, r);
            }
        }
        __syncthreads();  // staged reads done before L overwrites them
        if (c.w < 4) {
            const float back = ldexpf(1.0f, -(c.ex[2 * I] + sy));
            const float margin = 1.0f - 1.0f / 256.0f;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                T o[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float v = r[4 * g + q] * back;
                    c.fail |= !(fabsf(v) <= margin);
                    o[q] = (T)v;
                }
                u32x2 st;
                st[0] = pack2(o[0], o[1]);
                st[1] = pack2(o[2], o[3]);
                *(u32x2 *)&c.buf[tix(i, 64 * I + 32 * fm + 8 * g + 4 * h, W)] = st;
            }
        }
        __syncthreads();
        StepL<T, I + 1>::run(c, pf);
    }
};
template <typename T> struct StepL<T, 16> {
    static __device__ __forceinline__ void prefetch(const TrsmCtx<T> &, u32x4 (&)[TRSM_PF]) {}
    static __device__ __forceinline__ void run(TrsmCtx<T> &, u32x4 (&)[TRSM_PF]) {}
};

// ---- role U, block row I: U_I = L_II^{-1} (A_I - sum_{m<I} L(I, m) U_m).
template <typename T, int I> struct StepU {
    typedef typename pmma<T>::vec vec;
    static __device__ __forceinline__ void prefetch(const TrsmCtx<T> &c, u32x4 (&pf)[TRSM_PF])
    {
        if constexpr (I >= 1 && I < 16) {
            if (I < c.nl) {
                const T *op = c.inv + OP_L + I * 16 * 4096 + (c.fm * 4 * 64 + 32 * c.h + c.l32) * 8;
#pragma unroll
                for (int s = 0; s < 2 * I; ++s) {
                    const int K = c.kh * 32 * I + 16 * s;  // block K >> 6, step (K >> 4) & 3
                    pf[s] = *(const u32x4 *)(op + (K >> 6) * 4096 + ((K >> 4) & 3) * 64 * 8);
                }
            }
        }
    }
    static __device__ __forceinline__ void run(TrsmCtx<T> &c, u32x4 (&pf)[TRSM_PF])
    {
        if (I >= c.nl) return;
        const int W = c.W, h = c.h, l32 = c.l32, fm = c.fm, fn = c.fn;
        const int cc = 32 * fn + l32;  // slab column of this lane
        T *acol = c.A + (c.k0 + 64 * I + 32 * fm) + (c.base + cc) * c.lda;
        u32x2 xa[4];
#pragma unroll
        for (int g = 0; g < 4; ++g) xa[g] = *(const u32x2 *)(acol + 8 * g + 4 * h);
        const T *iv = c.inv + (size_t)I * IH_LEAF + (fm * 4 * 64 + 32 * h + l32) * 8;
        u32x4 lh[4], ll[4];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            lh[ks] = *(const u32x4 *)(iv + IH_LHI + ks * 64 * 8);
            ll[ks] = *(const u32x4 *)(iv + IH_LLO + ks * 64 * 8);
        }
        // this wave's half of P = L(I, <I) U(<I)
        f32x16 p = zero16();
#pragma unroll
        for (int s = 0; s < 2 * I; ++s) {
            const vec bv = as_vec<T>(*(const u32x4 *)&c.buf[six(c.kh * 32 * I + 16 * s + 8 * h, cc, W)]);
            p = pmma<T>::op(as_vec<T>(pf[s]), bv, p);
        }
        StepU<T, I + 1>::prefetch(c, pf);
        join_halves(c, p);
        // Z fragment: rows 32 fm + 8 g + 4 h + q of block row I, column cc
        float z[16];
#pragma unroll
        for (int g = 0; g < 4; ++g)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                z[4 * g + q] = to_f32(from_bits<T>(xa[g][q >> 1] >> (16 * (q & 1)))) - p[4 * g + q];
        const int sz = stage_split<T>(c, z, false, I);
        __syncthreads();
        f32x16 r = zero16();
        if (c.w < 4) {
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const vec zh = as_vec<T>(*(const u32x4 *)&c.buf[six(64 * I + 16 * ks + 8 * h, cc, W)]);
                const vec zl = as_vec<T>(*(const u32x4 *)&c.stg[six(16 * ks + 8 * h, cc, PT)]);
                r = pmma<T>::op(as_vec<T>(lh[ks]), zh, r);
                r = pmma<T>::op(as_vec<T>(ll[ks]), zh, r);
                r = pmma<T>::op(as_vec<T>(lh[ks]), zl, r);
            }
        }
        __syncthreads();
        if (c.w < 4) {
            const float back = ldexpf(1.0f, -(c.ex[2 * I + 1] + sz));
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                T o[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    o[q] = (T)(r[4 * g + q] * back);
                    c.bad |= !isfinite(to_f32(o[q]));
                }
                u32x2 st;
                st[0] = pack2(o[0], o[1]);
                st[1] = pack2(o[2], o[3]);
                *(u32x2 *)&c.buf[six(64 * I + 32 * fm + 8 * g + 4 * h, cc, W)] = st;
                *(u32x2 *)(acol + 8 * g + 4 * h) = st;
            }
        }
        __syncthreads();
        StepU<T, I + 1>::run(c, pf);
    }
};
template <typename T> struct StepU<T, 16> {
    static __device__ __forceinline__ void prefetch(const TrsmCtx<T> &, u32x4 (&)[TRSM_PF]) {}
    static __device__ __forceinline__ void run(TrsmCtx<T> &, u32x4 (&)[TRSM_PF]) {}
};

template <typename T>
__global__ __launch_bounds__(TRSM_THREADS) void k_trsm(TrsmArgs a)
{
    __shared__ __attribute__((aligned(16))) T buf[PT * NB_OUT];
    __shared__ __attribute__((aligned(16))) T stg[PT * PT];
    __shared__ float pbuf[4 * 16 * 64];
    __shared__ float red[8];
    if (block_flag(&a.flags[FLAG_FAIL])) return;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int W = a.W;
    const int64_t k0 = a.k0, kend = k0 + W, lda = a.lda;
    T *A = (T *)a.A;
    TrsmCtx<T> c;
    c.k0 = k0;
    c.lda = lda;
    c.W = W;
    c.nl = W / PT;
    c.w = w;
    c.kh = w >> 2;
    c.fm = w & 1;
    c.fn = (w >> 1) & 1;
    c.h = lane >> 5;
    c.l32 = lane & 31;
    c.A = A;
    c.LT = (const T *)a.LT;
    c.inv = (const T *)a.inv;
    c.buf = buf;
    c.stg = stg;
    c.pbuf = pbuf;
    c.red = red;
    c.bad = false;
    c.fail = false;
    {
        const int *ex = (const int *)((const T *)a.inv + IH_EXP);
#pragma unroll
        for (int k = 0; k < 32; ++k) c.ex[k] = ex[k];
    }
    u32x4 pf[TRSM_PF];
    if ((int)blockIdx.x < a.nrt) {
        // ---- L rows of the tile [row0, row0 + 64)
        const int64_t row0 = kend + (int64_t)blockIdx.x * PT;
        c.base = row0;
        for (int e = t; e < W * 8; e += TRSM_THREADS) {
            const int col = e >> 3, rc = e & 7;
            const u32x4 v = *(const u32x4 *)(A + (row0 + rc * 8) + (k0 + col) * lda);
#pragma unroll
            for (int q = 0; q < 8; ++q) buf[tix(rc * 8 + q, col, W)] = from_bits<T>(v[q >> 1] >> (16 * (q & 1)));
        }
        __syncthreads();
        StepL<T, 0>::run(c, pf);
        for (int e = t; e < W * 8; e += TRSM_THREADS) {
            const int col = e >> 3, rc = e & 7;
            u32x4 v;
#pragma unroll
            for (int p = 0; p < 4; ++p)
                v[p] = pack2(buf[tix(rc * 8 + 2 * p, col, W)], buf[tix(rc * 8 + 2 * p + 1, col, W)]);
            *(u32x4 *)(A + (row0 + rc * 8) + (k0 + col) * lda) = v;
        }
        T *LT = (T *)a.LT;
        const int cpr = W / 8;
        for (int e = t; e < PT * cpr; e += TRSM_THREADS) {
            const int ii = e / cpr, cc = (e % cpr) * 8;
            *(u32x4 *)(LT + (row0 + ii) * NB_OUT + cc) = *(const u32x4 *)&buf[tix(ii, cc, W)];
        }
    } else {
        // ---- U rows of the slab [col0, col0 + 64); buf holds the slab's
        // finished U rows (column-major, W rows)
        c.base = kend + (int64_t)(blockIdx.x - a.nrt) * PT;
        StepU<T, 0>::run(c, pf);
    }
    if (c.fail) set_flag(&a.flags[FLAG_FAIL], 1);
    if (c.bad) set_flag(&a.flags[FLAG_NONFINITE], 1);
}

template <typename T>
hipError_t top_t(int64_t k0, int W, void *A, int64_t lda, void *LT, uint64_t *pub, float *inv,
                 int *flags, uint32_t tag0, hipStream_t s)
{
    TopArgs a{k0, W, A, lda, LT, pub, inv, flags, tag0};
    hipLaunchKernelGGL(k_top<T>, dim3((unsigned)(W / PT)), dim3(TOP_THREADS), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t top_gemm_t(TopGemmArgs a, hipStream_t s)
{
    const unsigned grid = (unsigned)(a.ntop + (a.M / 256) * (a.N / 256) + (a.M2 / 256) * (a.N2 / 256));
    hipLaunchKernelGGL(k_top_gemm<T>, dim3(grid), dim3(TOP_THREADS), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t trsm_t(int64_t k0, int W, int nrt, void *A, int64_t lda, void *LT, const float *inv,
                  int *flags, hipStream_t s)
{
    TrsmArgs a{k0, W, nrt, A, lda, LT, inv, flags};
    hipLaunchKernelGGL(k_trsm<T>, dim3((unsigned)(2 * nrt)), dim3(TRSM_THREADS), 0, s, a);
    return hipGetLastError();
}

}  // namespace

size_t top_pub_words() { return (size_t)PUB_LEAF * (NB_OUT / PT); }
size_t top_inv_floats() { return (size_t)IH_TOTAL * 2 / 4; }

hipError_t launch_top(int prec, int64_t k0, int W, void *A, int64_t lda, void *LT, uint64_t *pub,
                      float *inv, int *flags, uint32_t tag0, hipStream_t s)
{
    if (W < PT || W > NB_OUT || W % PT || lda % 8 || k0 % PT) return hipErrorInvalidValue;
    switch (prec) {
    case N3P_FP16: return top_t<f16>(k0, W, A, lda, LT, pub, inv, flags, tag0, s);
    case N3P_BF16: return top_t<bf16>(k0, W, A, lda, LT, pub, inv, flags, tag0, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_top_gemm(int prec, int64_t k0, int W, void *A, int64_t lda, void *LT,
                           uint64_t *pub, float *inv, int *flags, uint32_t tag0, int64_t M,
                           int64_t N, int64_t K, const void *At, int64_t ldat, const void *B,
                           int64_t ldb, void *C, int64_t ldc, int64_t M2, int64_t N2,
                           const void *At2, const void *B2, void *C2, hipStream_t s)
{
    if (W < PT || W > NB_OUT || W % PT || lda % 8 || k0 % PT) return hipErrorInvalidValue;
    if (M <= 0 || N <= 0 || M % 256 || N % 256 || K % 32 || K <= 0) return hipErrorInvalidValue;
    if (M2 < 0 || N2 < 0 || M2 % 256 || N2 % 256) return hipErrorInvalidValue;
    if (M2 == 0 || N2 == 0) M2 = N2 = 0;
    TopGemmArgs g{TopArgs{k0, W, A, lda, LT, pub, inv, flags, tag0}, W / PT, (int)M, (int)N, (int)K,
                  At, ldat, B, ldb, C, ldc, (int)M2, (int)N2, At2, B2, C2};
    switch (prec) {
    case N3P_FP16: return top_gemm_t<f16>(g, s);
    case N3P_BF16: return top_gemm_t<bf16>(g, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_trsm(int prec, int64_t Np, int64_t k0, int W, void *A, int64_t lda, void *LT,
                       const float *inv, int *flags, hipStream_t s)
{
    const int64_t rest = Np - k0 - W;
    if (rest <= 0) return hipSuccess;
    if (W < PT || W > NB_OUT || W % PT || rest % PT || lda % 8) return hipErrorInvalidValue;
    const int nrt = (int)(rest / PT);
    switch (prec) {
    case N3P_FP16: return trsm_t<f16>(k0, W, nrt, A, lda, LT, inv, flags, s);
    case N3P_BF16: return trsm_t<bf16>(k0, W, nrt, A, lda, LT, inv, flags, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace n3p
