// k_pivot.hip -- the explicit partial-pivoting path of the factorisation
// (Gaussian elimination with row interchanges, Section 1.3; the
// half-precision factorisation of Section 2), taken when the no-interchange
// attempt of k_getrf.hip finds that partial pivoting would interchange rows.
//
// Per 64-column leaf: k_pivot_coop (pivot search, interchanges inside the
// leaf, multipliers, ipiv) and k_gather_u12 (the leaf's interchanges on the
// rest of its outer block, and its U row block there).  Per outer block:
// k_gather_block (the block's interchanges on all other columns),
// k_lt_rebuild (the block's L transposed), k_u12 (U row blocks right of the
// block).  The Schur-complement updates reuse the matrix-core GEMMs of
// k_getrf.hip.
#include <algorithm>

#include "n3p_internal.hpp"

namespace n3p {

// Partial pivoting (largest magnitude, ties to the lowest row) of one 64-column
// leaf over rows [c0, Np), spread over P workgroups that each hold a
// contiguous block of rows in registers (FP32 arithmetic, FP64 for FP64
// storage).  Per column every workgroup reduces its own candidate and
// publishes it -- row index, magnitude and the whole 64-value row -- as
// tag-stamped 64-bit words (tag = global column + 1), written and polled with
// agent-scope atomic accesses, so no cache-wide fence is needed.  Every
// workgroup then reads all P candidates and takes the same decision from the
// same words: no grid-wide barrier, one round trip for the candidates and one
// for the winning row per column.  One wavefront per workgroup polls and
// passes the result on through LDS.  Slots alternate with the column parity; a
// workgroup publishes column k + 2 only after every workgroup has published
// column k + 1, which each does only after it has finished reading column k.
//
// P <= PIVOT_MAX_WG workgroups of 256 threads, one row per thread (256 rows
// per workgroup), fill one CU each on an otherwise idle device, so all are
// resident together; this bounds the pivoting path to Np <= 128 * 256 = 32768
// rows (the host checks it before the first launch).  Every wait is bounded regardless: an
// expired wait raises FLAG_TIMEOUT and the wavefront stops waiting, so the grid
// always drains (the factors are then invalid and the caller reports the
// timeout).
//
// Columns are processed in 8 groups of 8.  The register row is rotated by 8
// slots after each group, so the current group's columns always sit in slots
// 0..7 (compile-time register indices): in group g, slot s holds panel column
// (s + 8 g) mod 64 and slots >= 64 - 8 g hold finished columns.
constexpr int PC_SPIN_LIMIT = 1 << 20;         // polls of ~1 us: a wait that long has failed
constexpr int PC_LIST_INTS = 1 + 4 * NB_LEAF;  // count + 128 (dest, src) pairs
constexpr int PC_NLIST = NB_OUT / NB_LEAF;     // one list per leaf of an outer block

template <typename CT> struct pc_cfg;
// rows per thread, words per value, threads per workgroup
template <> struct pc_cfg<float> { static constexpr int R = 1, W = 1, TH = 256; };
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
//   then int list[16][PC_LIST_INTS]: per leaf of the outer block, the count
//   and the (dest, src) row pairs of its interchanges composed into one
//   permutation.
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
    CT (*prow_l)[L];     // [parity]: the pivot row, as read by wavefront 0
    CT (*krow_x)[L];     // [parity]: row k, as read by wavefront 0 (workgroup holding p)
    int *pl;             // [parity]: the pivot row index
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
        // --- wavefront 0: the pivot row p from all P (<= 128) candidates, then
        // the winning row and row k in one round trip; shared through LDS
        if (wv == 0) {
            int p = k;
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
            const int pw = p / RW;  // workgroup holding row p
            const bool need_k = p != k && pw == wg;
            uint64_t w[2 * W];
            const uint64_t *src = rows + ((size_t)par * pmax + pw) * L * W + lane * W;
            const uint64_t *srck = rowk + (size_t)par * L * W + lane * W;
            int spins = 0;
            for (;;) {
                bool ok = true;
#pragma unroll
                for (int h = 0; h < W; ++h) {
                    w[h] = __hip_atomic_load(src + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok &= (uint32_t)(w[h] >> 32) == tag;
                    if (need_k) {
                        w[W + h] = __hip_atomic_load(srck + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        ok &= (uint32_t)(w[W + h] >> 32) == tag;
                    }
                }
                if (__all(ok) || dead) break;
                __builtin_amdgcn_s_sleep(1);
                if (++spins > PC_SPIN_LIMIT) {
                    set_flag(&flags[FLAG_TIMEOUT], 1);
                    dead = true;
                    break;
                }
            }
            prow_l[par][lane] = val_of<CT>(w);
            if (need_k) krow_x[par][lane] = val_of<CT>(w + W);
            if (lane == 0) pl[par] = p;
        }
        __syncthreads();
        const int p = pl[par];
        const int pw = p / RW;
        const bool holds_p = p != k && pw == wg && ((p - pw * RW) % TH) / 64 == wv;
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
                const CT ps = prow_l[par][s];
                const CT ks = holds_p ? krow_x[par][s] : (CT)0;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (isk[r]) v[r][s] = ps;
                    if (isp[r]) v[r][s] = ks;
                }
            }
        }
        // --- multipliers and the rank-1 update of the unfinished columns
        const CT pk = prow_l[par][KK];
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
                const CT ps = prow_l[par][s];
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
    __shared__ CT prow_l[2][L];
    __shared__ CT krow_x[2][L];
    __shared__ int pl[2];
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
    st.prow_l = prow_l;
    st.krow_x = krow_x;
    st.pl = pl;
    st.pivs = pivs;
    st.dead = false;
    st.nonfin = false;
    int *list = (int *)(st.rowk + 2 * L * W) + ((c0 - k0) / L) * PC_LIST_INTS;
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

// Interchanges of an outer block's leaves (lists 0 .. nl-1, applied in order)
// on the columns outside the block, [0, k0) and [kend, Np).  Two columns per
// 256-thread workgroup, one row move per thread; every read of a list
// completes before any write.
template <typename T>
__global__ __launch_bounds__(256) void k_gather_block(T *__restrict__ A, int64_t lda,
                                                      const int *__restrict__ lists, int nl,
                                                      int64_t k0, int64_t kend, int64_t ncol)
{
    const int64_t q = (int64_t)blockIdx.x * 2 + (threadIdx.x >> 7);
    const int e = threadIdx.x & 127;
    const bool colok = q < ncol;
    T *cp = A + (q < k0 ? q : q - k0 + kend) * lda;
    for (int l = 0; l < nl; ++l) {
        const int *list = lists + l * PC_LIST_INTS;
        const bool act = colok && e < list[0];
        T x = (T)0.0f;
        if (act) x = cp[list[2 + 2 * e]];
        __syncthreads();
        if (act) cp[list[1 + 2 * e]] = x;
        __syncthreads();
    }
}

// Forward substitution of one column's 64 rows [c0, c0 + 64) with the unit
// lower L11 (in LDS): lane = row, the solved entries broadcast by readlane.
template <typename T, typename CT>
__device__ __forceinline__ void u12_column(T *__restrict__ cp, const CT (*Lm)[NB_LEAF + 1], int lane,
                                           int *__restrict__ flags)
{
    constexpr int L = NB_LEAF;
    CT lrow[L];
#pragma unroll
    for (int k = 0; k < L; ++k) lrow[k] = Lm[lane][k];
    CT y = (CT)to_f32(cp[lane]);
#pragma unroll
    for (int k = 0; k < L - 1; ++k) {
        const CT yk = lane_bcast(y, k);
        if (lane > k) y -= lrow[k] * yk;
    }
    const T v = to_store_d<T>((double)y);
    if (!isfinite(to_f32(v))) set_flag(&flags[FLAG_NONFINITE], 1);  // the stored value
    cp[lane] = v;
}

template <typename T, typename CT>
__device__ __forceinline__ void load_l11(const T *__restrict__ A, int64_t lda, int64_t c0,
                                         CT (*Lm)[NB_LEAF + 1])
{
    for (int i = threadIdx.x; i < NB_LEAF * NB_LEAF; i += blockDim.x) {
        const int r = i % NB_LEAF, j = i / NB_LEAF;
        Lm[r][j] = (CT)to_f32(A[(c0 + r) + (c0 + j) * lda]);
    }
}

// The leaf's interchanges on the other columns of its outer block [k0, kend),
// and the leaf's U row block there: columns right of the leaf get the
// interchanges and then the substitution with the leaf's L11; columns left
// of it only the interchanges.  Four columns per 256-thread workgroup: the
// row moves of all four first (every read before any write), then one
// wavefront per column.
template <typename T>
__global__ __launch_bounds__(256) void k_gather_u12(T *__restrict__ A, int64_t lda,
                                                    const int *__restrict__ list, int64_t c0,
                                                    int64_t k0, int64_t kend,
                                                    int *__restrict__ flags)
{
    typedef typename compute_of<T>::type CT;
    constexpr int L = NB_LEAF;
    __shared__ CT Lm[L][L + 1];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int64_t ncol = kend - k0 - L, left = c0 - k0;
    const int64_t q0 = (int64_t)blockIdx.x * 4;
    const int n = list[0];
    T x[2];
    bool act[2];
    T *cp[2];
    int dst[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int item = t + 256 * h, e = item & 127;
        const int64_t q = q0 + (item >> 7);
        act[h] = q < ncol && e < n;
        cp[h] = A + (q < left ? k0 + q : k0 + q + L) * lda;
        x[h] = (T)0.0f;
        dst[h] = 0;
        if (act[h]) {
            x[h] = cp[h][list[2 + 2 * e]];
            dst[h] = list[1 + 2 * e];
        }
    }
    load_l11<T, CT>(A, lda, c0, Lm);
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h)
        if (act[h]) cp[h][dst[h]] = x[h];
    __syncthreads();
    const int64_t q = q0 + wv;
    if (q < ncol && q >= left) u12_column<T, CT>(A + (k0 + q + L) * lda + c0, Lm, lane, flags);
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
// with the unit lower L11 taken from A; one wavefront per column.
template <typename T>
__global__ __launch_bounds__(256) void k_u12(int64_t col0, int64_t col1, int64_t c0,
                                             T *__restrict__ A, int64_t lda,
                                             int *__restrict__ flags)
{
    typedef typename compute_of<T>::type CT;
    __shared__ CT Lm[NB_LEAF][NB_LEAF + 1];
    load_l11<T, CT>(A, lda, c0, Lm);
    __syncthreads();
    const int64_t jc = col0 + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (jc < col1) u12_column<T, CT>(A + jc * lda + c0, Lm, threadIdx.x & 63, flags);
}

// ================================================================ launchers
static int pc_rows_per_wg(int prec)
{
    return prec == N3P_FP64 ? pc_cfg<double>::TH * pc_cfg<double>::R
                            : pc_cfg<float>::TH * pc_cfg<float>::R;
}

static int64_t pc_pmax(int prec, int64_t Np)
{
    return (Np + pc_rows_per_wg(prec) - 1) / pc_rows_per_wg(prec);
}

static int64_t pc_words(int prec, int64_t Np)
{
    const int64_t pmax = pc_pmax(prec, Np), W = prec == N3P_FP64 ? 2 : 1;
    return 8 * pmax + 2 * pmax * NB_LEAF * W + 2 * NB_LEAF * W;
}

size_t pivot_xch_bytes(int prec, int64_t Np)
{
    return (size_t)pc_words(prec, Np) * 8 + (size_t)PC_NLIST * PC_LIST_INTS * 4;
}

static const int *pc_lists(int prec, int64_t Np, const void *xch)
{
    return (const int *)((const uint64_t *)xch + pc_words(prec, Np));
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
    if (m < NB_LEAF || m % NB_LEAF || P > PIVOT_MAX_WG) return hipErrorInvalidValue;
    switch (prec) {
    case N3P_FP16: return pivot_coop_t<f16, float>(Np, c0, k0, A, lda, ipiv, LT, xch, (int)pmax, (int)P, flags, s);
    case N3P_BF16: return pivot_coop_t<bf16, float>(Np, c0, k0, A, lda, ipiv, LT, xch, (int)pmax, (int)P, flags, s);
    case N3P_FP32: return pivot_coop_t<float, float>(Np, c0, k0, A, lda, ipiv, LT, xch, (int)pmax, (int)P, flags, s);
    case N3P_FP64: return pivot_coop_t<double, double>(Np, c0, k0, A, lda, ipiv, LT, xch, (int)pmax, (int)P, flags, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_gather_u12(int prec, int64_t Np, int64_t c0, int64_t k0, int64_t kend, void *A,
                             int64_t lda, const void *xch, int *flags, hipStream_t s)
{
    const int64_t ncol = kend - k0 - NB_LEAF;
    if (ncol <= 0) return hipSuccess;
    const int *list = pc_lists(prec, Np, xch) + ((c0 - k0) / NB_LEAF) * PC_LIST_INTS;
    const unsigned grid = (unsigned)((ncol + 3) / 4);
    switch (prec) {
    case N3P_FP16: hipLaunchKernelGGL(k_gather_u12<f16>, dim3(grid), dim3(256), 0, s, (f16 *)A, lda, list, c0, k0, kend, flags); break;
    case N3P_BF16: hipLaunchKernelGGL(k_gather_u12<bf16>, dim3(grid), dim3(256), 0, s, (bf16 *)A, lda, list, c0, k0, kend, flags); break;
    case N3P_FP32: hipLaunchKernelGGL(k_gather_u12<float>, dim3(grid), dim3(256), 0, s, (float *)A, lda, list, c0, k0, kend, flags); break;
    case N3P_FP64: hipLaunchKernelGGL(k_gather_u12<double>, dim3(grid), dim3(256), 0, s, (double *)A, lda, list, c0, k0, kend, flags); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_gather_block(int prec, int64_t Np, int64_t k0, int64_t kend, void *A,
                               int64_t lda, const void *xch, hipStream_t s)
{
    const int64_t ncol = k0 + (Np - kend);
    const int nl = (int)((kend - k0) / NB_LEAF);
    if (ncol <= 0 || nl <= 0 || nl > PC_NLIST) return nl > PC_NLIST ? hipErrorInvalidValue : hipSuccess;
    const int *lists = pc_lists(prec, Np, xch);
    const unsigned grid = (unsigned)((ncol + 1) / 2);
    switch (prec) {
    case N3P_FP16: hipLaunchKernelGGL(k_gather_block<f16>, dim3(grid), dim3(256), 0, s, (f16 *)A, lda, lists, nl, k0, kend, ncol); break;
    case N3P_BF16: hipLaunchKernelGGL(k_gather_block<bf16>, dim3(grid), dim3(256), 0, s, (bf16 *)A, lda, lists, nl, k0, kend, ncol); break;
    case N3P_FP32: hipLaunchKernelGGL(k_gather_block<float>, dim3(grid), dim3(256), 0, s, (float *)A, lda, lists, nl, k0, kend, ncol); break;
    case N3P_FP64: hipLaunchKernelGGL(k_gather_block<double>, dim3(grid), dim3(256), 0, s, (double *)A, lda, lists, nl, k0, kend, ncol); break;
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
    const unsigned grid = (unsigned)((ncol + 3) / 4);
    switch (prec) {
    case N3P_FP16: hipLaunchKernelGGL(k_u12<f16>, dim3(grid), dim3(256), 0, s, col0, col1, c0, (f16 *)A, lda, flags); break;
    case N3P_BF16: hipLaunchKernelGGL(k_u12<bf16>, dim3(grid), dim3(256), 0, s, col0, col1, c0, (bf16 *)A, lda, flags); break;
    case N3P_FP32: hipLaunchKernelGGL(k_u12<float>, dim3(grid), dim3(256), 0, s, col0, col1, c0, (float *)A, lda, flags); break;
    case N3P_FP64: hipLaunchKernelGGL(k_u12<double>, dim3(grid), dim3(256), 0, s, col0, col1, c0, (double *)A, lda, flags); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace n3p
