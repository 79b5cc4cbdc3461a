// k_pivot.hip -- the explicit partial-pivoting path of the factorisation
// (Gaussian elimination with row interchanges, Section 1.3; the
// half-precision factorisation of Section 2), taken when the no-interchange
// attempt of k_getrf.hip finds that partial pivoting would interchange rows.
//
// Per 64-column leaf: k_pivot_coop (pivot search, interchanges inside the
// leaf, multipliers, ipiv) and k_gather_u12 (the leaf's interchanges on the
// rest of its outer block, and its U row block there).  Per outer block:
// k_compose_lists and k_gather_block (the block's interchanges, composed into
// one list, on all other columns),
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
// publishes it as tag-stamped 64-bit words (tag = global column + 1), written
// and polled with agent-scope atomic accesses, so no cache-wide fence is
// needed: the row index and the candidate's values in the few columns the next
// pivot depends on.  Every wavefront reads all P candidates and takes the same
// decision from the same words -- no grid-wide barrier, and one round trip
// per column, because the rank-1 update is split: columns k+1 and k+2 are
// updated as soon as column k's pivot is known, the columns right of them one
// column later, when column k's pivot row (published with its candidate and
// read ahead right after the decision) has arrived.  Per element the updates
// still come in column order, so the factors are those of the unsplit
// elimination.
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
__device__ __forceinline__ void val_words(float v, uint32_t (&p)[1]) { p[0] = __float_as_uint(v); }
__device__ __forceinline__ void val_words(double v, uint32_t (&p)[2])
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    p[0] = (uint32_t)b;
    p[1] = (uint32_t)(b >> 32);
}

template <typename CT>
__device__ __forceinline__ bool better(CT a, int ia, CT b, int ib)
{
    return a > b || (a == b && ia < ib);
}

// Cross-lane moves within 16-lane rows (DPP), and lane reads into scalars.
template <int CTRL> __device__ __forceinline__ int dpp_i(int x)
{
    return __builtin_amdgcn_update_dpp(x, x, CTRL, 0xF, 0xF, false);
}
template <int CTRL> __device__ __forceinline__ float dpp_v(float x)
{
    return __int_as_float(dpp_i<CTRL>(__float_as_int(x)));
}
template <int CTRL> __device__ __forceinline__ double dpp_v(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = dpp_i<CTRL>((int)b), hi = dpp_i<CTRL>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float lane_read(float x, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ __forceinline__ double lane_read(double x, int l)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int CTRL, typename CT> __device__ __forceinline__ void amax_step(CT &a, int &i)
{
    const CT oa = dpp_v<CTRL>(a);
    const int oi = dpp_i<CTRL>(i);
    if (better(oa, oi, a, i)) { a = oa; i = oi; }
}
// The wavefront's largest a (ties to the lowest i), in every lane: pairs
// within quads, half rows and rows by DPP, then the four rows' results.
template <typename CT> __device__ __forceinline__ void wave_argmax(CT &a, int &i)
{
    amax_step<0xB1>(a, i);   // quad_perm [1,0,3,2]
    amax_step<0x4E>(a, i);   // quad_perm [2,3,0,1]
    amax_step<0x141>(a, i);  // row_half_mirror
    amax_step<0x140>(a, i);  // row_mirror
    CT b = lane_read(a, 0);
    int j = __builtin_amdgcn_readlane(i, 0);
#pragma unroll
    for (int r = 1; r < 4; ++r) {
        const CT rb = lane_read(a, 16 * r);
        const int rj = __builtin_amdgcn_readlane(i, 16 * r);
        if (better(rb, rj, b, j)) { b = rb; j = rj; }
    }
    a = b;
    i = j;
}

// 16-byte LDS vectors of the compute type
template <typename CT> struct cvec16;
template <> struct cvec16<float> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct cvec16<double> { typedef double type __attribute__((ext_vector_type(2))); };

// 16-byte vectors of the storage types (row stores into LT)
template <typename T> struct vec16;
template <> struct vec16<f16> { typedef h8 type; };
template <> struct vec16<bf16> { typedef b8 type; };
template <> struct vec16<float> { typedef f32x4 type; };
template <> struct vec16<double> { typedef double type __attribute__((ext_vector_type(2))); };

// Exchange area (64-bit words, zeroed once per factorisation):
//   cand [2][pmax][PC_CW]  : per workgroup and column k: its candidate's row
//                            index (W words, the first used), then the
//                            candidate's values in columns k-1, k, k+1, k+2
//                            (W words each)
//   ksm  [2][PC_CW]        : row k's values in columns k-1 .. k+3
//   rows [PC_NS][pmax][64W]: the candidate rows, in column order
//   rowk [PC_NS][64W]      : row k, in column order
//   dummy [pmax][4][64W]   : per wavefront, where its idle lanes' stores go
//   then int list[16][PC_LIST_INTS]: per leaf of the outer block, the count
//   and the (dest, src) row pairs of its interchanges composed into one
//   permutation.
// Everything of column k is published together, in step k; the rows as they
// stand then, still owing column k-1's update right of column k+1, which the
// reader applies (one multiply-add per lane, the same operation the owner
// would have done).  The small words are read in the round trip that decides
// the pivot; a row is read ahead right after the decision and, if it had not
// arrived, read again in step k + 1.  Slot reuse: small words are read in the
// step that publishes them (2 slots); a row of column k is read by step
// k + 1, and its slot is written again in step k + 3, which no workgroup
// reaches before every workgroup has finished step k + 1 (3 slots).
constexpr int PC_CW = 16;
constexpr int PC_NS = 3;

// State of one thread of the panel kernel (one row, position rowi of the
// panel); step<KK>(g) is column k = 8 g + KK.  Entering step k, every row
// below the finished ones holds columns k and k+1 updated through column k-1
// and the columns right of them through column k-2: the update by column k-1
// of those columns waits for column k-1's pivot row, which arrives in step k,
// overlapped with the round trip that decides column k's pivot.
template <typename T, typename CT>
struct PcState {
    static constexpr int W = pc_cfg<CT>::W, TH = pc_cfg<CT>::TH, L = NB_LEAF;
    static_assert(pc_cfg<CT>::R == 1, "one row per thread");
    static constexpr int NWV = TH / 64;
    static constexpr int RW = TH;  // rows per workgroup
    static constexpr int NONE = 0x7fffffff;
    typedef typename cvec16<CT>::type CV;
    static constexpr int NE = 16 / sizeof(CT);
    CT v[L];
    int rowi;
    bool dead, nonfin;
    int tid, lane, wv, P, wg, m, pmax;
    int64_t c0;
    // the previous column: its pivot row, the workgroup that published it,
    // the pivot value; the words of its complete pivot row and (at the
    // wavefront holding position pp) of its row k, read ahead
    int pp, ppw;
    CT ppk, ppk2;  // pivot values of columns k-1 and k-2
    uint64_t prw[W], pkw[W];
    uint64_t *cand, *ksm, *rows, *rowk, *dummy;
    int *flags;
    CT (*red_v)[NWV];
    int (*red_i)[NWV];
    CT (*csm)[NWV][4];  // [parity][wavefront]: its candidate's values, columns k-1 .. k+2
    CT (*ksl)[8];       // [parity]: row k's values, columns k-1 .. k+3 (workgroup 0)
    CT (*prow)[L];      // [wavefront]: the previous column's pivot row, complete
    CT (*krw)[L];       // [wavefront]: the previous column's row k, complete
    CT (*crow)[L];      // [wavefront]: a row being published
    int *pivs;

    __device__ __forceinline__ bool holds(int pos) const
    {
        return pos / RW == wg && (pos % RW) / 64 == wv;
    }

    // complete the read-ahead words of one 64-value row (lane = column) of
    // column kp: poll again until every word carries `tag`; then the update by
    // column kp-1 its columns right of kp+1 were still owed when it was
    // published (with the row's own multiplier and that column's pivot row,
    // still in prow[wv]), into dst[lane]; bounded
    __device__ __forceinline__ void finish_row(const uint64_t *src, uint32_t tag, uint64_t (&w)[W], CT *dst, int kp)
    {
        auto arrived = [&]() {
            bool ok = true;
#pragma unroll
            for (int h = 0; h < W; ++h) ok &= (uint32_t)(w[h] >> 32) == tag;
            return __all(ok) != 0;
        };
        // the first check outside the loop: it waits for these words alone,
        // not for the stores issued after them
        if (!arrived() && !dead) {
            int spins = 0;
            for (;;) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > PC_SPIN_LIMIT) {
                    set_flag(&flags[FLAG_TIMEOUT], 1);
                    dead = true;
                    break;
                }
#pragma unroll
                for (int h = 0; h < W; ++h) w[h] = __hip_atomic_load(src + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (arrived() || dead) break;
            }
        }
        CT x = val_of<CT>(w);
        if (kp >= 1 && ppk2 != (CT)0) {
            const CT l = lane_read(x, kp - 1);
            if (lane >= kp + 2) x = fma(-l, prow[wv][lane], x);
        }
        dst[lane] = x;
    }
    __device__ __forceinline__ const uint64_t *row_src(int kc, int q) const
    {
        return rows + ((size_t)((kc % PC_NS) * pmax + q) * L + lane) * W;
    }
    __device__ __forceinline__ const uint64_t *rowk_src(int kc) const
    {
        return rowk + ((size_t)(kc % PC_NS) * L + lane) * W;
    }

    // the thread at position pp takes the columns of row kp (complete, src in
    // column order) that the interchange of column kp left to now: all but
    // kp .. kp+3
    __device__ __forceinline__ void take_row(const CT *src, int kp, int cb)
    {
#pragma unroll
        for (int s0 = 0; s0 < L; s0 += NE) {
            const CV x = *(const CV *)(src + ((s0 + cb) & (L - 1)));
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                const int c = (s0 + e + cb) & (L - 1);
                v[s0 + e] = (c < kp || c >= kp + 4) ? x[e] : v[s0 + e];
            }
        }
    }
    // a row into LDS in column order (one lane)
    __device__ __forceinline__ void stage_row(CT *dst, int cb) const
    {
#pragma unroll
        for (int s0 = 0; s0 < L; s0 += NE) {
            CV x;
#pragma unroll
            for (int e = 0; e < NE; ++e) x[e] = v[s0 + e];
            *(CV *)(dst + ((s0 + cb) & (L - 1))) = x;
        }
    }

    // The interchange of column kp = k - 1 completed at position pp: the
    // wavefront holding it reads row kp, and position pp takes the columns of
    // it left to now (all but kp .. kp+3).  Before anything of step k.
    __device__ __forceinline__ void complete_moved(int k, int cb)
    {
        const int kp = k - 1;
        if (pp != kp && holds(pp)) {
            finish_row(rowk_src(kp), (uint32_t)(c0 + kp + 1), pkw, krw[wv], kp);
            if (rowi == pp) take_row(krw[wv], kp, cb);
        }
    }
    // Column kp = k - 1's pivot row, complete, into prow[wv] (every
    // wavefront); position kp takes it.
    __device__ __forceinline__ void complete(int k, int cb)
    {
        const int kp = k - 1;
        finish_row(row_src(kp, ppw), (uint32_t)(c0 + kp + 1), prw, prow[wv], kp);
        if (rowi == kp) {
#pragma unroll
            for (int s0 = 0; s0 < L; s0 += NE) {
                const CV x = *(const CV *)(prow[wv] + ((s0 + cb) & (L - 1)));
#pragma unroll
                for (int e = 0; e < NE; ++e) v[s0 + e] = x[e];
            }
        }
    }

    template <int KK> __device__ __forceinline__ void step(int g)
    {
        const int k = 8 * g + KK, lim = L - 8 * g, cb = 8 * g;
        const int par = k & 1;
        const uint32_t tag = (uint32_t)(c0 + k + 1);
        constexpr int SM = (KK + L - 1) % L, S0 = KK, S1 = KK + 1, S2 = KK + 2, S3 = KK + 3;
        // the row column k-1 moved is completed first: it may be published now
        // (as a candidate, or as row k)
        if (k > 0) complete_moved(k, cb);
        // --- this workgroup's candidate
        CT best = (CT)-1;
        int bi = NONE;
        if (rowi >= k && rowi < m) {
            CT a = fabs(v[S0]);
            if (a != a) { nonfin = true; a = (CT)0; }
            best = a;
            bi = rowi;
        }
        wave_argmax(best, bi);
        if (bi != NONE && rowi == bi) {
            csm[par][wv][0] = v[SM];
            csm[par][wv][1] = v[S0];
            csm[par][wv][2] = v[S1];
            csm[par][wv][3] = v[S2];
        }
        if (wg == 0 && rowi == k) {
            ksl[par][0] = v[SM];
            ksl[par][1] = v[S0];
            ksl[par][2] = v[S1];
            ksl[par][3] = v[S2];
            ksl[par][4] = v[S3];
        }
        if (lane == 0) { red_v[par][wv] = best; red_i[par][wv] = bi; }
        __syncthreads();
        best = red_v[par][0];
        bi = red_i[par][0];
        int bwv = 0;
#pragma unroll
        for (int w = 1; w < NWV; ++w)
            if (better(red_v[par][w], red_i[par][w], best, bi)) { best = red_v[par][w]; bi = red_i[par][w]; bwv = w; }
        // --- publish.  Every wavefront issues the same stores every column
        // (lanes with nothing to publish write a private dummy slot): the wait
        // for a load issued before them then need not wait for them too (one
        // wavefront's memory operations complete in order).
        uint64_t *dmy = dummy + ((size_t)(wg * NWV + wv) * L + lane) * W;
        {
            // the candidate's small words (wavefront 0): row index, then its
            // values in columns k-1 .. k+2
            const bool real = wv == 0 && bi != NONE && lane < 5;
            uint64_t *dst = real ? cand + ((size_t)par * pmax + wg) * PC_CW + lane * W : dmy;
            uint32_t pw[W];
            val_words(csm[par][bwv][(lane >= 1 && lane < 5) ? lane - 1 : 0], pw);
            if (lane == 0) {
                pw[0] = (uint32_t)bi;
#pragma unroll
                for (int h = 1; h < W; ++h) pw[h] = 0u;
            }
#pragma unroll
            for (int h = 0; h < W; ++h) put_word(dst + h, tag, pw[h]);
        }
        {
            // row k's small words (workgroup 0)
            const bool real = wg == 0 && wv == NWV - 1 && lane < 5;
            put_val(real ? ksm + (size_t)par * PC_CW + lane * W : dmy, tag, ksl[par][lane < 5 ? lane : 4]);
        }
        // the candidate row (its wavefront) and row k (workgroup 0), complete
        // but for column k-1's update of the columns right of k+1
        if (wv == bwv && bi != NONE && rowi == bi) stage_row(crow[wv], cb);
        {
            const bool real = wv == bwv && bi != NONE;
            put_val(real ? rows + ((size_t)((k % PC_NS) * pmax + wg) * L + lane) * W : dmy, tag, crow[wv][lane]);
        }
        if (wg == 0 && wv == 0 && rowi == k) stage_row(crow[0], cb);
        {
            const bool real = wg == 0 && wv == 0;
            put_val(real ? rowk + ((size_t)(k % PC_NS) * L + lane) * W : dmy, tag, crow[wv][lane]);
        }

        // --- every wavefront: the P candidates and row k's small words.  The
        // first read is issued once column k-1 is completed, late enough for
        // the other workgroups' words to have landed, and checked after
        // column k-1's deferred update
        uint64_t cw[2][5 * W] = {}, kw[5 * W];
        auto read_small = [&]() {
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                const int q = lane + 64 * hh;
                if (q < P)
#pragma unroll
                    for (int h = 0; h < 5 * W; ++h)
                        cw[hh][h] = __hip_atomic_load(cand + ((size_t)par * pmax + q) * PC_CW + h,
                                                      __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
#pragma unroll
            for (int h = 0; h < 5 * W; ++h)
                kw[h] = __hip_atomic_load(ksm + (size_t)par * PC_CW + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        };
        auto arrived = [&]() {
            bool ok = true;
#pragma unroll
            for (int hh = 0; hh < 2; ++hh)
                if (lane + 64 * hh < P)
#pragma unroll
                    for (int h = 0; h < 5 * W; ++h) ok &= (uint32_t)(cw[hh][h] >> 32) == tag;
#pragma unroll
            for (int h = 0; h < 5 * W; ++h) ok &= (uint32_t)(kw[h] >> 32) == tag;
            return __all(ok) != 0;
        };

        // --- while they travel: column k-1 completed, and its update of the
        // columns right of k+1 (finished columns keep their values)
        if (k > 0) complete(k, cb);
        read_small();
        if (k > 0 && ppk != (CT)0 && rowi > k - 1 && rowi < m) {
            const CT l = v[SM];
#pragma unroll
            for (int s0 = (S2 / NE) * NE; s0 < L; s0 += NE) {
                const CV x = *(const CV *)(prow[wv] + ((s0 + cb) & (L - 1)));
#pragma unroll
                for (int e = 0; e < NE; ++e) {
                    const int s = s0 + e;
                    if (s >= S2) {
                        const CT u = fma(-l, x[e], v[s]);
                        v[s] = s < lim ? u : v[s];
                    }
                }
            }
        }
        if (!arrived() && !dead) {
            int spins = 0;
            for (;;) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > PC_SPIN_LIMIT) {
                    set_flag(&flags[FLAG_TIMEOUT], 1);
                    dead = true;
                    break;
                }
                read_small();
                if (arrived() || dead) break;
            }
        }
        CT cv = (CT)-1;
        int ci = NONE;
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
            if (lane + 64 * hh < P) {
                const int qi = (int)(uint32_t)cw[hh][0];
                CT qv = fabs(val_of<CT>(cw[hh] + 2 * W));
                if (qv != qv) qv = (CT)0;
                if (better(qv, qi, cv, ci)) { cv = qv; ci = qi; }
            }
        }
        wave_argmax(cv, ci);
        const int p = (!dead && ci >= k && ci < m) ? ci : k;
        const int pwg = p / RW;
        // read ahead: the complete pivot row, and (holding position p) row k
        const bool hold = p != k && holds(p);
#pragma unroll
        for (int h = 0; h < W; ++h) prw[h] = __hip_atomic_load(row_src(k, pwg) + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (hold)
#pragma unroll
            for (int h = 0; h < W; ++h) pkw[h] = __hip_atomic_load(rowk_src(k) + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // the pivot row's values in columns k-1 .. k+2, from the lane that read them
        CT pv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const CT a = val_of<CT>(cw[0] + W + j * W), b = val_of<CT>(cw[1] + W + j * W);
            pv[j] = lane_read(pwg >= 64 ? b : a, pwg & 63);
        }
        const CT pk = pv[1];
        CT pw1 = pv[2], pw2 = pv[3];
        const bool fix = k > 0 && ppk != (CT)0;  // column k-1's update still owed
        if (fix && k + 2 < L) pw2 = fma(-pv[0], prow[wv][k + 2], pw2);
        if (wg == 0 && tid == 0) pivs[k] = p;
        if (pk == (CT)0 && wg == 0 && tid == 0) atomicCAS(&flags[FLAG_ZEROPIV], 0, (int)(c0 + k + 1));
        // --- the interchange: position p takes row k's columns k .. k+3 (the
        // rest of row k follows in step k+1; position k takes the pivot row then)
        if (p != k && rowi == p) {
            CT r[5];
#pragma unroll
            for (int j = 0; j < 5; ++j) r[j] = val_of<CT>(kw + j * W);
            if (fix && k + 2 < L) r[3] = fma(-r[0], prow[wv][k + 2], r[3]);
            if (fix && k + 3 < L) r[4] = fma(-r[0], prow[wv][k + 3], r[4]);
            v[S0] = r[1];
            if (S1 < lim) v[S1] = r[2];
            if (S2 < lim) v[S2] = r[3];
            if (S3 < lim) v[S3] = r[4];
        }
        // --- the multiplier, and the update of columns k+1 and k+2
        if (pk != (CT)0 && rowi > k && rowi < m) {
            const CT l = v[S0] / pk;
            v[S0] = l;
            if (S1 < lim) v[S1] = fma(-l, pw1, v[S1]);
            if (S2 < lim) v[S2] = fma(-l, pw2, v[S2]);
        }
        pp = p;
        ppw = pwg;
        ppk2 = ppk;
        ppk = pk;
    }

    // rotate by 8 slots: the next group's columns move to slots 0..7
    __device__ __forceinline__ void rotate()
    {
        CT t8[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) t8[q] = v[q];
#pragma unroll
        for (int s = 0; s < L - 8; ++s) v[s] = v[s + 8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[L - 8 + q] = t8[q];
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
    constexpr int W = S::W, L = NB_LEAF, RW = S::RW, NWV = S::NWV;
    __shared__ CT red_v[2][NWV];
    __shared__ int red_i[2][NWV];
    __shared__ CT csm[2][NWV][4];
    __shared__ CT ksl[2][8];
    __shared__ __attribute__((aligned(16))) CT prow[NWV][L];
    __shared__ __attribute__((aligned(16))) CT krw[NWV][L];
    __shared__ __attribute__((aligned(16))) CT crow[NWV][L];
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
    st.pp = -1;
    st.ppw = 0;
    st.ppk = (CT)0;
    st.ppk2 = (CT)0;
    st.cand = xch;
    st.ksm = xch + (size_t)2 * pmax * PC_CW;
    st.rows = st.ksm + 2 * PC_CW;
    st.rowk = st.rows + (size_t)PC_NS * pmax * L * W;
    st.dummy = st.rowk + (size_t)PC_NS * L * W;
    st.flags = flags;
    st.red_v = red_v;
    st.red_i = red_i;
    st.csm = csm;
    st.ksl = ksl;
    st.prow = prow;
    st.krw = krw;
    st.crow = crow;
    st.pivs = pivs;
    st.dead = false;
    st.nonfin = false;
    int *list = (int *)(st.dummy + (size_t)pmax * NWV * L * W) + ((c0 - k0) / L) * PC_LIST_INTS;
    const int tid = st.tid, lane = st.lane, wv = st.wv, wg = st.wg, m = st.m;

    st.rowi = wg * RW + tid;
#pragma unroll
    for (int j = 0; j < L; ++j) st.v[j] = (CT)0;
    if (st.rowi < m) {
        const T *src = A + (c0 + st.rowi) + c0 * lda;
#pragma unroll
        for (int j = 0; j < L; ++j) st.v[j] = (CT)to_f32(src[j * lda]);
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
    // the last column's moved row and pivot row (slots back in column order)
    st.complete_moved(L, 0);
    st.complete(L, 0);
    if (st.nonfin) set_flag(&flags[FLAG_NONFINITE], 1);

    // --- the factored panel into A; rows below the leaf also into LT (K contiguous)
    typedef typename vec16<T>::type V16;
    constexpr int VE = 16 / sizeof(T);
    bool bad = false;
    if (st.rowi < m) {
        T *dst = A + (c0 + st.rowi) + c0 * lda;
        T *lt = LT + (c0 + st.rowi) * (int64_t)NB_OUT + (c0 - k0);
        const bool below = st.rowi >= L;
#pragma unroll
        for (int q = 0; q < L / VE; ++q) {
            V16 pk16;
#pragma unroll
            for (int e = 0; e < VE; ++e) {
                const T x = to_store_d<T>((double)st.v[q * VE + e]);
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

// The interchange lists of an outer block's leaves (0 .. nl-1, applied in
// order) composed into one list of (dest, src) row moves.  LDS holds, for each
// row position >= k0, the offset of the row whose values end there; the lists
// are applied to it in order (every read of a list before any write), and the
// positions whose row changed make the list.  At most the block's rows and as
// many rows from below change (each leaf moves at most 64 rows up).  One
// workgroup; the order of the composed list is immaterial.
constexpr int PC_CMAX = 2 * NB_OUT;
constexpr int PC_COMP_INTS = 1 + 2 * PC_CMAX;
__global__ __launch_bounds__(1024) void k_compose_lists(const int *__restrict__ lists, int nl, int64_t k0,
                                                        int64_t Np, int *__restrict__ out)
{
    __shared__ unsigned short src_of[PIVOT_MAX_NP];
    __shared__ int cnt;
    const int t = threadIdx.x;
    const int n = (int)(Np - k0);
    for (int i = t; i < n; i += 1024) src_of[i] = (unsigned short)i;
    if (t == 0) cnt = 0;
    __syncthreads();
    for (int l = 0; l < nl; ++l) {
        const int *list = lists + l * PC_LIST_INTS;
        const int c = list[0];
        int d = 0;
        unsigned short v = 0;
        if (t < c) {
            d = list[1 + 2 * t] - (int)k0;
            v = src_of[list[2 + 2 * t] - (int)k0];
        }
        __syncthreads();
        if (t < c) src_of[d] = v;
        __syncthreads();
    }
    for (int i = t; i < n; i += 1024) {
        if (src_of[i] != i) {
            const int e = atomicAdd(&cnt, 1);
            if (e < PC_CMAX) {
                out[1 + 2 * e] = (int)k0 + i;
                out[2 + 2 * e] = (int)k0 + src_of[i];
            }
        }
    }
    __syncthreads();
    if (t == 0) out[0] = min(cnt, PC_CMAX);
}

// The composed interchanges of an outer block on the columns outside it,
// [0, k0) and [kend, Np): four columns per 256-thread workgroup, every read
// before any write.
template <typename T>
__global__ __launch_bounds__(256) void k_gather_block(T *__restrict__ A, int64_t lda,
                                                      const int *__restrict__ comp, int64_t k0,
                                                      int64_t kend, int64_t ncol)
{
    constexpr int PER = PC_CMAX / 256, NC = 4;
    const int t = threadIdx.x;
    const int c = comp[0];
    T *cp[NC];
    bool colok[NC];
#pragma unroll
    for (int j = 0; j < NC; ++j) {
        const int64_t q = (int64_t)blockIdx.x * NC + j;
        colok[j] = q < ncol;
        cp[j] = A + (q < k0 ? q : q - k0 + kend) * lda;
    }
    int d[PER];
    T x[PER][NC];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int e = t + 256 * i;
        d[i] = -1;
        if (e < c) {
            d[i] = comp[1 + 2 * e];
            const int sr = comp[2 + 2 * e];
#pragma unroll
            for (int j = 0; j < NC; ++j)
                if (colok[j]) x[i][j] = cp[j][sr];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i)
        if (d[i] >= 0)
#pragma unroll
            for (int j = 0; j < NC; ++j)
                if (colok[j]) cp[j][d[i]] = x[i][j];
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
    const int64_t nwv = pc_cfg<float>::TH / 64;
    return 2 * pmax * PC_CW + 2 * PC_CW + PC_NS * pmax * NB_LEAF * W + PC_NS * NB_LEAF * W +
           pmax * nwv * NB_LEAF * W;
}

size_t pivot_xch_bytes(int prec, int64_t Np)
{
    return (size_t)pc_words(prec, Np) * 8 + ((size_t)PC_NLIST * PC_LIST_INTS + PC_COMP_INTS) * 4;
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
    if (nl > PC_NLIST || Np > PIVOT_MAX_NP) return hipErrorInvalidValue;
    if (ncol <= 0 || nl <= 0) return hipSuccess;
    const int *lists = pc_lists(prec, Np, xch);
    int *comp = (int *)lists + PC_NLIST * PC_LIST_INTS;
    hipLaunchKernelGGL(k_compose_lists, dim3(1), dim3(1024), 0, s, lists, nl, k0, Np, comp);
    const unsigned grid = (unsigned)((ncol + 3) / 4);
    switch (prec) {
    case N3P_FP16: hipLaunchKernelGGL(k_gather_block<f16>, dim3(grid), dim3(256), 0, s, (f16 *)A, lda, comp, k0, kend, ncol); break;
    case N3P_BF16: hipLaunchKernelGGL(k_gather_block<bf16>, dim3(grid), dim3(256), 0, s, (bf16 *)A, lda, comp, k0, kend, ncol); break;
    case N3P_FP32: hipLaunchKernelGGL(k_gather_block<float>, dim3(grid), dim3(256), 0, s, (float *)A, lda, comp, k0, kend, ncol); break;
    case N3P_FP64: hipLaunchKernelGGL(k_gather_block<double>, dim3(grid), dim3(256), 0, s, (double *)A, lda, comp, k0, kend, ncol); break;
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
