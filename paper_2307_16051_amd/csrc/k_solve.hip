// k_solve.hip -- the preconditioner-vector product U^{-1} L^{-1} P r
// (Section 2.2) and the single-precision residual r = b - A u.
//
// Triangular solves: one persistent launch per solve.  Row blocks of BS rows
// are taken in dependency order through an atomic ticket (a block only waits
// on blocks with smaller tickets, which are already running, so the waits
// always end).  Block i inverts its diagonal block and premultiplies the
// tile of its nearest predecessor by that inverse while the chain is still
// far away, accumulates the contributions of the other finished blocks as
// they are published, and once its nearest predecessor publishes, finishes
// with one BS x BS product and publishes its piece of the solution as words
// stamped with the launch's epoch (no flag reset between launches).  Factors are read in their
// storage precision and promoted in registers (interprecision transfer on
// the fly, Section 2.3).  Every wait is bounded; an expired wait raises
// FLAG_TIMEOUT and the block proceeds so that the grid always drains.
#include <algorithm>
#include <mutex>

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

// Solution values are published as 64-bit words (epoch << 32 | 32 bits of
// data): FP32 values take one word, FP64 values two.  A reader polls the words
// it needs until their tag equals the launch's epoch, so the value arrives in
// the same memory round trip as its readiness (no separate flag), and no
// cache-wide fence is needed: the words are written and read with
// agent-scope (coherent) atomic accesses.
template <typename V> struct tagged;
template <> struct tagged<float> {
    static constexpr int W = 1;
    static __device__ __forceinline__ void put(uint64_t *t, int64_t i, float v, uint32_t ep)
    {
        const uint64_t w = ((uint64_t)ep << 32) | (uint32_t)__float_as_uint(v);
        __hip_atomic_store(&t[i], w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    static __device__ __forceinline__ float get(const uint64_t *t, int64_t i, uint32_t ep, int *spins,
                                                int *flags)
    {
        uint64_t w = __hip_atomic_load(&t[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        while ((uint32_t)(w >> 32) != ep) {
            __builtin_amdgcn_s_sleep(1);
            if (++*spins > SPIN_LIMIT) { set_flag(&flags[FLAG_TIMEOUT], 1); break; }
            w = __hip_atomic_load(&t[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        return __uint_as_float((uint32_t)w);
    }
};
template <> struct tagged<double> {
    static constexpr int W = 2;
    static __device__ __forceinline__ void put(uint64_t *t, int64_t i, double v, uint32_t ep)
    {
        const uint64_t b = (uint64_t)__double_as_longlong(v);
        __hip_atomic_store(&t[2 * i], ((uint64_t)ep << 32) | (b & 0xffffffffULL), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&t[2 * i + 1], ((uint64_t)ep << 32) | (b >> 32), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    static __device__ __forceinline__ double get(const uint64_t *t, int64_t i, uint32_t ep, int *spins,
                                                 int *flags)
    {
        uint32_t part[2];
        for (int h = 0; h < 2; ++h) {
            uint64_t w = __hip_atomic_load(&t[2 * i + h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            while ((uint32_t)(w >> 32) != ep) {
                __builtin_amdgcn_s_sleep(1);
                if (++*spins > SPIN_LIMIT) { set_flag(&flags[FLAG_TIMEOUT], 1); break; }
                w = __hip_atomic_load(&t[2 * i + h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            part[h] = (uint32_t)w;
        }
        return __longlong_as_double((long long)(((uint64_t)part[1] << 32) | part[0]));
    }
};

// sync layout: int ticket at [0]; tagged words (uint64) from byte offset 16
__device__ __forceinline__ uint64_t *tag_words(int *sync) { return (uint64_t *)(sync + 4); }

// One published value per lane: lane c of a wavefront fetches the word(s) of
// column c of a tile, re-polls until every lane's tag matches, and then the
// values are broadcast lane by lane (v_readlane) into the row updates.
template <typename V>
struct lane_word {
    uint64_t w[tagged<V>::W];
    __device__ __forceinline__ void issue(const uint64_t *t, int64_t idx, bool valid)
    {
#pragma unroll
        for (int h = 0; h < tagged<V>::W; ++h)
            w[h] = valid ? __hip_atomic_load(&t[idx * tagged<V>::W + h], __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT)
                         : 0;
    }
    // backoff: extra sleep between polls, in units of 256 cycles.  A block
    // waiting for a tile far behind its own row block has time to spare, and
    // every poll of the newest words competes with the poll of the block
    // that needs them next, so far blocks poll rarely.
    __device__ __forceinline__ void settle(const uint64_t *t, int64_t idx, bool valid, uint32_t ep,
                                           int *spins, int *flags, int backoff = 0)
    {
        for (;;) {
            if (ready(valid, ep)) return;
            __builtin_amdgcn_s_sleep(1);
            for (int k = 0; k < backoff; ++k) __builtin_amdgcn_s_sleep(4);
            *spins += backoff > 0 ? backoff : 0;  // the bound counts sleeps, not polls
            if (++*spins > SPIN_LIMIT) {
                set_flag(&flags[FLAG_TIMEOUT], 1);
                return;
            }
            bool ok = true;
            if (valid) {
#pragma unroll
                for (int h = 0; h < tagged<V>::W; ++h) ok &= (uint32_t)(w[h] >> 32) == ep;
            }
            if (!ok) issue(t, idx, valid);
        }
    }
    __device__ __forceinline__ bool ready(bool valid, uint32_t ep) const
    {
        bool ok = true;
        if (valid) {
#pragma unroll
            for (int h = 0; h < tagged<V>::W; ++h) ok &= (uint32_t)(w[h] >> 32) == ep;
        }
        return __all(ok);
    }
    // The wait on the last hand-off before a block can finish.  settle()
    // re-polls only after its previous poll has returned, so a value that
    // lands just after a poll passed is seen almost two memory round trips
    // later.  Here, once the first poll (*this, already issued) has missed,
    // four polls are kept in flight, issued a quarter of a round trip apart:
    // the value is seen about one trip after it lands.  Straight-line code (fully
    // unrolled), so each check waits for its own poll only; after RING
    // rounds it falls back to settle().
    template <int RING>
    __device__ __forceinline__ void settle_ring(const uint64_t *t, int64_t idx, bool valid,
                                                uint32_t ep, int *spins, int *flags)
    {
        if (ready(valid, ep)) return;
        issue(t, idx, valid);
        lane_word b, c, d;
        __builtin_amdgcn_s_sleep(9);
        b.issue(t, idx, valid);
        __builtin_amdgcn_s_sleep(9);
        c.issue(t, idx, valid);
        __builtin_amdgcn_s_sleep(9);
        d.issue(t, idx, valid);
#pragma unroll
        for (int r = 0; r < RING; ++r) {
            if (ready(valid, ep)) return;
            issue(t, idx, valid);
            if (b.ready(valid, ep)) { *this = b; return; }
            b.issue(t, idx, valid);
            if (c.ready(valid, ep)) { *this = c; return; }
            c.issue(t, idx, valid);
            if (d.ready(valid, ep)) { *this = d; return; }
            d.issue(t, idx, valid);
        }
        *spins += 4 * RING;
        settle(t, idx, valid, ep, spins, flags);
    }
    __device__ __forceinline__ V value() const
    {
        if constexpr (tagged<V>::W == 1) {
            return __uint_as_float((uint32_t)w[0]);
        } else {
            const uint64_t lo = (uint32_t)w[0], hi = (uint32_t)w[1];
            return __longlong_as_double((long long)((hi << 32) | lo));
        }
    }
};

template <typename T, typename V, int BS>
__device__ __forceinline__ void load_tile_row(V (&fv)[BS], const T *__restrict__ LU, int64_t lda,
                                              int64_t rowc, int64_t c0, int64_t n)
{
    // unconditional loads (column index clamped in bounds) so that all BS
    // loads issue back to back; entries past column n-1 are zeroed after
    T raw[BS];
#pragma unroll
    for (int c = 0; c < BS; ++c) raw[c] = LU[rowc + std::min<int64_t>(c0 + c, n - 1) * lda];
#pragma unroll
    for (int c = 0; c < BS; ++c) fv[c] = c0 + c < n ? (V)to_f32(raw[c]) : (V)0;
}

// Diagonal-block helpers.  Each block inverts its own BS x BS diagonal block
// D (held row-major, stride BS, in Dr) and forms Mx = D^{-1} E, with E the
// neighbouring off-diagonal tile it depends on last (stride BS, in Eb).  Then
// only one product with the neighbour's solution is left after it arrives:
// lower x_b = D^{-1} (b_b - sum_{j<b-1} L_bj x_j) - D^{-1} L_{b,b-1} x_{b-1},
// upper x_b = D^{-1} (y_b - sum_{j>b+1} U_bj x_j) - D^{-1} U_{b,b+1} x_{b+1}.
// (Rounding differs from substitution only in the order of the sums.)
//
// Inverse of the diagonal block, wavefront 0, lane c = column c of the
// inverse (LOWER: unit lower; else upper with reciprocals rd of its
// diagonal).  Dr entries on or beyond the diagonal's wrong side are ignored.
template <typename V, int BS, bool LOWER>
__device__ __forceinline__ void diag_inverse(const V *__restrict__ Dr, const V *__restrict__ rd,
                                             V *__restrict__ Di, int lane)
{
    // each row's sum in four interleaved partial sums, so the dependent
    // chain is about a quarter as long
    V xi[BS];
    if constexpr (LOWER) {
#pragma unroll
        for (int i = 0; i < BS; ++i) {
            V a[4] = {lane == i ? (V)1 : (V)0, 0, 0, 0};
#pragma unroll
            for (int k = 0; k < i; ++k) a[k & 3] -= Dr[i * BS + k] * xi[k];
            xi[i] = (a[0] + a[1]) + (a[2] + a[3]);
        }
    } else {
#pragma unroll
        for (int i = BS - 1; i >= 0; --i) {
            V a[4] = {lane == i ? (V)1 : (V)0, 0, 0, 0};
#pragma unroll
            for (int k = i + 1; k < BS; ++k) a[k & 3] -= Dr[i * BS + k] * xi[k];
            xi[i] = ((a[0] + a[1]) + (a[2] + a[3])) * rd[i];
        }
    }
#pragma unroll
    for (int i = 0; i < BS; ++i) Di[i * (BS + 1) + lane] = xi[i];
}

// Mx = Di Eb (BS x BS each), all four wavefronts: lane = row, wavefront wv
// = columns 16 wv .. 16 wv + 15.  Di stride BS + 1, Eb stride BS, Mx stride BS + 1.
template <typename V, int BS>
__device__ __forceinline__ void diag_times_tile(const V *__restrict__ Di, const V *__restrict__ Eb,
                                                V *__restrict__ Mx, int lane, int wv)
{
    constexpr int CW = BS / 4;
    V m[CW];
#pragma unroll
    for (int c = 0; c < CW; ++c) m[c] = 0;
#pragma unroll 8
    for (int k = 0; k < BS; ++k) {
        const V d = Di[lane * (BS + 1) + k];
#pragma unroll
        for (int c = 0; c < CW; ++c) m[c] += d * Eb[k * BS + wv * CW + c];
    }
#pragma unroll
    for (int c = 0; c < CW; ++c) Mx[lane * (BS + 1) + wv * CW + c] = m[c];
}

// sum_c r[c] v[c] with v held one value per lane, four independent partial sums.
template <typename V, int BS>
__device__ __forceinline__ V row_times_lanes(const V (&r)[BS], V v)
{
    V a[4] = {0, 0, 0, 0};
#pragma unroll
    for (int c = 0; c < BS; ++c) a[c & 3] += r[c] * lane_bcast(v, c);
    return (a[0] + a[1]) + (a[2] + a[3]);
}
// The same product with v passed through LDS (vb: this wavefront's BS
// entries): one store and BS/4 broadcast reads instead of BS readlanes,
// which the compiler chains through one SGPR with a wait state each.
// (Same sums in the same order as row_times_lanes, so the same result.)
// vb must be 16-byte aligned.
template <typename V, int BS>
__device__ __forceinline__ V row_times_lds(const V (&r)[BS], V v, V *vb, int lane)
{
    constexpr int K = 16 / sizeof(V);
    vb[lane] = v;  // one wavefront's LDS accesses complete in order
    V a[4] = {0, 0, 0, 0};
#pragma unroll
    for (int c = 0; c < BS; c += K) {
        V u[K];
        __builtin_memcpy(u, vb + c, 16);
#pragma unroll
        for (int k = 0; k < K; ++k) a[(c + k) & 3] += r[c + k] * u[k];
    }
    return (a[0] + a[1]) + (a[2] + a[3]);
}
// row `lane` of an LDS matrix with stride BS + 1, into registers
template <typename V, int BS>
__device__ __forceinline__ void load_row(V (&r)[BS], const V *__restrict__ R, int lane)
{
#pragma unroll
    for (int c = 0; c < BS; ++c) r[c] = R[lane * (BS + 1) + c];
}

// ---------------------------------------------------------------- lower
// round_out (both solves): every solution entry is rounded to the factor
// type T as it is formed, before later blocks use it -- the solve held in
// the low precision for the scaled correction of eq. (2.19) (Section 2.3).
//
// y = L^{-1} (P b): L unit lower (below the diagonal of LU), perm[i] = the
// original row placed at position i (null = identity).  Block `blk` owns rows
// [blk*BS, blk*BS + BS) (lane = row); wavefront w consumes tiles w, w+4, ...
// below blk - 1, keeping the next tile's loads in flight while it consumes
// the current one.  Tile blk - 1 enters through Mx = D^{-1} L_{b,b-1}.
template <typename T, typename V, int BS>
__global__ __launch_bounds__(256) void k_trsv_lower(int64_t n, const T *__restrict__ LU, int64_t lda,
                                                    const int32_t *__restrict__ perm,
                                                    const V *__restrict__ b, V *__restrict__ y,
                                                    int *__restrict__ sync, uint32_t epoch,
                                                    int *__restrict__ flags, int round_out)
{
    static_assert(BS == 64, "a wavefront spans one tile");
    __shared__ int s_blk;
    __shared__ __attribute__((aligned(16))) V Dr[BS * (BS + 1)];  // D (stride BS), then Mx (stride BS + 1)
    __shared__ __attribute__((aligned(16))) V Eb[BS * BS];        // L_{b,b-1}
    __shared__ V Di[BS * (BS + 1)];                               // D^{-1}
    __shared__ V part[4][BS];
    __shared__ __attribute__((aligned(16))) V vb[4][BS];  // each wavefront's broadcast vector
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (tid == 0) s_blk = __hip_atomic_fetch_add(&sync[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int blk = s_blk;
    uint64_t *tags = tag_words(sync);
    const int64_t r0 = (int64_t)blk * BS;
    const int64_t row = r0 + lane;
    const bool rv = row < n;
    const int64_t rowc = rv ? row : 0;
    V acc = 0;
    int spins = 0;
    V fv[BS], fvn[BS];
    lane_word<V> cur, nxt;
    const int last = blk - 1;  // tiles jb < last go through the loop
    for (int e = tid; e < BS * BS; e += 256) {
        const int i = e % BS, j = e / BS;
        const bool in = r0 + i < n;
        Dr[i * BS + j] = (j < i && in) ? (V)to_f32(LU[(r0 + i) + (r0 + j) * lda]) : (V)0;
        if (blk > 0) Eb[i * BS + j] = in ? (V)to_f32(LU[(r0 + i) + (r0 - BS + j) * lda]) : (V)0;
    }
    __syncthreads();
    if (wv == 0) diag_inverse<V, BS, true>(Dr, nullptr, Di, lane);
    __syncthreads();
    if (blk > 0) diag_times_tile<V, BS>(Di, Eb, Dr, lane, wv);
    int jb = wv;
    if (jb < last) {
        load_tile_row<T, V, BS>(fv, LU, lda, rowc, (int64_t)jb * BS, n);
        cur.issue(tags, (int64_t)jb * BS + lane, true);
    }
    for (; jb < last; jb += 4) {
        const int nj = jb + 4;
        if (nj < last) {
            load_tile_row<T, V, BS>(fvn, LU, lda, rowc, (int64_t)nj * BS, n);
            nxt.issue(tags, (int64_t)nj * BS + lane, true);
        }
        cur.settle(tags, (int64_t)jb * BS + lane, true, epoch, &spins, flags, std::min(32, last - jb - 2));
        acc += row_times_lds<V, BS>(fv, cur.value(), vb[wv], lane);
#pragma unroll
        for (int c = 0; c < BS; ++c) fv[c] = fvn[c];
        cur = nxt;
    }
    part[wv][lane] = acc;
    __syncthreads();
    if (wv == 0) {
        V z = 0;
        if (rv) {
            const int64_t src = perm ? (int64_t)perm[row] : row;
            z = b[src] - ((part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]));
        }
        V rr[BS];
        load_row<V, BS>(rr, Di, lane);
        V w = row_times_lds<V, BS>(rr, z, vb[0], lane);
        if (blk > 0) {
            // the only work left after the predecessor publishes: one product
            // with a row already in registers
            load_row<V, BS>(rr, Dr, lane);
            lane_word<V> xp;
            xp.issue(tags, (int64_t)last * BS + lane, true);
            xp.template settle_ring<8>(tags, (int64_t)last * BS + lane, true, epoch, &spins, flags);
            w -= row_times_lds<V, BS>(rr, xp.value(), vb[0], lane);
        }
        if (round_out) w = (V)to_f32((T)w);  // solution held in the factor precision
        if (rv) {
            y[row] = w;
            tagged<V>::put(tags, row, w, epoch);
        }
    }
}

// ---------------------------------------------------------------- upper
// x = S U^{-1} y with S = diag(colscale) (null = identity).  Blocks run from
// the last to the first; other blocks read the unscaled solution (tagged).
// Tile blk + 1 enters through Mx = D^{-1} U_{b,b+1}.
template <typename T, typename V, int BS>
__global__ __launch_bounds__(256) void k_trsv_upper(int64_t n, const T *__restrict__ LU, int64_t lda,
                                                    const V *__restrict__ yin,
                                                    const float *__restrict__ colscale,
                                                    V *__restrict__ x, int *__restrict__ sync,
                                                    uint32_t epoch, int *__restrict__ flags,
                                                    int round_out)
{
    static_assert(BS == 64, "a wavefront spans one tile");
    __shared__ int s_blk;
    __shared__ __attribute__((aligned(16))) V Dr[BS * (BS + 1)];  // D (stride BS), then Mx (stride BS + 1)
    __shared__ __attribute__((aligned(16))) V Eb[BS * BS];        // U_{b,b+1}
    __shared__ V Di[BS * (BS + 1)];                               // D^{-1}
    __shared__ V rd[BS];
    __shared__ V part[4][BS];
    __shared__ __attribute__((aligned(16))) V vb[4][BS];  // each wavefront's broadcast vector
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int nb = (int)((n + BS - 1) / BS);
    if (tid == 0) s_blk = nb - 1 - __hip_atomic_fetch_add(&sync[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int blk = s_blk;
    uint64_t *tags = tag_words(sync);
    const int64_t r0 = (int64_t)blk * BS;
    const int64_t row = r0 + lane;
    const bool rv = row < n;
    const int64_t rowc = rv ? row : 0;
    V acc = 0;
    int spins = 0;
    V fv[BS], fvn[BS];
    lane_word<V> cur, nxt;
    const int next = blk + 1;  // tiles jb > next go through the loop
    const bool has_next = next < nb;
    for (int e = tid; e < BS * BS; e += 256) {
        const int i = e % BS, j = e / BS;
        const bool in = r0 + i < n && r0 + j < n;
        const V u = in ? (V)to_f32(LU[(r0 + i) + (r0 + j) * lda]) : (V)0;
        Dr[i * BS + j] = j > i ? u : (V)0;
        if (i == j) rd[i] = in ? (V)1 / u : (V)1;
        if (has_next) {
            const bool in2 = r0 + i < n && r0 + BS + j < n;
            Eb[i * BS + j] = in2 ? (V)to_f32(LU[(r0 + i) + (r0 + BS + j) * lda]) : (V)0;
        }
    }
    __syncthreads();
    if (wv == 0) diag_inverse<V, BS, false>(Dr, rd, Di, lane);
    __syncthreads();
    if (has_next) diag_times_tile<V, BS>(Di, Eb, Dr, lane, wv);
    int jb = nb - 1 - wv;
    if (jb > next) {
        load_tile_row<T, V, BS>(fv, LU, lda, rowc, (int64_t)jb * BS, n);
        cur.issue(tags, (int64_t)jb * BS + lane, (int64_t)jb * BS + lane < n);
    }
    for (; jb > next; jb -= 4) {
        const int nj = jb - 4;
        if (nj > next) {
            load_tile_row<T, V, BS>(fvn, LU, lda, rowc, (int64_t)nj * BS, n);
            nxt.issue(tags, (int64_t)nj * BS + lane, true);
        }
        const bool valid = (int64_t)jb * BS + lane < n;
        cur.settle(tags, (int64_t)jb * BS + lane, valid, epoch, &spins, flags, std::min(32, jb - next - 2));
        acc += row_times_lds<V, BS>(fv, valid ? cur.value() : (V)0, vb[wv], lane);
#pragma unroll
        for (int c = 0; c < BS; ++c) fv[c] = fvn[c];
        cur = nxt;
    }
    part[wv][lane] = acc;
    __syncthreads();
    if (wv == 0) {
        const V z = rv ? yin[row] - ((part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane])) : (V)0;
        V rr[BS];
        load_row<V, BS>(rr, Di, lane);
        V w = row_times_lds<V, BS>(rr, z, vb[0], lane);
        if (has_next) {
            load_row<V, BS>(rr, Dr, lane);
            const bool valid = (int64_t)next * BS + lane < n;
            lane_word<V> xn;
            xn.issue(tags, (int64_t)next * BS + lane, valid);
            xn.template settle_ring<8>(tags, (int64_t)next * BS + lane, valid, epoch, &spins, flags);
            w -= row_times_lds<V, BS>(rr, valid ? xn.value() : (V)0, vb[0], lane);
        }
        if (round_out) w = (V)to_f32((T)w);
        if (rv) {
            tagged<V>::put(tags, row, w, epoch);
            x[row] = colscale ? w * (V)colscale[row] : w;
        }
    }
}

__global__ void k_zero_ticket(int *sync) { sync[0] = 0; }

// ticket (4 ints, keeps the tag words 16-byte aligned) + 2 tag words per entry
size_t trsv_sync_ints(int64_t n) { return (size_t)(4 + 4 * n); }

template <typename T, typename V>
static hipError_t trsv_lower_t(int64_t n, const void *LU, int64_t lda, const int32_t *perm,
                               const V *b, V *y, int *sync, uint32_t epoch, int *flags,
                               hipStream_t s, int round_out = 0)
{
    const unsigned nb = (unsigned)((n + TRSV_BS - 1) / TRSV_BS);
    hipLaunchKernelGGL(k_zero_ticket, dim3(1), dim3(1), 0, s, sync);
    hipLaunchKernelGGL((k_trsv_lower<T, V, TRSV_BS>), dim3(nb), dim3(256), 0, s, n, (const T *)LU,
                       lda, perm, b, y, sync, epoch, flags, round_out);
    return hipGetLastError();
}

template <typename T, typename V>
static hipError_t trsv_upper_t(int64_t n, const void *LU, int64_t lda, const V *y,
                               const float *colscale, V *x, int *sync, uint32_t epoch, int *flags,
                               hipStream_t s, int round_out = 0)
{
    const unsigned nb = (unsigned)((n + TRSV_BS - 1) / TRSV_BS);
    hipLaunchKernelGGL(k_zero_ticket, dim3(1), dim3(1), 0, s, sync);
    hipLaunchKernelGGL((k_trsv_upper<T, V, TRSV_BS>), dim3(nb), dim3(256), 0, s, n, (const T *)LU,
                       lda, y, colscale, x, sync, epoch, flags, round_out);
    return hipGetLastError();
}

hipError_t launch_trsv_lower(int prec, int64_t n, const void *LU, int64_t lda, const int32_t *perm,
                             const float *b, float *y, int *sync, uint32_t epoch, int *flags,
                             hipStream_t s, int round_out)
{
    switch (prec) {
    case N3P_FP16: return trsv_lower_t<f16, float>(n, LU, lda, perm, b, y, sync, epoch, flags, s, round_out);
    case N3P_BF16: return trsv_lower_t<bf16, float>(n, LU, lda, perm, b, y, sync, epoch, flags, s, round_out);
    case N3P_FP32: return trsv_lower_t<float, float>(n, LU, lda, perm, b, y, sync, epoch, flags, s, round_out);
    case N3P_FP64: return trsv_lower_t<double, float>(n, LU, lda, perm, b, y, sync, epoch, flags, s, round_out);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_trsv_upper(int prec, int64_t n, const void *LU, int64_t lda, const float *y,
                             const float *colscale, float *x, int *sync, uint32_t epoch, int *flags,
                             hipStream_t s, int round_out)
{
    switch (prec) {
    case N3P_FP16: return trsv_upper_t<f16, float>(n, LU, lda, y, colscale, x, sync, epoch, flags, s, round_out);
    case N3P_BF16: return trsv_upper_t<bf16, float>(n, LU, lda, y, colscale, x, sync, epoch, flags, s, round_out);
    case N3P_FP32: return trsv_upper_t<float, float>(n, LU, lda, y, colscale, x, sync, epoch, flags, s, round_out);
    case N3P_FP64: return trsv_upper_t<double, float>(n, LU, lda, y, colscale, x, sync, epoch, flags, s, round_out);
    }
    return hipErrorInvalidValue;
}

// out = I_s^h(a * in): the scaled vector rounded to the factor type (held as
// FP32 values), the right-hand side of the low-precision solves of eq. (2.19)
template <typename T>
__global__ __launch_bounds__(256) void k_scale_round(int64_t n, const float *__restrict__ in, float a,
                                                     float *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = to_f32((T)(in[i] * a));
}

hipError_t launch_scale_round(int prec, int64_t n, const float *in, float a, float *out, hipStream_t s)
{
    const unsigned g = (unsigned)((n + 255) / 256);
    switch (prec) {
    case N3P_FP16: hipLaunchKernelGGL(k_scale_round<f16>, dim3(g), dim3(256), 0, s, n, in, a, out); break;
    case N3P_BF16: hipLaunchKernelGGL(k_scale_round<bf16>, dim3(g), dim3(256), 0, s, n, in, a, out); break;
    case N3P_FP32:
    case N3P_FP64: hipLaunchKernelGGL(k_scale_round<float>, dim3(g), dim3(256), 0, s, n, in, a, out); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_trsv_lower_f64(int64_t n, const double *LU, int64_t lda, const int32_t *perm,
                                 const double *b, double *y, int *sync, uint32_t epoch, int *flags,
                                 hipStream_t s)
{
    return trsv_lower_t<double, double>(n, LU, lda, perm, b, y, sync, epoch, flags, s);
}

hipError_t launch_trsv_upper_f64(int64_t n, const double *LU, int64_t lda, const double *y,
                                 double *x, int *sync, uint32_t epoch, int *flags, hipStream_t s)
{
    return trsv_upper_t<double, double>(n, LU, lda, y, nullptr, x, sync, epoch, flags, s);
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

// The same partial sums with four consecutive rows per thread (one 16-byte
// load per column, so a wavefront reads 1 KB contiguous): needs n, lda and A
// 16-byte aligned.  Per row the same four sums in the same order as above,
// so the results are identical.
constexpr int MV_ROWS4 = 1024;
__global__ __launch_bounds__(256) void k_gemv_f32_part4(int64_t n, const float *__restrict__ A,
                                                        int64_t lda, const float *__restrict__ u,
                                                        double *__restrict__ part)
{
    typedef float f4 __attribute__((ext_vector_type(4)));
    __shared__ float ush[MV_CH];
    const int64_t j0 = (int64_t)blockIdx.y * MV_CH;
    const int64_t jn = std::min<int64_t>(MV_CH, n - j0);
    if (threadIdx.x < jn) ush[threadIdx.x] = u[j0 + threadIdx.x];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * MV_ROWS4 + 4 * (int64_t)threadIdx.x;
    if (i >= n) return;
    const float *ap = A + i + j0 * lda;
    double s[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int k = 0; k < 4; ++k) s[q][k] = 0.0;
    int64_t c = 0;
    for (; c + 4 <= jn; c += 4) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const f4 a = *(const f4 *)(ap + (c + k) * lda);
            const double uk = (double)ush[c + k];
#pragma unroll
            for (int q = 0; q < 4; ++q) s[q][k] += (double)a[q] * uk;
        }
    }
    for (; c < jn; ++c) {
        const f4 a = *(const f4 *)(ap + c * lda);
        const double uk = (double)ush[c];
#pragma unroll
        for (int q = 0; q < 4; ++q) s[q][0] += (double)a[q] * uk;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
        part[(int64_t)blockIdx.y * n + i + q] = (s[q][0] + s[q][1]) + (s[q][2] + s[q][3]);
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
    if (n % 4 == 0 && lda % 4 == 0 && ((uintptr_t)A & 15) == 0)
        hipLaunchKernelGGL(k_gemv_f32_part4, dim3((unsigned)((n + MV_ROWS4 - 1) / MV_ROWS4), nch),
                           dim3(256), 0, s, n, A, lda, u, part);
    else
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

// ------------------------------------------------ allocation-free matvec
// Fixed scratch for the allocation-free form of r = b - A u: the FP64
// partial sums of one call, n * ceil(n / MV_CH) doubles for n <= GEMV_NOALLOC_MAX_N
// (8 MiB).  Each device holds its own copy at its own address until the
// process ends.  In host code `scratch` names a host-side stand-in, not device
// memory, so it is never passed to a kernel: the device address is looked up
// with hipGetSymbolAddress once per device (with that device current) and
// that pointer is what the kernels receive.
constexpr int64_t GEMV_NOALLOC_MAX_N = N3P_GEMV_NOALLOC_MAX_N;
constexpr size_t GEMV_NOALLOC_DOUBLES = (size_t)GEMV_NOALLOC_MAX_N * (GEMV_NOALLOC_MAX_N / MV_CH);
static_assert(GEMV_NOALLOC_MAX_N % MV_CH == 0, "scratch sized for whole column chunks");
static __device__ __align__(256) double scratch[GEMV_NOALLOC_DOUBLES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_dev[NOALLOC_MAX_DEVICES];

static hipError_t noalloc_scratch(double **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_dev[dev] = (double *)ptr;
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

hipError_t launch_gemv_resid_noalloc(int64_t n, const float *A, int64_t lda, const float *u,
                                     const float *b, float *r, hipStream_t s)
{
    if (n < 1 || n > GEMV_NOALLOC_MAX_N) return hipErrorInvalidValue;
    double *part = nullptr;
    const hipError_t e = noalloc_scratch(&part);
    if (e != hipSuccess) return e;
    return launch_gemv_resid(n, A, lda, u, b, r, part, s);
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


// ====================================================== batched engine kernels
// One workgroup per slot (N <= B_MAX_NP): y = L^{-1} r (unit lower), then
// z = U^{-1} y, d = S z (S the FP16 column scale), and uprev = u, u += d:
// the correction step of the IR algorithm of Section 2.2 with the stored half-precision factors
// promoted to FP32 as they are read (Section 2.3).  Blocked by 64: one wave
// substitutes the diagonal block (a row per lane, readlane broadcasts), then
// all waves update the remaining rows with coalesced column reads while the
// next diagonal block's loads are in flight.
template <typename T>
__global__ __launch_bounds__(B_SOLVE_THREADS) void k_b_solve(const BDesc *__restrict__ d,
                                                             const BState *__restrict__ st,
                                                             int nslots)
{
    constexpr int NT = B_SOLVE_THREADS;
    __shared__ float y[B_MAX_NP];
    __shared__ float Dg[64][65];
    const int s = blockIdx.x;
    if (s >= nslots || st[s].phase != BP_RUN || !st[s].factor || !st[s].ir_on) return;
    const BDesc &q = d[s];
    const int64_t Np = q.Np, n = q.n;
    const T *__restrict__ A = (const T *)q.A;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int nb = (int)(Np / 64);
    // the next diagonal block is fetched into registers while the current
    // block's update runs, and stored to Dg once the substitution is done
    static_assert(NT * 4 == 64 * 64, "four diagonal entries per thread");
    float pre[4];
    auto fetch = [&](int64_t b0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = t + r * NT, i = e & 63, k = e >> 6;
            pre[r] = to_f32(A[(b0 + i) + (b0 + k) * Np]);
        }
    };
    auto put = [&]() {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = t + r * NT, i = e & 63, k = e >> 6;
            Dg[i][k] = pre[r];
        }
    };
    for (int64_t i = t; i < Np; i += NT) y[i] = q.r[i];
    fetch(0);
    put();
    __syncthreads();
    for (int blk = 0; blk < nb; ++blk) {  // forward, unit lower
        const int64_t b0 = (int64_t)blk * 64;
        if (wave == 0) {
            float lr[64];
#pragma unroll
            for (int k = 0; k < 64; ++k) lr[k] = lane > k ? Dg[lane][k] : 0.0f;
            float yi = y[b0 + lane];
#pragma unroll
            for (int k = 0; k < 64; ++k) yi -= lr[k] * lane_bcast(yi, k);
            y[b0 + lane] = yi;
        }
        __syncthreads();
        const bool more = blk + 1 < nb;
        if (more) fetch(b0 + 64);
        for (int64_t i = b0 + 64 + t; i < Np; i += NT) {
            const T *__restrict__ col = A + i + b0 * Np;
            float acc = y[i];
#pragma unroll 16
            for (int k = 0; k < 64; ++k) acc -= to_f32(col[(int64_t)k * Np]) * y[b0 + k];
            y[i] = acc;
        }
        if (more) put();
        __syncthreads();
    }
    fetch((int64_t)(nb - 1) * 64);
    put();
    __syncthreads();
    for (int blk = nb - 1; blk >= 0; --blk) {  // backward, upper
        const int64_t b0 = (int64_t)blk * 64;
        if (wave == 0) {
            float ur[64];
#pragma unroll
            for (int k = 0; k < 64; ++k) ur[k] = lane < k ? Dg[lane][k] : 0.0f;
            const float rd = 1.0f / Dg[lane][lane];
            float yi = y[b0 + lane];
#pragma unroll
            for (int k = 63; k >= 0; --k) {
                if (lane == k) yi *= rd;
                yi -= ur[k] * lane_bcast(yi, k);
            }
            y[b0 + lane] = yi;
        }
        __syncthreads();
        const bool more = blk > 0;
        if (more) fetch(b0 - 64);
        for (int64_t i = t; i < b0; i += NT) {
            const T *__restrict__ col = A + i + b0 * Np;
            float acc = y[i];
#pragma unroll 16
            for (int k = 0; k < 64; ++k) acc -= to_f32(col[(int64_t)k * Np]) * y[b0 + k];
            y[i] = acc;
        }
        if (more) put();
        __syncthreads();
    }
    for (int64_t i = t; i < Np; i += NT) {
        float di = 0.0f;
        if (i < n) di = q.colscale ? y[i] * q.colscale[i] : y[i];
        const float ui = q.u[i];
        q.uprev[i] = ui;
        q.u[i] = ui + di;
    }
}

// r = b - J u with FP64 accumulation; items are 256-row blocks of a slot
__global__ __launch_bounds__(256) void k_b_gemv(const BDesc *__restrict__ d,
                                                const BState *__restrict__ st, int nslots)
{
    __shared__ float us[B_MAX_NP];
    __shared__ int off[B_MAX_SLOTS + 1];
    const int total = b_offsets(nslots, off, [&](int s) {
        return (st[s].phase == BP_RUN && st[s].factor && st[s].ir_on) ? (int)((d[s].Np + 255) / 256) : 0;
    });
    const int t = threadIdx.x;
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int s = b_find(off, nslots, item);
        const BDesc &q = d[s];
        const int64_t n = q.n;
        for (int64_t j = t; j < n; j += 256) us[j] = q.u[j];
        __syncthreads();
        const int64_t i = (int64_t)(item - off[s]) * 256 + t;
        if (i < n) {
            const float *__restrict__ row = q.J + i;
            double acc = (double)q.b[i];
            int64_t j = 0;
            for (; j + 8 <= n; j += 8) {
                float a[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) a[u] = row[(j + u) * n];
#pragma unroll
                for (int u = 0; u < 8; ++u) acc -= (double)a[u] * (double)us[j + u];
            }
            for (; j < n; ++j) acc -= (double)row[j * n] * (double)us[j];
            q.r[i] = (float)acc;
        } else if (i < q.Np) {
            q.r[i] = 0.0f;
        }
        __syncthreads();
    }
}

hipError_t launch_b_solve(int prec, const BDesc *d, const BState *st, int nslots, hipStream_t s)
{
    switch (prec) {
    case N3P_FP16: hipLaunchKernelGGL(k_b_solve<f16>, dim3(nslots), dim3(B_SOLVE_THREADS), 0, s, d, st, nslots); break;
    case N3P_BF16: hipLaunchKernelGGL(k_b_solve<bf16>, dim3(nslots), dim3(B_SOLVE_THREADS), 0, s, d, st, nslots); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_b_gemv(const BDesc *d, const BState *st, int nslots, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_b_gemv, dim3(grid), dim3(256), 0, s, d, st, nslots);
    return hipGetLastError();
}

}  // namespace n3p
