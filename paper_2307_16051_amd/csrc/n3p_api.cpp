// n3p_api.cpp -- host driver and C ABI of libn3p.
//
// Newton's method in three precisions (Kelley, arXiv 2307.16051):
//   * Algorithm 2.1 (newton3p) drives the outer loop on the host; every
//     vector and matrix operation runs in the HIP kernels of this library;
//   * the IR algorithm of Section 2.2 with the stopping policy of Section 3.1
//     (success below eta ||b||, failure when the residual grows, best iterate
//     returned) solves the step equation, or GMRES-IR (end of Section 2.2)
//     computes each correction;
//   * the right-hand side is scaled to unit norm before the solve and the
//     step unscaled afterwards (eqs. (2.17)-(2.18)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "n3p_internal.hpp"

namespace n3p {
hipError_t launch_leaf_spec2(int prec, int64_t Np, int64_t c0, void *A, int64_t lda, void *LT,
                             int64_t k0, void *DG, const void *DGprev, int64_t cprev, int *flags,
                             hipStream_t s);
hipError_t launch_put_diag(int prec, int64_t c0, void *A, int64_t lda, const void *DG,
                           const int *flags, hipStream_t s);
}  // namespace n3p

using namespace n3p;

namespace {

#define HIPCHK(expr)                                                                  \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess) {                                                       \
            if (std::getenv("N3P_DEBUG"))                                             \
                std::fprintf(stderr, "n3p: %s failed: %s (%s:%d)\n", #expr,           \
                             hipGetErrorString(e_), __FILE__, __LINE__);              \
            return N3P_E_HIP;                                                         \
        }                                                                             \
    } while (0)

#define CHK(expr)                     \
    do {                              \
        int st_ = (expr);             \
        if (st_ < 0) return st_;      \
    } while (0)

constexpr size_t ALIGN = 256;

struct Bump {
    size_t off = 0;
    size_t take(size_t bytes)
    {
        size_t o = (off + ALIGN - 1) / ALIGN * ALIGN;
        off = o + bytes;
        return o;
    }
};

bool valid_prec(int p) { return p >= N3P_FP16 && p <= N3P_FP64; }
int64_t padded(int64_t n) { return round_up(std::max<int64_t>(n, 1), NB_PAD); }

// ------------------------------------------------------------ factor state
struct FactorWs {
    int prec = 0;
    int64_t Np = 0;
    void *A = nullptr;        // Np x Np, ld Np
    void *LT = nullptr;       // Np x NB_OUT
    void *DG = nullptr;       // 2 x NB_LEAF^2
    void *xch = nullptr;      // pivoting path: exchange words and interchange list
    int32_t *ipiv = nullptr;  // Np
    int32_t *perm = nullptr;  // Np (device), valid if pivoted
    int *flags = nullptr;     // NFLAGS
    uint64_t *pub = nullptr;  // FP16/BF16: publication words of the diagonal-square kernel
    float *inv = nullptr;     // FP16/BF16: the leaves' triangular inverses
};

bool top_path(int prec) { return prec == N3P_FP16 || prec == N3P_BF16; }

size_t factor_bytes(int prec, int64_t Np, Bump &b, FactorWs *f, char *base)
{
    const size_t es = elem_size(prec);
    size_t oA = b.take((size_t)Np * Np * es);
    // the diagonal-square path double-buffers LT by block parity (the next
    // block's square is factored while this block's update still reads LT)
    size_t oLT = b.take((size_t)Np * NB_OUT * es * (top_path(prec) ? 2 : 1));
    size_t oDG = b.take((size_t)2 * NB_LEAF * NB_LEAF * es);
    size_t oS = b.take(pivot_xch_bytes(prec, Np));
    size_t oI = b.take((size_t)Np * 4);
    size_t oP = b.take((size_t)Np * 4);
    size_t oF = b.take((size_t)NFLAGS * 4);
    size_t oPub = top_path(prec) ? b.take(top_pub_words() * 8) : 0;
    size_t oInv = top_path(prec) ? b.take(top_inv_floats() * 4) : 0;
    if (f && base) {
        f->pub = top_path(prec) ? (uint64_t *)(base + oPub) : nullptr;
        f->inv = top_path(prec) ? (float *)(base + oInv) : nullptr;
        f->prec = prec;
        f->Np = Np;
        f->A = base + oA;
        f->LT = base + oLT;
        f->DG = base + oDG;
        f->xch = base + oS;
        f->ipiv = (int32_t *)(base + oI);
        f->perm = (int32_t *)(base + oP);
        f->flags = (int *)(base + oF);
    }
    return b.off;
}

struct FactorResult {
    bool pivoted = false;
    int info = 0;        // k+1 of the first zero pivot
    bool nonfinite = false;
    bool timeout = false;
};

int read_flags(const FactorWs &f, hipStream_t s, int *h)
{
    HIPCHK(hipMemcpyAsync(h, f.flags, NFLAGS * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return 0;
}

// No-interchange attempt (verified against the partial-pivoting rule).
// Three levels of right-looking updates: after each 64-column leaf the rest
// of its 256-column middle block (below) and the middle block's rows to the
// right (to the end of the matrix); after each middle block, K = 256, the
// rest of the 1024-column outer block (below) and the outer block's rows to
// its right; after each outer block, K = 1024, the trailing matrix.
int getrf_spec(const FactorWs &f, hipStream_t s)
{
    const int prec = f.prec;
    const int64_t Np = f.Np, lda = Np;
    const size_t es = elem_size(prec);
    char *A = (char *)f.A;
    char *LT = (char *)f.LT;
    char *DG = (char *)f.DG;
    const size_t dgb = (size_t)NB_LEAF * NB_LEAF * es;
    const bool mfma16 = prec == N3P_FP16 || prec == N3P_BF16;
    auto at = [&](int64_t i, int64_t j) { return (void *)(A + ((size_t)i + (size_t)j * lda) * es); };
    // C(r0.., c0..) of the two updates (r0 = first row below the source
    // panel, [cb, ce) its block's columns): the rest of the block below the
    // panel, and the block's rows right of the block.  At: LT rows from r0,
    // K columns from kc within the outer block; B: the panel's U rows.
    auto update = [&](int64_t r0, int64_t ce, int64_t prow, int64_t kc, int64_t K) -> int {
        const void *At = LT + ((size_t)r0 * NB_OUT + (size_t)kc) * es;
        if (mfma16) {
            HIPCHK(launch_gemm_pair(prec, Np - r0, ce - r0, At, NB_OUT, at(prow, r0), lda,
                                    at(r0, r0), lda, ce - r0, Np - ce, At, NB_OUT, at(prow, ce),
                                    lda, at(r0, ce), lda, K, f.flags, s));
        } else {
            HIPCHK(launch_gemm_sub(prec, Np - r0, ce - r0, K, At, NB_OUT, at(prow, r0), lda,
                                   at(r0, r0), lda, f.flags, true, s));
            if (ce < Np)
                HIPCHK(launch_gemm_sub(prec, ce - r0, Np - ce, K, At, NB_OUT, at(prow, ce), lda,
                                       at(r0, ce), lda, f.flags, true, s));
        }
        return 0;
    };
    for (int64_t k0 = 0; k0 < Np; k0 += NB_OUT) {
        const int64_t kend = std::min<int64_t>(k0 + NB_OUT, Np);
        for (int64_t m0 = k0; m0 < kend; m0 += NB_MID) {
            const int64_t mend = std::min<int64_t>(m0 + NB_MID, kend);
            for (int64_t c0 = m0; c0 < mend; c0 += NB_LEAF) {
                const int64_t leaf = c0 / NB_LEAF;
                void *dg = DG + (leaf % 2) * dgb;
                const void *dgp = leaf > 0 ? DG + ((leaf - 1) % 2) * dgb : nullptr;
                HIPCHK(launch_leaf_spec2(prec, Np, c0, f.A, lda, f.LT, k0, dg, dgp, c0 - NB_LEAF,
                                         f.flags, s));
                const int64_t c1 = c0 + NB_LEAF;
                if (c1 < mend) CHK(update(c1, mend, c0, c0 - k0, NB_LEAF));
            }
            if (mend < kend) CHK(update(mend, kend, m0, m0 - k0, mend - m0));
        }
        if (kend < Np) {
            const void *At = LT + (size_t)kend * NB_OUT * es;
            HIPCHK(launch_gemm_sub(prec, Np - kend, Np - kend, kend - k0, At, NB_OUT, at(k0, kend),
                                   lda, at(kend, kend), lda, f.flags, true, s));
        }
    }
    const int64_t last = Np / NB_LEAF - 1;
    HIPCHK(launch_put_diag(prec, Np - NB_LEAF, f.A, lda, DG + (last % 2) * dgb, f.flags, s));
    return 0;
}

// No-interchange attempt for FP16 / BF16 (verified against the
// partial-pivoting rule), one outer block of up to NB_OUT columns at a time,
// with look-ahead: block j's L below its square and U right of it (k_trsm),
// the update of block j + 1's square, then that square factored in the same
// launch as the rest of block j's update (the rows below the square included).  LT alternates between
// two buffers by block parity.  Publication tags are unique within a
// factorisation (the area is cleared once at its start).
int getrf_spec_top(const FactorWs &f, hipStream_t s)
{
    const int prec = f.prec;
    const int64_t Np = f.Np, lda = Np;
    const size_t es = elem_size(prec);
    char *A = (char *)f.A;
    char *LTb[2] = {(char *)f.LT, (char *)f.LT + (size_t)Np * NB_OUT * es};
    auto at = [&](int64_t i, int64_t j) { return (void *)(A + ((size_t)i + (size_t)j * lda) * es); };
    HIPCHK(launch_fill_i32((int *)f.pub, 0, (int64_t)(top_pub_words() * 2), s));
    uint32_t tag0 = 1;
    HIPCHK(launch_top(prec, 0, (int)std::min<int64_t>(NB_OUT, Np), f.A, lda, LTb[0], f.pub, f.inv,
                      f.flags, tag0, s));
    for (int64_t j = 0;; ++j) {
        const int64_t k0 = j * NB_OUT;
        const int W = (int)std::min<int64_t>(NB_OUT, Np - k0);
        const int64_t kend = k0 + W;
        if (kend >= Np) break;
        char *LTj = LTb[j & 1];
        const void *Lbelow = LTj + (size_t)kend * NB_OUT * es;
        HIPCHK(launch_trsm(prec, Np, k0, W, f.A, lda, LTj, f.inv, f.flags, s));
        const int W1 = (int)std::min<int64_t>(NB_OUT, Np - kend);
        // the next square first; the rows below it join the fused update
        HIPCHK(launch_gemm_sub(prec, W1, W1, W, Lbelow, NB_OUT, at(k0, kend), lda,
                               at(kend, kend), lda, f.flags, true, s));
        tag0 += NB_OUT / NB_LEAF;
        const int64_t rest = Np - kend - W1;
        if (rest > 0) {
            HIPCHK(launch_top_gemm(prec, kend, W1, f.A, lda, LTb[(j + 1) & 1], f.pub, f.inv, f.flags,
                                   tag0, Np - kend, rest, W, Lbelow, NB_OUT, at(k0, kend + W1),
                                   lda, at(kend, kend + W1), lda, rest, W1,
                                   (const char *)Lbelow + (size_t)W1 * NB_OUT * es, at(k0, kend),
                                   at(kend + W1, kend), s));
        } else {
            HIPCHK(launch_top(prec, kend, W1, f.A, lda, LTb[(j + 1) & 1], f.pub, f.inv, f.flags,
                              tag0, s));
        }
    }
    return 0;
}

// Explicit partial pivoting, blocked like getrf_spec, except that rows to
// the right of an outer block are touched only once the whole block is
// pivoted (a later leaf may interchange a row of the block with one below it).
// Per leaf: the cooperative panel (pivot search, interchanges inside the leaf,
// L21, ipiv), the leaf's interchanges on the rest of the outer block with its
// U row block there, and the rank-64 update inside the block.  Per outer
// block: the block's interchanges on every other column, LT rebuilt, the U
// row block right of the block (leaf by leaf: triangular solve, then rank-64
// update of the block's later rows), and the K = NB_OUT update of the
// trailing matrix.
// The side stream of the pivoting path, one per device (default priority,
// like every stream here).  A block's U rows and trailing update beyond the
// next block's columns run on it, beside the next block's panel: the panel
// holds at most 64 workgroups of the 256 CUs.
static hipStream_t pivot_side_stream()
{
    static std::mutex mu;
    static std::vector<hipStream_t> streams;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(mu);
    if ((int)streams.size() <= dev) streams.resize((size_t)dev + 1, nullptr);
    if (!streams[dev] && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess)
        streams[dev] = nullptr;
    return streams[dev];
}

int getrf_pivot(const FactorWs &f, hipStream_t s)
{
    const int prec = f.prec;
    const int64_t Np = f.Np, lda = Np;
    const size_t es = elem_size(prec);
    char *A = (char *)f.A;
    auto at = [&](int64_t i, int64_t j) { return (void *)(A + ((size_t)i + (size_t)j * lda) * es); };
    // FP16/BF16: LT is double-buffered, so a block's update beyond the next
    // block can still read its LT while the next block's panel writes the other
    hipStream_t s2 = top_path(prec) ? pivot_side_stream() : nullptr;
    char *LTb[2] = {(char *)f.LT, (char *)f.LT + (s2 ? (size_t)Np * NB_OUT * es : 0)};
    struct Ev {
        hipEvent_t e = nullptr;
        ~Ev()
        {
            if (e) (void)hipEventDestroy(e);  // a destructor has nobody to report to
        }
    } ready, done;  // ready: a block's interchanges and LT formed; done: its side work
    if (s2) {
        HIPCHK(hipEventCreateWithFlags(&ready.e, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&done.e, hipEventDisableTiming));
    }
    bool side = false;  // side work queued that the main stream has not waited for
    HIPCHK(launch_pivot_reset(prec, Np, f.xch, s));
    for (int64_t blk = 0, k0 = 0; k0 < Np; ++blk, k0 += NB_OUT) {
        const int64_t kend = std::min<int64_t>(k0 + NB_OUT, Np);
        char *LT = LTb[blk & 1];
        auto lt = [&](int64_t row, int64_t col) { return (const void *)(LT + ((size_t)row * NB_OUT + (size_t)col) * es); };
        for (int64_t c0 = k0; c0 < kend; c0 += NB_LEAF) {
            HIPCHK(launch_pivot_coop(prec, Np, c0, k0, f.A, lda, f.ipiv, LT, f.xch, f.flags, s));
            HIPCHK(launch_gather_u12(prec, Np, c0, k0, kend, f.A, lda, f.xch, f.flags, s));
            const int64_t c1 = c0 + NB_LEAF;
            if (c1 < kend) {
                HIPCHK(launch_gemm_sub(prec, Np - c1, kend - c1, NB_LEAF, lt(c1, c0 - k0), NB_OUT,
                                       at(c0, c1), lda, at(c1, c1), lda, f.flags, false, s));
            }
        }
        // the block's interchanges reach the columns the side work updates
        if (side) {
            HIPCHK(hipStreamWaitEvent(s, done.e, 0));
            side = false;
        }
        HIPCHK(launch_gather_block(prec, Np, k0, kend, f.A, lda, f.xch, s));
        if (kend < Np) {
            HIPCHK(launch_lt_rebuild(prec, Np, k0, k0, kend - k0, f.A, lda, LT, s));
            // columns [kend, kn) here; with a side stream, [kn, Np) there
            const int64_t kn = s2 ? std::min<int64_t>(kend + NB_OUT, Np) : Np;
            if (kn < Np) {
                HIPCHK(hipEventRecord(ready.e, s));
                HIPCHK(hipStreamWaitEvent(s2, ready.e, 0));
            }
            auto u_rows_and_update = [&](int64_t j0, int64_t j1, hipStream_t st) -> int {
                for (int64_t c0 = k0; c0 < kend; c0 += NB_LEAF) {
                    const int64_t c1 = c0 + NB_LEAF;
                    HIPCHK(launch_u12(prec, c0, j0, j1, f.A, lda, f.flags, st));
                    if (c1 < kend)
                        HIPCHK(launch_gemm_sub(prec, kend - c1, j1 - j0, NB_LEAF, lt(c1, c0 - k0), NB_OUT,
                                               at(c0, j0), lda, at(c1, j0), lda, f.flags, false, st));
                }
                HIPCHK(launch_gemm_sub(prec, Np - kend, j1 - j0, kend - k0, lt(kend, 0), NB_OUT,
                                       at(k0, j0), lda, at(kend, j0), lda, f.flags, false, st));
                return 0;
            };
            CHK(u_rows_and_update(kend, kn, s));
            if (kn < Np) {
                CHK(u_rows_and_update(kn, Np, s2));
                HIPCHK(hipEventRecord(done.e, s2));
                side = true;
            }
        }
    }
    if (side) HIPCHK(hipStreamWaitEvent(s, done.e, 0));
    return 0;
}

// Factor f.A in place.  `refill` restores the unfactored matrix into f.A
// (needed when the no-interchange attempt is abandoned).  `xdev` (optional):
// one double copied to *xhost in the same host wait as the flags (work the
// caller queued before the factorisation).
template <typename Refill>
int getrf_run(const FactorWs &f, hipStream_t s, Refill refill, FactorResult *res,
              const double *xdev = nullptr, double *xhost = nullptr)
{
    int h[NFLAGS];
    HIPCHK(launch_fill_i32(f.flags, 0, NFLAGS, s));
    if (top_path(f.prec)) CHK(getrf_spec_top(f, s));
    else CHK(getrf_spec(f, s));
    // identity interchanges, queued before the wait (the pivoting path
    // overwrites every entry if it runs)
    HIPCHK(launch_iota_i32(f.ipiv, f.Np, s));
    if (xdev) HIPCHK(hipMemcpyAsync(xhost, xdev, sizeof(double), hipMemcpyDeviceToHost, s));
    CHK(read_flags(f, s, h));
    res->pivoted = false;
    if (h[FLAG_FAIL]) {
        // the pivoting path holds one row per thread in at most PIVOT_MAX_WG
        // resident workgroups
        if (f.Np > PIVOT_MAX_NP) {
            if (std::getenv("N3P_DEBUG"))
                std::fprintf(stderr, "n3p: the matrix needs row interchanges and the pivoting "
                                     "path supports n <= %lld\n", (long long)PIVOT_MAX_NP);
            return N3P_E_INVALID;
        }
        CHK(refill());
        HIPCHK(launch_fill_i32(f.flags, 0, NFLAGS, s));
        CHK(getrf_pivot(f, s));
        CHK(read_flags(f, s, h));
        res->pivoted = true;
        // permutation vector for the triangular solves: perm[k] = original row at position k
        std::vector<int32_t> ip((size_t)f.Np), pm((size_t)f.Np);
        HIPCHK(hipMemcpyAsync(ip.data(), f.ipiv, f.Np * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int64_t k = 0; k < f.Np; ++k) pm[k] = (int32_t)k;
        for (int64_t k = 0; k < f.Np; ++k) {
            const int64_t p = ip[k];
            if (p < 0 || p >= f.Np) return N3P_E_HIP;
            std::swap(pm[k], pm[p]);
        }
        HIPCHK(hipMemcpyAsync(f.perm, pm.data(), f.Np * sizeof(int32_t), hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    res->info = h[FLAG_ZEROPIV];
    res->nonfinite = h[FLAG_NONFINITE] != 0;
    res->timeout = h[FLAG_TIMEOUT] != 0;
    return 0;
}

// ---------------------------------------------------------- solve workspace
struct SolveWs {
    int64_t n = 0, Np = 0;
    int prec = 0, ls = 0, m = 0;
    FactorWs f;
    float *J = nullptr;        // n x n FP32 (ld n)
    float *colscale = nullptr; // Np
    double *F = nullptr, *D = nullptr, *h = nullptr, *part = nullptr, *scal = nullptr;
    size_t part_len = 0;
    float *b = nullptr, *u = nullptr, *uprev = nullptr, *r = nullptr, *d = nullptr, *y = nullptr,
          *xs = nullptr, *z = nullptr, *av = nullptr, *w = nullptr, *V = nullptr;
    double *H = nullptr, *ydev = nullptr;
    double *b64 = nullptr, *y64 = nullptr, *x64 = nullptr, *xs64 = nullptr;
    int *sync = nullptr;
    uint64_t *stamps = nullptr;  // per-phase timestamps (NSTAMPS)
    // FFT form of the H-equation (fft_residual / matrix_free)
    int L = 0;
    bool fftres = false, mf = false;
    double2 *tw = nullptr, *Hh = nullptr, *t1 = nullptr, *t2 = nullptr, *W = nullptr;
    size_t bytes = 0;
};

constexpr int NSTAMPS = 1024;  // phase timestamps: <= 12 per Newton step, <= 64 steps

size_t part_len_for(int64_t n)
{
    // gemv partials: n x ceil(n/256); dense residual partials: n x ceil(n/512); norms: 256
    return (size_t)std::max<int64_t>(256, n * ((n + 255) / 256));
}

size_t solve_layout(int64_t n, int prec, int ls, int m, int fftmode, SolveWs *w, char *base)
{
    // fftmode: bit 0 FFT residual, bit 1 matrix-free J v (no stored FP32 J)
    Bump b;
    const int64_t Np = padded(n);
    FactorWs f;
    factor_bytes(prec, Np, b, &f, base);
    const bool mf = (fftmode & 2) != 0;
    size_t oJ = mf ? 0 : b.take((size_t)n * n * 4);
    size_t oCS = b.take((size_t)Np * 4);
    size_t oF = b.take((size_t)n * 8), oD = b.take((size_t)n * 8), oH = b.take((size_t)2 * n * 8);
    const size_t pl = part_len_for(n);
    size_t oP = b.take(pl * 8);
    size_t oS = b.take(64 * 8);
    size_t vec = (size_t)Np * 4;
    size_t ob = b.take(vec), ou = b.take(vec), oup = b.take(vec), orr = b.take(vec), od = b.take(vec),
           oy = b.take(vec), oxs = b.take(vec), oz = b.take(vec), oav = b.take(vec), ow = b.take(vec);
    size_t oV = 0, oHh = 0, oyd = 0;
    if (ls == N3P_GMRES_IR) {
        oV = b.take((size_t)(m + 1) * vec);
        oHh = b.take((size_t)(m + 2) * 8);
        oyd = b.take((size_t)(m + 1) * 8);
    }
    size_t ob64 = 0, oy64 = 0, ox64 = 0, oxs64 = 0;
    if (prec == N3P_FP64 && ls == N3P_DIRECT) {
        ob64 = b.take((size_t)Np * 8);
        oy64 = b.take((size_t)Np * 8);
        ox64 = b.take((size_t)Np * 8);
        oxs64 = b.take((size_t)Np * 8);
    }
    size_t osync = b.take(trsv_sync_ints(Np) * 4);
    size_t ostamp = b.take((size_t)NSTAMPS * 8);
    const int L = fftmode ? fft_length(n) : 0;
    size_t otw = 0, oHf = 0, ot1 = 0, ot2 = 0, oW = 0;
    if (L) {
        otw = b.take((size_t)L * 16);
        oHf = b.take((size_t)L * 16);
        ot1 = b.take((size_t)L * 16);
        ot2 = b.take((size_t)L * 16);
        oW = b.take((size_t)L * 16);
    }
    if (w && base) {
        w->L = L;
        w->fftres = L && (fftmode & 1);
        w->mf = L && mf;
        if (L) {
            w->tw = (double2 *)(base + otw);
            w->Hh = (double2 *)(base + oHf);
            w->t1 = (double2 *)(base + ot1);
            w->t2 = (double2 *)(base + ot2);
            w->W = (double2 *)(base + oW);
        }
        w->n = n;
        w->Np = Np;
        w->prec = prec;
        w->ls = ls;
        w->m = m;
        w->f = f;
        w->J = mf ? nullptr : (float *)(base + oJ);
        w->colscale = (float *)(base + oCS);
        w->F = (double *)(base + oF);
        w->D = (double *)(base + oD);
        w->h = (double *)(base + oH);
        w->part = (double *)(base + oP);
        w->part_len = pl;
        w->scal = (double *)(base + oS);
        w->stamps = (uint64_t *)(base + ostamp);
        w->b = (float *)(base + ob);
        w->u = (float *)(base + ou);
        w->uprev = (float *)(base + oup);
        w->r = (float *)(base + orr);
        w->d = (float *)(base + od);
        w->y = (float *)(base + oy);
        w->xs = (float *)(base + oxs);
        w->z = (float *)(base + oz);
        w->av = (float *)(base + oav);
        w->w = (float *)(base + ow);
        if (ls == N3P_GMRES_IR) {
            w->V = (float *)(base + oV);
            w->H = (double *)(base + oHh);
            w->ydev = (double *)(base + oyd);
        }
        if (prec == N3P_FP64 && ls == N3P_DIRECT) {
            w->b64 = (double *)(base + ob64);
            w->y64 = (double *)(base + oy64);
            w->x64 = (double *)(base + ox64);
            w->xs64 = (double *)(base + oxs64);
        }
        w->sync = (int *)(base + osync);
        w->bytes = b.off;
    }
    return b.off + ALIGN;
}

// ---------------------------------------------------------------- helpers
struct Epoch {
    uint32_t v = 0;
    uint32_t next() { return ++v; }
};

int d2h_double(const double *dev, double *host, hipStream_t s)
{
    HIPCHK(hipMemcpyAsync(host, dev, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return 0;
}

// Linear-solver context shared by IR and GMRES-IR.  Vector buffers have
// room for Np entries; only the first n are used.
struct LinCtx {
    int prec;
    int64_t n;
    const float *A;
    int64_t lda;
    const void *LU;
    int64_t ldlu;
    const int32_t *perm;     // null: no interchanges
    const float *colscale;   // null: unscaled factors
    float *y, *xs;           // triangular-solve internals
    float *r, *d, *uprev;    // IR residual, correction, previous iterate
    float *z, *av, *w, *V;   // GMRES: preconditioned residual, A v, Arnoldi vector, basis
    int64_t ldv;
    double *part, *scal, *H, *ydev;
    int *sync;
    int *flags;
    Epoch *epoch;
    hipStream_t s;
    // matrix-free J v of the H-equation (null tw: use the stored A)
    const double2 *tw, *Hh;
    double2 *t1, *t2, *W;
    const double *D;
    double c;
    int L;
    // IR corrections by eq. (2.19): the solves run in the factor precision
    // on the residual scaled to unit norm (Section 2.3)
    bool ir_half = false;
};

// r = b - A u  (A stored FP32, or the H-equation operator when matrix-free)
int lin_resid(LinCtx &c, const float *u, const float *b, float *r, double *part)
{
    if (c.tw)
        HIPCHK(launch_hk_jv(c.n, c.n, c.L, c.c, c.D, u, b, r, c.tw, c.Hh, c.t1, c.t2, c.W, c.s));
    else
        HIPCHK(launch_gemv_resid(c.n, c.A, c.lda, u, b, r, part, c.s));
    return 0;
}

// y = A v
int lin_matvec(LinCtx &c, const float *v, float *y)
{
    if (c.tw)
        HIPCHK(launch_hk_jv(c.n, c.n, c.L, c.c, c.D, v, nullptr, y, c.tw, c.Hh, c.t1, c.t2, c.W, c.s));
    else
        HIPCHK(launch_gemv_f32(c.n, c.A, c.lda, v, y, c.part, c.s));
    return 0;
}

// out = S U^{-1} L^{-1} P in   (the preconditioner-vector product)
int apply_prec(LinCtx &c, const float *in, float *out)
{
    HIPCHK(launch_trsv_lower(c.prec, c.n, c.LU, c.ldlu, c.perm, in, c.y, c.sync, c.epoch->next(),
                             c.flags, c.s));
    HIPCHK(launch_trsv_upper(c.prec, c.n, c.LU, c.ldlu, c.y, c.colscale, out, c.sync,
                             c.epoch->next(), c.flags, c.s));
    return 0;
}

// out = rn * I_h^s(U^{-1} L^{-1} I_s^h(in / rn)) (eq. (2.19)): the scaled
// right-hand side and every solution entry rounded to the factor type
int apply_prec_half(LinCtx &c, const float *in, double rn, float *out)
{
    HIPCHK(launch_scale_round(c.prec, c.n, in, (float)(1.0 / rn), c.z, c.s));
    HIPCHK(launch_trsv_lower(c.prec, c.n, c.LU, c.ldlu, c.perm, c.z, c.y, c.sync, c.epoch->next(),
                             c.flags, c.s, 1));
    HIPCHK(launch_trsv_upper(c.prec, c.n, c.LU, c.ldlu, c.y, c.colscale, out, c.sync,
                             c.epoch->next(), c.flags, c.s, 1));
    HIPCHK(launch_scal_copy_f32(c.n, out, out, rn, c.s));
    return 0;
}

int norm32(LinCtx &c, const float *v, double *out)
{
    HIPCHK(launch_nrm2_f32(c.n, v, c.part, c.scal, c.s));
    return d2h_double(c.scal, out, c.s);
}

struct LinOut {
    int sweeps = 0, inner = 0;
    bool failed = false;
    double rel = 0.0;
};

// Left-preconditioned restarted GMRES(m) with modified Gram-Schmidt, from
// d = 0, on M^{-1} A d = M^{-1} r (end of Section 2.2).  Stops when the
// preconditioned residual estimate falls below rtol times its initial value.
// r is not modified; d receives the correction.
int gmres_lp(LinCtx &c, const float *r, float *d, int m, double rtol, int max_restarts, int *its)
{
    const int64_t n = c.n;
    HIPCHK(launch_fill_f32(d, 0.0f, n, c.s));
    CHK(apply_prec(c, r, c.z));
    double beta0 = 0.0;
    CHK(norm32(c, c.z, &beta0));
    *its = 0;
    if (!(beta0 > 0.0)) return 0;
    std::vector<double> Hm((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), hcol(m + 2), yv(m);
    double beta = beta0;
    for (int rs = 0; rs < max_restarts; ++rs) {
        if (rs > 0) CHK(norm32(c, c.z, &beta));
        if (beta <= rtol * beta0) break;
        HIPCHK(launch_scal_copy_f32(n, c.V, c.z, 1.0 / beta, c.s));
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int k_used = 0;
        bool conv = false;
        for (int j = 0; j < m; ++j) {
            CHK(lin_matvec(c, c.V + (int64_t)j * c.ldv, c.av));
            CHK(apply_prec(c, c.av, c.w));
            HIPCHK(launch_mgs(n, c.V, c.ldv, j, c.w, c.H, c.s));
            HIPCHK(hipMemcpyAsync(hcol.data(), c.H, (size_t)(j + 2) * sizeof(double),
                                  hipMemcpyDeviceToHost, c.s));
            HIPCHK(hipStreamSynchronize(c.s));
            for (int i = 0; i < j; ++i) {  // previous Givens rotations
                const double t = cs[i] * hcol[i] + sn[i] * hcol[i + 1];
                hcol[i + 1] = -sn[i] * hcol[i] + cs[i] * hcol[i + 1];
                hcol[i] = t;
            }
            const double den = std::hypot(hcol[j], hcol[j + 1]);
            if (den == 0.0) { cs[j] = 1.0; sn[j] = 0.0; }
            else { cs[j] = hcol[j] / den; sn[j] = hcol[j + 1] / den; }
            hcol[j] = cs[j] * hcol[j] + sn[j] * hcol[j + 1];
            hcol[j + 1] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            for (int i = 0; i <= j; ++i) Hm[(size_t)i * m + j] = hcol[i];
            k_used = j + 1;
            (*its)++;
            if (std::fabs(g[j + 1]) <= rtol * beta0) { conv = true; break; }
            if (hcol[j] == 0.0) break;
        }
        for (int i = k_used - 1; i >= 0; --i) {
            double acc = g[i];
            for (int q = i + 1; q < k_used; ++q) acc -= Hm[(size_t)i * m + q] * yv[q];
            yv[i] = Hm[(size_t)i * m + i] != 0.0 ? acc / Hm[(size_t)i * m + i] : 0.0;
        }
        HIPCHK(hipMemcpyAsync(c.ydev, yv.data(), (size_t)k_used * sizeof(double),
                              hipMemcpyHostToDevice, c.s));
        HIPCHK(launch_krylov_update(n, c.V, c.ldv, k_used, c.ydev, d, c.s));
        if (conv || rs + 1 == max_restarts) break;
        // z = M^{-1} (r - A d) for the next cycle
        CHK(lin_resid(c, d, r, c.av, c.part));
        CHK(apply_prec(c, c.av, c.z));
    }
    HIPCHK(hipStreamSynchronize(c.s));
    return 0;
}

// Refinement loop shared by IR and GMRES-IR (Section 2.2, policy of Section
// 3.1): r = b - A u; repeat { d = correction(r); u += d; r = b - A u } until
// ||r|| < tol ||b|| (success), the sweep cap, or ||r|| grows (failure: the
// previous, best, iterate is restored).
// nb_pre (optional): ||b||, with u = 0 and r = b already in place (queued by
// the caller ahead of the factorisation).
int refine(LinCtx &c, const float *b, float *u, double tol, int max_sweeps, bool zero_start,
           bool gmres, int m, double gtol, int max_restarts, LinOut *o,
           const double *nb_pre = nullptr)
{
    double nb = 0.0;
    if (nb_pre) nb = *nb_pre;
    else CHK(norm32(c, b, &nb));
    double rn = nb;
    if (nb_pre) {
        // u = 0 and r = b were set with ||b||
    } else if (zero_start) {
        HIPCHK(launch_fill_f32(u, 0.0f, c.n, c.s));
        HIPCHK(launch_vcopy_f32(c.n, c.r, b, c.s));
    } else {
        CHK(lin_resid(c, u, b, c.r, c.part));
        CHK(norm32(c, c.r, &rn));
    }
    o->sweeps = 0;
    o->inner = 0;
    o->failed = false;
    while (!(rn < tol * nb) && o->sweeps < max_sweeps) {
        if (gmres) {
            int its = 0;
            CHK(gmres_lp(c, c.r, c.d, m, gtol, max_restarts, &its));
            o->inner += its;
        } else {
            if (c.ir_half && rn > 0.0) CHK(apply_prec_half(c, c.r, rn, c.d));
            else CHK(apply_prec(c, c.r, c.d));
            o->inner += 1;
        }
        HIPCHK(launch_vcopy_f32(c.n, c.uprev, u, c.s));
        HIPCHK(launch_axpy_f32(c.n, u, c.d, 1.0f, c.s));
        CHK(lin_resid(c, u, b, c.r, c.part));
        double rnew = 0.0;
        CHK(norm32(c, c.r, &rnew));
        o->sweeps++;
        if (!(rnew <= rn)) {  // growth (or NaN): keep the previous iterate
            HIPCHK(launch_vcopy_f32(c.n, u, c.uprev, c.s));
            o->failed = true;
            break;
        }
        rn = rnew;
    }
    if (!o->failed && !(rn < tol * nb)) o->failed = true;
    o->rel = nb > 0 ? rn / nb : 0.0;
    return 0;
}

}  // namespace

// ===================================================================== C ABI
extern "C" {

N3P_API const char *n3p_status_str(int st)
{
    switch (st) {
    case N3P_OK: return "N3P_OK";
    case N3P_NOT_CONVERGED: return "N3P_NOT_CONVERGED";
    case N3P_E_INVALID: return "N3P_E_INVALID";
    case N3P_E_NOMEM: return "N3P_E_NOMEM";
    case N3P_E_SINGULAR: return "N3P_E_SINGULAR";
    case N3P_E_NONFINITE: return "N3P_E_NONFINITE";
    case N3P_E_CALLBACK: return "N3P_E_CALLBACK";
    case N3P_E_HIP: return "N3P_E_HIP";
    case N3P_E_TIMEOUT: return "N3P_E_TIMEOUT";
    case N3P_E_PIVOTING: return "N3P_E_PIVOTING";
    default: return "N3P_UNKNOWN";
    }
}

N3P_API const char *n3p_version(void) { return "n3p 0.1.0 gfx950"; }

N3P_API void n3p_default_options(n3p_options *o)
{
    if (!o) return;
    o->tau_r = 1e-10;
    o->tau_a = 0.0;
    o->tau_abs_override = -1.0;
    o->eta = 1e-6;
    o->maxit = 20;
    o->max_ir_sweeps = 10;
    o->gmres_restart = 20;
    o->gmres_tol = 1e-4;
    o->gmres_max_restarts = 10;
    o->scale_mode = N3P_SCALE_AUTO;
    o->timing = 1;
    o->fft_residual = 0;
    o->matrix_free = 0;
    o->ir_scaled_half = 0;
}

N3P_API int n3p_problem_heq(n3p_problem *p, int64_t n, double c)
{
    if (!p || n < 1 || !(c >= 0.0) || c > 1.0) return N3P_E_INVALID;
    std::memset(p, 0, sizeof(*p));
    p->kind = 0;
    p->n = n;
    p->c = c;
    return N3P_OK;
}

N3P_API int n3p_problem_dense_tanh(n3p_problem *p, int64_t n, const double *A, int64_t lda,
                                   const double *b)
{
    if (!p || n < 1 || !A || !b || lda < n) return N3P_E_INVALID;
    std::memset(p, 0, sizeof(*p));
    p->kind = 1;
    p->n = n;
    p->A = A;
    p->b = b;
    p->lda = lda;
    return N3P_OK;
}

N3P_API int n3p_problem_callbacks(n3p_problem *p, int64_t n, n3p_residual_fn F, n3p_jacobian_fn J,
                                  void *ctx)
{
    if (!p || n < 1 || !F || !J) return N3P_E_INVALID;
    std::memset(p, 0, sizeof(*p));
    p->kind = 2;
    p->n = n;
    p->residual = F;
    p->jacobian = J;
    p->ctx = ctx;
    return N3P_OK;
}

static int opt_m(const n3p_options *o)
{
    return o ? std::max(1, std::min(64, o->gmres_restart)) : 20;
}

static int fft_mode(const n3p_options *opt)
{
    return opt ? ((opt->fft_residual ? 1 : 0) | (opt->matrix_free ? 2 : 0)) : 0;
}

N3P_API size_t n3p_workspace_size(int64_t n, int lu_prec, int ls, const n3p_options *opt)
{
    if (n < 1 || !valid_prec(lu_prec) || ls < N3P_IR || ls > N3P_DIRECT) return 0;
    if (fft_mode(opt) && !fft_length(n)) return 0;
    return solve_layout(n, lu_prec, ls, opt_m(opt), fft_mode(opt), nullptr, nullptr);
}

static int eval_residual(const n3p_problem *p, const SolveWs &w, const double *x, hipStream_t s)
{
    switch (p->kind) {
    case 0:
        if (w.fftres)
            HIPCHK(launch_hk_residual(w.n, w.L, p->c, x, w.tw, w.Hh, w.t1, w.t2, w.W, w.F, w.D, s));
        else
            HIPCHK(launch_heq_residual(w.n, p->c, x, w.h, w.F, w.D, s));
        break;
    case 1: HIPCHK(launch_dense_tanh_residual(w.n, p->A, p->lda, p->b, x, w.F, w.part, s)); break;
    case 2:
        if (p->residual(p->ctx, x, w.F, w.n, (void *)s) != 0) return N3P_E_CALLBACK;
        break;
    default: return N3P_E_INVALID;
    }
    HIPCHK(launch_nrm2_f64(w.n, w.F, w.part, w.scal, s));
    return 0;
}

// Build J (FP32) and the factorisation copy in w.f.A; target_log2 < 0 => no scaling
static int build_jacobian(const n3p_problem *p, const SolveWs &w, const double *x, float tl,
                          bool scale, hipStream_t s)
{
    float *cs = scale ? w.colscale : nullptr;
    switch (p->kind) {
    case 0:
        // the row factors go to the partial-sum scratch (n doubles), which
        // nothing reads between the residual's norm and the linear solve
        HIPCHK(launch_heq_jac_round(w.prec, w.n, w.Np, p->c, w.D, w.h, w.J, w.n, w.f.A, w.Np, cs,
                                    tl, w.f.flags, w.part, s));
        return 0;
    case 1:
        if (w.prec == N3P_FP64) {  // the FP64 factorisation takes the unrounded Jacobian
            HIPCHK(launch_dense_tanh_jacobian_f64(w.n, w.Np, p->A, p->lda, x, w.J, w.n,
                                                  (double *)w.f.A, w.Np, s));
            return 0;
        }
        HIPCHK(launch_dense_tanh_jacobian(w.n, p->A, p->lda, x, w.J, w.n, s));
        break;
    case 2:
        if (p->jacobian(p->ctx, x, w.J, w.n, w.n, (void *)s) != 0) return N3P_E_CALLBACK;
        break;
    default: return N3P_E_INVALID;
    }
    HIPCHK(launch_round_scale(w.prec, w.n, w.Np, w.J, w.n, w.f.A, w.Np, cs, tl, w.f.flags, s));
    return 0;
}

N3P_API int n3p_solve(const n3p_problem *p, double *x, int lu_prec, int ls,
                      const n3p_options *opt_in, void *ws, size_t ws_bytes, void *stream,
                      n3p_report *rep)
{
    n3p_options opt;
    if (opt_in) opt = *opt_in;
    else n3p_default_options(&opt);
    if (rep) std::memset(rep, 0, sizeof(*rep));
    if (!p || !x || !ws || !valid_prec(lu_prec) || ls < N3P_IR || ls > N3P_DIRECT || p->n < 1 ||
        opt.maxit < 0 || opt.maxit >= N3P_MAX_HIST || opt.max_ir_sweeps < 1 ||
        (opt.ir_scaled_half != 0 && (opt.ir_scaled_half != 1 || ls != N3P_IR)))
        return N3P_E_INVALID;
    const int m = opt_m(&opt);
    const int fm = fft_mode(&opt);
    if (fm && (p->kind != 0 || !fft_length(p->n))) return N3P_E_INVALID;
    const size_t need = solve_layout(p->n, lu_prec, ls, m, fm, nullptr, nullptr);
    if (ws_bytes < need) return N3P_E_NOMEM;
    char *base = (char *)(((uintptr_t)ws + ALIGN - 1) / ALIGN * ALIGN);
    SolveWs w;
    solve_layout(p->n, lu_prec, ls, m, fm, &w, base);
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = w.n;

    float t_jac = 0, t_getrf = 0, t_solve = 0, t_resid = 0;
    // per-phase times: timestamps on the GPU timeline (no host wait), read
    // once when the solve ends
    int tslot = 0;
    std::vector<std::pair<int, float *>> tpairs;
    auto tstart = [&]() -> int {
        if (opt.timing && tslot + 2 <= NSTAMPS) HIPCHK(launch_stamp(w.stamps + tslot, s));
        return 0;
    };
    auto tstop = [&](float *acc) -> int {
        if (opt.timing && tslot + 2 <= NSTAMPS) {
            HIPCHK(launch_stamp(w.stamps + tslot + 1, s));
            tpairs.emplace_back(tslot, acc);
            tslot += 2;
        }
        return 0;
    };
    // the two events bracketing the solve; the guard destroys them on every
    // return path, early error returns included
    struct EventPair {
        hipEvent_t a = nullptr, b = nullptr;
        ~EventPair()
        {
            // nothing to report from a destructor: a failed destroy leaves the
            // error to the next call that checks
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } ev;
    HIPCHK(hipEventCreate(&ev.a));
    HIPCHK(hipEventCreate(&ev.b));
    HIPCHK(hipEventRecord(ev.a, s));

    Epoch epoch;
    HIPCHK(launch_fill_i32(w.sync, 0, (int64_t)trsv_sync_ints(w.Np), s));
    HIPCHK(launch_fill_i32(w.f.flags, 0, NFLAGS, s));
    if (p->kind == 0) HIPCHK(launch_hinv(n, w.h, s));
    if (w.L) HIPCHK(launch_hk_setup(n, w.L, w.tw, w.Hh, w.t1, w.t2, s));

    int status = N3P_OK;
    double fn = 0.0;
    CHK(tstart());
    {
        int st = eval_residual(p, w, x, s);
        if (st) return st;
    }
    CHK(d2h_double(w.scal, &fn, s));
    CHK(tstop(&t_resid));
    if (!std::isfinite(fn)) return N3P_E_NONFINITE;
    const double f0 = fn;
    const double tau = opt.tau_abs_override >= 0 ? opt.tau_abs_override : opt.tau_r * fn + opt.tau_a;
    if (rep) {
        rep->f0 = f0;
        rep->resid_rel[0] = 1.0;
    }
    int its = 0;
    const bool fp16 = lu_prec == N3P_FP16;
    const bool want_scale = fp16 && opt.scale_mode == N3P_SCALE_AUTO;
    LinCtx lc{};
    lc.prec = lu_prec;
    lc.n = n;
    lc.A = w.J;
    lc.lda = n;
    lc.LU = w.f.A;
    lc.ldlu = w.Np;
    lc.y = w.y;
    lc.xs = w.xs;
    lc.z = w.z;
    lc.ir_half = opt.ir_scaled_half == 1;
    lc.av = w.av;
    lc.w = w.w;
    lc.V = w.V;
    lc.ldv = w.Np;
    lc.r = w.r;
    lc.d = w.d;
    lc.uprev = w.uprev;
    lc.part = w.part;
    lc.scal = w.scal + 1;
    lc.H = w.H;
    lc.ydev = w.ydev;
    lc.sync = w.sync;
    lc.flags = w.f.flags;
    lc.epoch = &epoch;
    lc.s = s;
    if (w.mf) {
        lc.tw = w.tw;
        lc.Hh = w.Hh;
        lc.t1 = w.t1;
        lc.t2 = w.t2;
        lc.W = w.W;
        lc.D = w.D;
        lc.c = p->c;
        lc.L = w.L;
    }

    // FP16 column targets: column max in [256, 512), 2^7 headroom below 65504.
    // A factorisation that overflows is redone with targets 2^6 lower, and the
    // lower targets are kept for the rest of the solve (the Jacobian changes
    // little from one Newton step to the next, so its growth does too).  The
    // pivoting path starts at the lower targets: a matrix that needs row
    // interchanges is not diagonally dominant, so its elimination can grow
    // (a diagonally dominant one grows at most twofold and never pivots).
    float tl = 9.0f;
    // IR and GMRES-IR: b = -F/||F||, ||b||, u = 0 and r = b depend on F only,
    // so they are queued ahead of the Jacobian and the factorisation, and
    // ||b|| comes back in the factorisation's flag read (no extra host wait)
    const bool pre_rhs = ls != N3P_DIRECT;
    while (fn > tau && its < opt.maxit) {
        double nb_pre = 0.0;
        if (pre_rhs) {
            HIPCHK(launch_rhs_unit(n, w.Np, w.F, w.scal, w.b, s));
            HIPCHK(launch_nrm2_f32(n, w.b, w.part, lc.scal, s));
            HIPCHK(launch_fill_f32(w.u, 0.0f, n, s));
            HIPCHK(launch_vcopy_f32(n, lc.r, w.b, s));
        }
        // --- J = F'(x) stored FP32, J_h = I_s^h(J) (column scaled for FP16)
        bool scaled = want_scale;
        FactorResult fr;
        for (int attempt = 0; attempt < 2; ++attempt) {
            CHK(tstart());
            CHK(build_jacobian(p, w, x, tl, scaled, s));
            CHK(tstop(&t_jac));
            CHK(tstart());
            auto refill = [&]() -> int {
                if (want_scale && scaled && tl > 3.0f) tl -= 6.0f;
                // the FP64 factorisation of a built-in problem takes the FP64
                // Jacobian again (J holds only its FP32 rounding)
                if ((w.prec == N3P_FP64 || w.mf) && p->kind != 2)
                    return build_jacobian(p, w, x, tl, scaled, s);
                HIPCHK(launch_round_scale(w.prec, n, w.Np, w.J, n, w.f.A, w.Np,
                                          scaled ? w.colscale : nullptr, tl, w.f.flags, s));
                return 0;
            };
            CHK(getrf_run(w.f, s, refill, &fr, pre_rhs ? lc.scal : nullptr, &nb_pre));
            CHK(tstop(&t_getrf));
            if (fr.timeout) return N3P_E_TIMEOUT;
            if (fr.nonfinite && want_scale && attempt == 0 && tl > 3.0f) {
                tl -= 6.0f;  // retry with the column targets 2^6 lower
                continue;
            }
            break;
        }
        if (fr.nonfinite) { status = N3P_E_NONFINITE; break; }
        if (fr.info > 0) { status = N3P_E_SINGULAR; break; }
        lc.perm = fr.pivoted ? w.f.perm : nullptr;
        lc.colscale = (fp16 && scaled) ? w.colscale : nullptr;

        // --- step: J u = -F/||F|| (eq. (2.17)); s = ||F|| u (eq. (2.18))
        CHK(tstart());
        LinOut lo;
        const double *fnd = w.scal;  // device ||F||
        if (lu_prec == N3P_FP64 && ls == N3P_DIRECT) {
            // Newton with a double-precision factorisation: one FP64 solve
            HIPCHK(launch_rhs_unit_f64(n, w.Np, w.F, fnd, w.b64, s));
            HIPCHK(launch_trsv_lower_f64(n, (const double *)w.f.A, w.Np, lc.perm, w.b64, w.y64,
                                         w.sync, epoch.next(), w.f.flags, s));
            HIPCHK(launch_trsv_upper_f64(n, (const double *)w.f.A, w.Np, w.y64, w.x64, w.sync,
                                         epoch.next(), w.f.flags, s));
            lo.sweeps = 1;
            lo.inner = 1;
            HIPCHK(launch_newton_update_f64(n, x, fnd, w.x64, s));
        } else {
            if (!pre_rhs) HIPCHK(launch_rhs_unit(n, w.Np, w.F, fnd, w.b, s));
            if (ls == N3P_DIRECT) {
                CHK(apply_prec(lc, w.b, w.u));
                lo.sweeps = 1;
                lo.inner = 1;
                CHK(lin_resid(lc, w.u, w.b, w.r, w.part));
                double rn = 0, nb = 0;
                CHK(norm32(lc, w.r, &rn));
                CHK(norm32(lc, w.b, &nb));
                lo.rel = nb > 0 ? rn / nb : 0;
            } else {
                CHK(refine(lc, w.b, w.u, opt.eta, opt.max_ir_sweeps, true, ls == N3P_GMRES_IR, m,
                           opt.gmres_tol, opt.gmres_max_restarts, &lo, &nb_pre));
            }
            HIPCHK(launch_newton_update_f32(n, x, fnd, w.u, s));
        }
        CHK(tstop(&t_solve));
        {
            int h[NFLAGS];
            CHK(read_flags(w.f, s, h));
            if (h[FLAG_TIMEOUT]) return N3P_E_TIMEOUT;
        }
        // --- F(x)
        CHK(tstart());
        {
            int st = eval_residual(p, w, x, s);
            if (st) return st;
        }
        CHK(d2h_double(w.scal, &fn, s));
        CHK(tstop(&t_resid));
        if (rep) {
            rep->lin_its[its] = ls == N3P_GMRES_IR ? lo.inner : lo.sweeps;
            rep->lin_outer[its] = lo.sweeps;
            rep->lin_fail[its] = lo.failed ? 1 : 0;
            rep->lin_rel[its] = lo.rel;
            rep->pivoted[its] = fr.pivoted ? 1 : 0;
        }
        ++its;
        if (rep) rep->resid_rel[its] = fn / f0;
        if (!std::isfinite(fn)) { status = N3P_E_NONFINITE; break; }
    }
    if (status == N3P_OK && fn > tau) status = N3P_NOT_CONVERGED;
    HIPCHK(hipEventRecord(ev.b, s));
    HIPCHK(hipEventSynchronize(ev.b));
    float tot = 0;
    HIPCHK(hipEventElapsedTime(&tot, ev.a, ev.b));
    if (tslot > 0) {
        std::vector<uint64_t> st((size_t)tslot);
        HIPCHK(hipMemcpyAsync(st.data(), w.stamps, (size_t)tslot * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (const auto &pr : tpairs)
            *pr.second += (float)((double)(st[pr.first + 1] - st[pr.first]) * STAMP_MS_PER_TICK);
    }
    if (rep) {
        rep->status = status;
        rep->its = its;
        rep->fnorm = fn;
        rep->ms_jac = t_jac;
        rep->ms_getrf = t_getrf;
        rep->ms_solve = t_solve;
        rep->ms_resid = t_resid;
        rep->ms_total = tot;
    }
    return status;
}

// ------------------------------------------------------------- components
N3P_API size_t n3p_getrf_workspace_size(int64_t n, int prec)
{
    if (n < 1 || !valid_prec(prec)) return 0;
    Bump b;
    factor_bytes(prec, padded(n), b, nullptr, nullptr);
    b.take(trsv_sync_ints(padded(n)) * 4);
    const int64_t Np = padded(n);
    const size_t vs = prec == N3P_FP64 ? 8 : 4;
    b.take((size_t)Np * vs);  // y
    b.take((size_t)Np * vs);  // xs
    b.take((size_t)Np * vs);  // b copy
    return b.off + ALIGN;
}

static void getrs_layout(int64_t n, int prec, char *base, FactorWs *f, int **sync, void **y,
                         void **xs, void **bc)
{
    Bump b;
    factor_bytes(prec, padded(n), b, f, base);
    size_t os = b.take(trsv_sync_ints(padded(n)) * 4);
    const int64_t Np = padded(n);
    const size_t vs = prec == N3P_FP64 ? 8 : 4;
    size_t oy = b.take((size_t)Np * vs), ox = b.take((size_t)Np * vs), ob = b.take((size_t)Np * vs);
    *sync = (int *)(base + os);
    *y = base + oy;
    *xs = base + ox;
    *bc = base + ob;
}

N3P_API int n3p_getrf(int prec, int64_t n, void *A, int64_t lda, int32_t *ipiv, int *info,
                      void *ws, size_t ws_bytes, void *stream)
{
    if (!valid_prec(prec) || n < 1 || !A || lda < n || !ipiv || !ws) return N3P_E_INVALID;
    if (ws_bytes < n3p_getrf_workspace_size(n, prec)) return N3P_E_NOMEM;
    char *base = (char *)(((uintptr_t)ws + ALIGN - 1) / ALIGN * ALIGN);
    FactorWs f;
    int *sync;
    void *y, *xs, *bc;
    getrs_layout(n, prec, base, &f, &sync, &y, &xs, &bc);
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(launch_pad_copy_in(prec, n, f.Np, A, lda, f.A, s));
    auto refill = [&]() -> int {
        HIPCHK(launch_pad_copy_in(prec, n, f.Np, A, lda, f.A, s));
        return 0;
    };
    FactorResult fr;
    CHK(getrf_run(f, s, refill, &fr));
    if (fr.timeout) return N3P_E_TIMEOUT;
    HIPCHK(launch_pad_copy_out(prec, n, f.Np, f.A, A, lda, s));
    HIPCHK(hipMemcpyAsync(ipiv, f.ipiv, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    int inf = fr.info;
    if (inf > n) inf = 0;
    if (fr.nonfinite) inf = -1;
    if (info) *info = inf;
    return inf > 0 ? N3P_E_SINGULAR : (inf < 0 ? N3P_E_NONFINITE : N3P_OK);
}

N3P_API int n3p_getrs(int prec, int64_t n, const void *LU, int64_t lda, const int32_t *ipiv, void *b,
                      void *ws, size_t ws_bytes, void *stream)
{
    if (!valid_prec(prec) || n < 1 || !LU || lda < n || !ipiv || !b || !ws) return N3P_E_INVALID;
    if (ws_bytes < n3p_getrf_workspace_size(n, prec)) return N3P_E_NOMEM;
    char *base = (char *)(((uintptr_t)ws + ALIGN - 1) / ALIGN * ALIGN);
    FactorWs f;
    int *sync;
    void *y, *xs, *bc;
    getrs_layout(n, prec, base, &f, &sync, &y, &xs, &bc);
    hipStream_t s = (hipStream_t)stream;
    // permutation from the interchange list (host; O(n))
    std::vector<int32_t> ip((size_t)n), pm((size_t)n);
    HIPCHK(hipMemcpyAsync(ip.data(), ipiv, (size_t)n * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int64_t k = 0; k < n; ++k) pm[k] = (int32_t)k;
    for (int64_t k = 0; k < n; ++k) {
        if (ip[k] < k || ip[k] >= n) return N3P_E_INVALID;
        std::swap(pm[k], pm[ip[k]]);
    }
    HIPCHK(hipMemcpyAsync(f.perm, pm.data(), (size_t)n * 4, hipMemcpyHostToDevice, s));
    HIPCHK(launch_fill_i32(sync, 0, (int64_t)trsv_sync_ints(padded(n)), s));
    HIPCHK(launch_fill_i32(f.flags, 0, NFLAGS, s));
    const size_t vs = prec == N3P_FP64 ? 8 : 4;
    HIPCHK(hipMemcpyAsync(bc, b, (size_t)n * vs, hipMemcpyDeviceToDevice, s));
    if (prec == N3P_FP64) {
        HIPCHK(launch_trsv_lower_f64(n, (const double *)LU, lda, f.perm, (const double *)bc,
                                     (double *)y, sync, 1, f.flags, s));
        HIPCHK(launch_trsv_upper_f64(n, (const double *)LU, lda, (const double *)y, (double *)b,
                                     sync, 2, f.flags, s));
    } else {
        HIPCHK(launch_trsv_lower(prec, n, LU, lda, f.perm, (const float *)bc, (float *)y, sync, 1,
                                 f.flags, s));
        HIPCHK(launch_trsv_upper(prec, n, LU, lda, (const float *)y, nullptr, (float *)b, sync, 2,
                                 f.flags, s));
    }
    int h[NFLAGS];
    CHK(read_flags(f, s, h));
    if (h[FLAG_TIMEOUT]) return N3P_E_TIMEOUT;
    return N3P_OK;
}

static size_t lin_layout(int64_t n, int m, char *base, LinCtx *c, int32_t **perm)
{
    Bump b;
    const int64_t Np = padded(n);
    const size_t vec = (size_t)Np * 4;
    float **vs[] = {&c->y, &c->xs, &c->r, &c->d, &c->uprev, &c->z, &c->av, &c->w};
    for (auto v : vs) {
        size_t o = b.take(vec);
        if (base) *v = (float *)(base + o);
    }
    size_t oV = b.take((size_t)(m + 1) * vec);
    size_t oH = b.take((size_t)(m + 2) * 8);
    size_t oY = b.take((size_t)(m + 1) * 8);
    size_t oP = b.take(part_len_for(n) * 8);
    size_t oS = b.take(64 * 8);
    size_t oSy = b.take(trsv_sync_ints(Np) * 4);
    size_t oF = b.take(NFLAGS * 4);
    size_t oPm = b.take((size_t)Np * 4);
    if (base) {
        c->V = (float *)(base + oV);
        c->ldv = Np;
        c->H = (double *)(base + oH);
        c->ydev = (double *)(base + oY);
        c->part = (double *)(base + oP);
        c->scal = (double *)(base + oS);
        c->sync = (int *)(base + oSy);
        c->flags = (int *)(base + oF);
        *perm = (int32_t *)(base + oPm);
    }
    return b.off + ALIGN;
}

N3P_API size_t n3p_linsolve_workspace_size(int64_t n, int m)
{
    if (n < 1) return 0;
    m = std::max(1, std::min(64, m));
    LinCtx c{};
    int32_t *p = nullptr;
    return lin_layout(n, m, nullptr, &c, &p);
}

static int lin_common(int prec, int64_t n, const float *A, int64_t lda, const void *LU,
                      int64_t ldlu, const int32_t *ipiv, const float *colscale, int m, void *ws,
                      size_t ws_bytes, hipStream_t s, LinCtx *c, Epoch *ep)
{
    if (!valid_prec(prec) || n < 1 || !A || lda < n || !LU || ldlu < n || !ws) return N3P_E_INVALID;
    if (ws_bytes < n3p_linsolve_workspace_size(n, m)) return N3P_E_NOMEM;
    char *base = (char *)(((uintptr_t)ws + ALIGN - 1) / ALIGN * ALIGN);
    int32_t *perm_buf = nullptr;
    lin_layout(n, m, base, c, &perm_buf);
    HIPCHK(launch_fill_i32(c->sync, 0, (int64_t)trsv_sync_ints(padded(n)), s));
    HIPCHK(launch_fill_i32(c->flags, 0, NFLAGS, s));
    c->perm = nullptr;
    if (ipiv) {
        std::vector<int32_t> ip((size_t)n), pm((size_t)n);
        HIPCHK(hipMemcpyAsync(ip.data(), ipiv, (size_t)n * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        bool ident = true;
        for (int64_t k = 0; k < n; ++k) pm[k] = (int32_t)k;
        for (int64_t k = 0; k < n; ++k) {
            if (ip[k] < k || ip[k] >= n) return N3P_E_INVALID;
            if (ip[k] != k) ident = false;
            std::swap(pm[k], pm[ip[k]]);
        }
        if (!ident) {
            HIPCHK(hipMemcpyAsync(perm_buf, pm.data(), (size_t)n * 4, hipMemcpyHostToDevice, s));
            HIPCHK(hipStreamSynchronize(s));
            c->perm = perm_buf;
        }
    }
    c->prec = prec;
    c->n = n;
    c->A = A;
    c->lda = lda;
    c->LU = LU;
    c->ldlu = ldlu;
    c->colscale = colscale;
    c->epoch = ep;
    c->s = s;
    return 0;
}

N3P_API size_t n3p_heq_fft_workspace_size(int64_t n)
{
    const int L = n >= 1 ? fft_length(n) : 0;
    return L ? (size_t)5 * L * sizeof(double2) + 5 * ALIGN : 0;
}

namespace {
struct FftWs {
    int L = 0;
    double2 *tw = nullptr, *H = nullptr, *t1 = nullptr, *t2 = nullptr, *W = nullptr;
};
int fft_ws(int64_t n, void *ws, size_t bytes, FftWs *f)
{
    const size_t need = n3p_heq_fft_workspace_size(n);
    if (!need) return N3P_E_INVALID;
    if (!ws || bytes < need) return N3P_E_NOMEM;
    Bump b;
    char *base = (char *)(((uintptr_t)ws + ALIGN - 1) / ALIGN * ALIGN);
    f->L = fft_length(n);
    const size_t sz = (size_t)f->L * sizeof(double2);
    f->tw = (double2 *)(base + b.take(sz));
    f->H = (double2 *)(base + b.take(sz));
    f->t1 = (double2 *)(base + b.take(sz));
    f->t2 = (double2 *)(base + b.take(sz));
    f->W = (double2 *)(base + b.take(sz));
    return 0;
}
}  // namespace

N3P_API int n3p_heq_residual_fft(int64_t n, double c, const double *x, double *F, double *D,
                                 void *ws, size_t ws_bytes, void *stream)
{
    if (n < 1 || !x || !F) return N3P_E_INVALID;
    FftWs f;
    CHK(fft_ws(n, ws, ws_bytes, &f));
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(launch_hk_setup(n, f.L, f.tw, f.H, f.t1, f.t2, s));
    HIPCHK(launch_hk_residual(n, f.L, c, x, f.tw, f.H, f.t1, f.t2, f.W, F, D, s));
    return 0;
}

N3P_API int n3p_heq_jv(int64_t n, double c, const double *D, const float *v, float *y, void *ws,
                       size_t ws_bytes, void *stream)
{
    if (n < 1 || !D || !v || !y) return N3P_E_INVALID;
    FftWs f;
    CHK(fft_ws(n, ws, ws_bytes, &f));
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(launch_hk_setup(n, f.L, f.tw, f.H, f.t1, f.t2, s));
    HIPCHK(launch_hk_jv(n, n, f.L, c, D, v, nullptr, y, f.tw, f.H, f.t1, f.t2, f.W, s));
    return 0;
}

N3P_API int n3p_ir(int prec, int64_t n, const float *A, int64_t lda, const void *LU, int64_t ldlu,
                   const int32_t *ipiv, const float *colscale, const float *b, float *u, double tol,
                   int max_sweeps, int *sweeps, int *failed, double *rel_res, void *ws,
                   size_t ws_bytes, void *stream)
{
    if (!b || !u || max_sweeps < 1) return N3P_E_INVALID;
    hipStream_t s = (hipStream_t)stream;
    LinCtx c{};
    Epoch ep;
    CHK(lin_common(prec, n, A, lda, LU, ldlu, ipiv, colscale, 1, ws, ws_bytes, s, &c, &ep));
    LinOut o;
    CHK(refine(c, b, u, tol, max_sweeps, false, false, 1, 0.0, 1, &o));
    int h[NFLAGS];
    HIPCHK(hipMemcpyAsync(h, c.flags, sizeof(h), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (h[FLAG_TIMEOUT]) return N3P_E_TIMEOUT;
    if (sweeps) *sweeps = o.sweeps;
    if (failed) *failed = o.failed ? 1 : 0;
    if (rel_res) *rel_res = o.rel;
    return N3P_OK;
}

N3P_API int n3p_ir_scaled_half(int prec, int64_t n, const float *A, int64_t lda, const void *LU,
                               int64_t ldlu, const int32_t *ipiv, const float *colscale,
                               const float *b, float *u, double tol, int max_sweeps, int *sweeps,
                               int *failed, double *rel_res, void *ws, size_t ws_bytes,
                               void *stream)
{
    if (!b || !u || max_sweeps < 1) return N3P_E_INVALID;
    hipStream_t s = (hipStream_t)stream;
    LinCtx c{};
    Epoch ep;
    CHK(lin_common(prec, n, A, lda, LU, ldlu, ipiv, colscale, 1, ws, ws_bytes, s, &c, &ep));
    c.ir_half = true;
    LinOut o;
    CHK(refine(c, b, u, tol, max_sweeps, false, false, 1, 0.0, 1, &o));
    int h[NFLAGS];
    HIPCHK(hipMemcpyAsync(h, c.flags, sizeof(h), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (h[FLAG_TIMEOUT]) return N3P_E_TIMEOUT;
    if (sweeps) *sweeps = o.sweeps;
    if (failed) *failed = o.failed ? 1 : 0;
    if (rel_res) *rel_res = o.rel;
    return N3P_OK;
}

N3P_API int n3p_gmres_ir(int prec, int64_t n, const float *A, int64_t lda, const void *LU,
                         int64_t ldlu, const int32_t *ipiv, const float *colscale, const float *b,
                         float *u, double tol, int max_outer, int m, double gmres_tol, int *sweeps,
                         int *gmres_its, int *failed, double *rel_res, void *ws, size_t ws_bytes,
                         void *stream)
{
    if (!b || !u || max_outer < 1 || m < 1 || m > 64) return N3P_E_INVALID;
    hipStream_t s = (hipStream_t)stream;
    LinCtx c{};
    Epoch ep;
    CHK(lin_common(prec, n, A, lda, LU, ldlu, ipiv, colscale, m, ws, ws_bytes, s, &c, &ep));
    LinOut o;
    CHK(refine(c, b, u, tol, max_outer, false, true, m, gmres_tol, 10, &o));
    int h[NFLAGS];
    HIPCHK(hipMemcpyAsync(h, c.flags, sizeof(h), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (h[FLAG_TIMEOUT]) return N3P_E_TIMEOUT;
    if (sweeps) *sweeps = o.sweeps;
    if (gmres_its) *gmres_its = o.inner;
    if (failed) *failed = o.failed ? 1 : 0;
    if (rel_res) *rel_res = o.rel;
    return N3P_OK;
}

N3P_API int n3p_gemv_resid_f32(int64_t n, const float *A, int64_t lda, const float *u,
                               const float *b, float *r, void *ws, size_t ws_bytes, void *stream)
{
    if (n < 1 || !A || lda < n || !u || !b || !r || !ws) return N3P_E_INVALID;
    if (ws_bytes < part_len_for(n) * 8) return N3P_E_NOMEM;
    HIPCHK(launch_gemv_resid(n, A, lda, u, b, r, (double *)ws, (hipStream_t)stream));
    return N3P_OK;
}

N3P_API int n3p_gemv_resid_f32_noalloc(int64_t n, const float *A, int64_t lda, const float *u,
                                       const float *b, float *r, void *stream)
{
    if (n < 1 || n > N3P_GEMV_NOALLOC_MAX_N || !A || lda < n || !u || !b || !r)
        return N3P_E_INVALID;
    HIPCHK(launch_gemv_resid_noalloc(n, A, lda, u, b, r, (hipStream_t)stream));
    return N3P_OK;
}

N3P_API int n3p_mfma_rate_probe(int prec, int blocks, int iters, float *out, double *flops,
                                void *stream)
{
    if ((prec != N3P_FP16 && prec != N3P_BF16) || blocks < 1 || iters < 1 || iters > (1 << 20) ||
        !out || !flops)
        return N3P_E_INVALID;
    HIPCHK(launch_mfma_rate(prec, blocks, iters, out, flops, (hipStream_t)stream));
    return N3P_OK;
}

N3P_API int n3p_heq_residual(int64_t n, double c, const double *x, double *F, double *D,
                             void *stream)
{
    if (n < 1 || !x || !F) return N3P_E_INVALID;
    HIPCHK(launch_heq_residual(n, c, x, nullptr, F, D, (hipStream_t)stream));
    return N3P_OK;
}

N3P_API int n3p_heq_jacobian(int64_t n, double c, const double *D, float *J, int64_t ldj,
                             void *stream)
{
    if (n < 1 || !D || !J || ldj < n) return N3P_E_INVALID;
    HIPCHK(launch_heq_jacobian(n, c, D, nullptr, J, ldj, (hipStream_t)stream));
    return N3P_OK;
}

}  // extern "C"
