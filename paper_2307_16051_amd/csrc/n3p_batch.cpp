// n3p_batch.cpp -- batched engine and continuous-batching request loop.
//
// Many independent H-equation solves (eq. (3.2)) advance through Algorithm 2.1
// together: one engine step performs one Newton iteration for every admitted
// request -- Jacobian stored FP32 and rounded to half precision, the
// half-precision LU, IR sweeps (the IR algorithm of Section 2.2 with the Section 3.1 policy),
// the FP64 update and residual -- as a fixed sequence of batched kernels that
// walk a device table of slots.  Requests join at step boundaries as slots and
// pool memory free up, and leave when their stopping test passes, so work of
// requests admitted at different times overlaps on the device.  The step
// phases are captured once as HIP graphs and replayed; the slot table they
// read lives in device memory, so a replay serves whatever requests are
// present.  The engine never allocates device memory: the caller's pool holds
// the slot table and every request's buffers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <thread>
#include <vector>

#include "n3p_internal.hpp"

namespace n3p {
hipError_t launch_hinv(int64_t n, double *h, hipStream_t s);
}
using namespace n3p;

#define BHIP(expr)                                                                    \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess) {                                                       \
            if (std::getenv("N3P_DEBUG"))                                             \
                std::fprintf(stderr, "n3p: %s failed: %s (%s:%d)\n", #expr,           \
                             hipGetErrorString(e_), __FILE__, __LINE__);              \
            return N3P_E_HIP;                                                         \
        }                                                                             \
    } while (0)
#define BCHK(expr)                    \
    do {                              \
        int st_ = (expr);             \
        if (st_ < 0) return st_;      \
    } while (0)

namespace {

constexpr size_t BALIGN = 256;
inline size_t al(size_t v) { return (v + BALIGN - 1) / BALIGN * BALIGN; }

// Per-request buffers, in pool order.  Returns the bytes needed; fills d
// when base is non-null.
size_t request_layout(int64_t n, int prec, BDesc *d, char *base)
{
    const int64_t Np = round_up(std::max<int64_t>(n, 1), B_LEAF);
    const size_t es = 2;  // FP16 / BF16 factors
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = al(off + bytes);
        return o;
    };
    const size_t oA = take((size_t)Np * Np * es), oLT = take((size_t)Np * B_LEAF * es),
                 oDG = take((size_t)2 * B_LEAF * B_LEAF * es), oJ = take((size_t)n * n * 4),
                 oCS = take((size_t)Np * 4), ox = take((size_t)n * 8), oF = take((size_t)n * 8),
                 oD = take((size_t)n * 8), oh = take((size_t)2 * n * 8), ob = take((size_t)Np * 4),
                 ou = take((size_t)Np * 4), oup = take((size_t)Np * 4), orr = take((size_t)Np * 4),
                 oy = take((size_t)Np * 4), ofl = take((size_t)NFLAGS * 4);
    if (d && base) {
        std::memset(d, 0, sizeof(*d));
        d->n = n;
        d->Np = Np;
        d->prec = prec;
        d->A = base + oA;
        d->LT = base + oLT;
        d->DG = base + oDG;
        d->J = (float *)(base + oJ);
        d->colscale = prec == N3P_FP16 ? (float *)(base + oCS) : nullptr;
        d->x = (double *)(base + ox);
        d->F = (double *)(base + oF);
        d->D = (double *)(base + oD);
        d->h = (double *)(base + oh);
        d->b = (float *)(base + ob);
        d->u = (float *)(base + ou);
        d->uprev = (float *)(base + oup);
        d->r = (float *)(base + orr);
        d->y = (float *)(base + oy);
        d->flags = (int *)(base + ofl);
    }
    return off;
}

size_t fixed_bytes(int max_slots)
{
    return al(sizeof(BDesc) * (size_t)max_slots) + al(sizeof(BState) * (size_t)max_slots);
}

// First-fit allocator over [0, size) of the pool, in 256-byte units.
struct Pool {
    std::map<size_t, size_t> free_;  // offset -> length
    void init(size_t size) { free_.clear(); if (size) free_[0] = size; }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = al(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, o2 = it->first + bytes;
                free_.erase(it);
                if (rest) free_[o2] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = al(bytes);
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t largest() const
    {
        size_t m = 0;
        for (auto &kv : free_) m = std::max(m, kv.second);
        return m;
    }
};

bool valid_cfg(const n3p_engine_config &c)
{
    return c.max_slots >= 1 && c.max_slots <= B_MAX_SLOTS && c.max_n >= 1 &&
           round_up(c.max_n, B_LEAF) <= B_MAX_NP && (c.lu_prec == N3P_FP16 || c.lu_prec == N3P_BF16) &&
           c.leaf_grid >= 1 && c.gemm_grid >= 1 && c.vec_grid >= 1 &&
           (c.gemm_kc == 32 || c.gemm_kc == 64);
}

}  // namespace

struct n3p_engine {
    n3p_engine_config cfg{};
    BParams prm{};
    hipStream_t s = nullptr;
    char *pool = nullptr;
    size_t pool_bytes = 0;
    BDesc *d_desc = nullptr;
    BState *d_state = nullptr;
    std::vector<BDesc> hdesc;
    std::vector<BState> hstate;
    std::vector<size_t> slot_off, slot_bytes;  // pool region per slot (0 bytes: free)
    std::vector<int> slot_np;                   // padded size of the slot's request
    Pool alloc;
    size_t req_base = 0;                        // first pool byte usable by requests
    std::map<int, hipGraphExec_t> g_factor;     // keyed by the number of leaves
    hipGraphExec_t g_sweep = nullptr, g_final = nullptr;
    bool any_fresh = false;

    int nslots() const { return cfg.max_slots; }

    // ---- phase launch sequences (captured into graphs when use_graphs)
    int seq_factor(int leaves)
    {
        BHIP(launch_b_jac(cfg.lu_prec, d_desc, d_state, nslots(), prm.target_log2, cfg.vec_grid, s));
        for (int l = 0; l < leaves; ++l) {
            BHIP(launch_b_leaf(cfg.lu_prec, d_desc, d_state, nslots(), l, cfg.leaf_grid, s));
            BHIP(launch_b_gemm(cfg.lu_prec, d_desc, d_state, nslots(), l, cfg.gemm_kc, cfg.gemm_grid, s));
        }
        BHIP(launch_b_ir_init(d_desc, d_state, nslots(), prm, s));
        return 0;
    }
    int seq_sweep()
    {
        BHIP(launch_b_solve(cfg.lu_prec, d_desc, d_state, nslots(), s));
        BHIP(launch_b_gemv(d_desc, d_state, nslots(), cfg.vec_grid, s));
        BHIP(launch_b_ir_check(d_desc, d_state, nslots(), prm, s));
        return 0;
    }
    int seq_final()
    {
        BHIP(launch_b_ir_final(d_desc, d_state, nslots(), prm, s));
        BHIP(launch_b_residual(d_desc, d_state, nslots(), 1 << BP_RUN, cfg.vec_grid, s));
        BHIP(launch_b_newton_check(d_desc, d_state, nslots(), 1 << BP_RUN, prm, s));
        return 0;
    }
    template <typename Seq>
    int capture(hipGraphExec_t *exec, Seq seq)
    {
        hipGraph_t g = nullptr;
        BHIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        const int st = seq();
        hipGraph_t gg = nullptr;
        const hipError_t e = hipStreamEndCapture(s, &gg);
        if (st) return st;
        BHIP(e);
        g = gg;
        BHIP(hipGraphInstantiate(exec, g, nullptr, nullptr, 0));
        BHIP(hipGraphDestroy(g));
        return 0;
    }
    int run_factor(int leaves)
    {
        if (!cfg.use_graphs) return seq_factor(leaves);
        auto it = g_factor.find(leaves);
        if (it == g_factor.end()) {
            hipGraphExec_t ex = nullptr;
            BCHK(capture(&ex, [&] { return seq_factor(leaves); }));
            it = g_factor.emplace(leaves, ex).first;
        }
        BHIP(hipGraphLaunch(it->second, s));
        return 0;
    }
    int run_sweep()
    {
        if (!cfg.use_graphs) return seq_sweep();
        if (!g_sweep) BCHK(capture(&g_sweep, [&] { return seq_sweep(); }));
        BHIP(hipGraphLaunch(g_sweep, s));
        return 0;
    }
    int run_final()
    {
        if (!cfg.use_graphs) return seq_final();
        if (!g_final) BCHK(capture(&g_final, [&] { return seq_final(); }));
        BHIP(hipGraphLaunch(g_final, s));
        return 0;
    }
    int pull_states()
    {
        BHIP(hipMemcpyAsync(hstate.data(), d_state, sizeof(BState) * hstate.size(),
                            hipMemcpyDeviceToHost, s));
        BHIP(hipStreamSynchronize(s));
        return 0;
    }
    int push_slot(int k)
    {
        BHIP(hipMemcpyAsync(d_desc + k, &hdesc[k], sizeof(BDesc), hipMemcpyHostToDevice, s));
        BHIP(hipMemcpyAsync(d_state + k, &hstate[k], sizeof(BState), hipMemcpyHostToDevice, s));
        BHIP(hipStreamSynchronize(s));  // the host copies may change right after
        return 0;
    }

    int step(int *n_done)
    {
        if (any_fresh) {
            BHIP(launch_b_fill_x0(d_desc, d_state, nslots(), s));
            BHIP(launch_b_residual(d_desc, d_state, nslots(), 1 << BP_FRESH, cfg.vec_grid, s));
            BHIP(launch_b_newton_check(d_desc, d_state, nslots(), 1 << BP_FRESH, prm, s));
            any_fresh = false;
        }
        int leaves = 0;
        for (int k = 0; k < nslots(); ++k)
            if (hstate[k].phase == BP_RUN || hstate[k].phase == BP_FRESH)
                leaves = std::max(leaves, slot_np[k] / B_LEAF);
        if (leaves > 0) {
            BCHK(run_factor(leaves));
            // two sweeps cover most steps; then sweep while any slot is still refining
            BCHK(run_sweep());
            BCHK(run_sweep());
            for (int sw = 2; sw < prm.max_sweeps; ++sw) {
                BCHK(pull_states());
                bool on = false;
                for (int k = 0; k < nslots(); ++k) on |= hstate[k].phase == BP_RUN && hstate[k].ir_on;
                if (!on) break;
                BCHK(run_sweep());
            }
            BCHK(run_final());
        }
        BCHK(pull_states());
        int done = 0;
        for (int k = 0; k < nslots(); ++k) done += hstate[k].phase == BP_DONE;
        if (n_done) *n_done = done;
        return 0;
    }

    int admit(int64_t n, double c, int *slot)
    {
        if (n < 1 || n > cfg.max_n || !(c >= 0.0 && c < 1.0)) return N3P_E_INVALID;
        int k = -1;
        for (int i = 0; i < nslots(); ++i)
            if (hstate[i].phase == BP_FREE && slot_bytes[i] == 0) { k = i; break; }
        if (k < 0) return N3P_E_NOMEM;
        const size_t need = request_layout(n, cfg.lu_prec, nullptr, nullptr);
        size_t off = 0;
        if (!alloc.alloc(need, &off)) return N3P_E_NOMEM;
        slot_off[k] = off;
        slot_bytes[k] = need;
        request_layout(n, cfg.lu_prec, &hdesc[k], pool + req_base + off);
        hdesc[k].c = c;
        slot_np[k] = (int)hdesc[k].Np;
        std::memset(&hstate[k], 0, sizeof(BState));
        hstate[k].phase = BP_FRESH;
        BCHK(push_slot(k));
        BHIP(launch_hinv(n, hdesc[k].h, s));
        any_fresh = true;
        *slot = k;
        return 0;
    }

    int release(int k)
    {
        if (slot_bytes[k]) alloc.release(slot_off[k], slot_bytes[k]);
        slot_bytes[k] = 0;
        slot_np[k] = 0;
        std::memset(&hdesc[k], 0, sizeof(BDesc));
        std::memset(&hstate[k], 0, sizeof(BState));
        hstate[k].phase = BP_FREE;
        BCHK(push_slot(k));
        return 0;
    }

    void report(int k, n3p_report *rep) const
    {
        if (!rep) return;
        std::memset(rep, 0, sizeof(*rep));
        const BState &z = hstate[k];
        rep->status = z.status;
        rep->its = z.its;
        rep->f0 = z.f0;
        rep->fnorm = z.fn;
        for (int i = 0; i <= z.its && i < N3P_MAX_HIST; ++i) rep->resid_rel[i] = z.rel[i];
        for (int i = 0; i < z.its && i < N3P_MAX_HIST; ++i) {
            rep->lin_its[i] = z.lin[i];
            rep->lin_outer[i] = z.lin[i];
        }
    }

    // releases only; a destructor has nobody to report a failure to
    ~n3p_engine()
    {
        for (auto &kv : g_factor) (void)hipGraphExecDestroy(kv.second);
        if (g_sweep) (void)hipGraphExecDestroy(g_sweep);
        if (g_final) (void)hipGraphExecDestroy(g_final);
        if (s) (void)hipStreamDestroy(s);
    }
};

extern "C" {

N3P_API void n3p_engine_default_config(n3p_engine_config *c)
{
    if (!c) return;
    c->max_slots = 64;
    c->max_n = 2048;
    c->lu_prec = N3P_FP16;
    c->use_graphs = 1;
    c->leaf_grid = 512;
    c->gemm_grid = 2048;
    c->gemm_kc = 32;
    c->vec_grid = 1024;
}

N3P_API size_t n3p_engine_request_bytes(int64_t n, int lu_prec)
{
    if (n < 1 || round_up(n, B_LEAF) > B_MAX_NP || (lu_prec != N3P_FP16 && lu_prec != N3P_BF16))
        return 0;
    return al(request_layout(n, lu_prec, nullptr, nullptr));
}

N3P_API size_t n3p_engine_fixed_bytes(int max_slots)
{
    if (max_slots < 1 || max_slots > B_MAX_SLOTS) return 0;
    return fixed_bytes(max_slots) + BALIGN;
}

N3P_API int n3p_engine_create(n3p_engine **out, const n3p_engine_config *cfg,
                              const n3p_options *opt, void *pool, size_t pool_bytes, void *stream)
{
    if (!out) return N3P_E_INVALID;
    *out = nullptr;
    n3p_engine_config c;
    if (cfg) c = *cfg;
    else n3p_engine_default_config(&c);
    n3p_options o;
    if (opt) o = *opt;
    else n3p_default_options(&o);
    // the engine's IR promotes the factors on the fly (no eq. (2.19) option)
    if (!valid_cfg(c) || !pool || o.maxit < 0 || o.max_ir_sweeps < 1 || o.ir_scaled_half != 0)
        return N3P_E_INVALID;
    char *base = (char *)(((uintptr_t)pool + BALIGN - 1) / BALIGN * BALIGN);
    const size_t lost = (size_t)(base - (char *)pool);
    const size_t fixed = fixed_bytes(c.max_slots);
    if (pool_bytes < lost + fixed) return N3P_E_NOMEM;
    n3p_engine *e = new (std::nothrow) n3p_engine;
    if (!e) return N3P_E_NOMEM;
    e->cfg = c;
    e->prm.tau_r = o.tau_r;
    e->prm.tau_a = o.tau_a;
    e->prm.eta = o.eta;
    e->prm.maxit = o.maxit;
    e->prm.max_sweeps = o.max_ir_sweeps;
    e->prm.target_log2 = 9.0f;
    e->pool = base;
    e->pool_bytes = pool_bytes - lost;
    e->d_desc = (BDesc *)base;
    e->d_state = (BState *)(base + al(sizeof(BDesc) * (size_t)c.max_slots));
    e->req_base = fixed;
    e->alloc.init(e->pool_bytes - fixed);
    e->hdesc.assign(c.max_slots, BDesc{});
    e->hstate.assign(c.max_slots, BState{});
    e->slot_off.assign(c.max_slots, 0);
    e->slot_bytes.assign(c.max_slots, 0);
    e->slot_np.assign(c.max_slots, 0);
    // own stream (graph capture needs one), ordered after the caller's stream
    hipEvent_t ev = nullptr;
    if (hipStreamCreateWithFlags(&e->s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(ev, (hipStream_t)stream) != hipSuccess ||
        hipStreamWaitEvent(e->s, ev, 0) != hipSuccess) {
        if (ev) (void)hipEventDestroy(ev);  // already failing: report the first error
        delete e;
        return N3P_E_HIP;
    }
    if (hipEventDestroy(ev) != hipSuccess) {
        delete e;
        return N3P_E_HIP;
    }
    int st = 0;
    if (hipMemcpyAsync(e->d_desc, e->hdesc.data(), sizeof(BDesc) * c.max_slots,
                       hipMemcpyHostToDevice, e->s) != hipSuccess ||
        hipMemcpyAsync(e->d_state, e->hstate.data(), sizeof(BState) * c.max_slots,
                       hipMemcpyHostToDevice, e->s) != hipSuccess ||
        hipStreamSynchronize(e->s) != hipSuccess)
        st = N3P_E_HIP;
    if (st) {
        delete e;
        return st;
    }
    *out = e;
    return 0;
}

N3P_API int n3p_engine_destroy(n3p_engine *e)
{
    if (!e) return N3P_E_INVALID;
    const hipError_t r = hipStreamSynchronize(e->s);
    delete e;
    return r == hipSuccess ? 0 : N3P_E_HIP;
}

N3P_API int n3p_engine_admit(n3p_engine *e, int64_t n, double c, int *slot)
{
    if (!e || !slot) return N3P_E_INVALID;
    return e->admit(n, c, slot);
}

N3P_API int n3p_engine_step(n3p_engine *e, int *n_done)
{
    if (!e) return N3P_E_INVALID;
    return e->step(n_done);
}

N3P_API int n3p_engine_slot_state(const n3p_engine *e, int slot, int *phase, int *its)
{
    if (!e || slot < 0 || slot >= e->nslots()) return N3P_E_INVALID;
    if (phase) *phase = e->hstate[slot].phase;
    if (its) *its = e->hstate[slot].its;
    return 0;
}

N3P_API int n3p_engine_collect(n3p_engine *e, int slot, double *x_out, n3p_report *rep)
{
    if (!e || slot < 0 || slot >= e->nslots() || e->hstate[slot].phase != BP_DONE)
        return N3P_E_INVALID;
    if (x_out)
        BHIP(hipMemcpyAsync(x_out, e->hdesc[slot].x, sizeof(double) * e->hdesc[slot].n,
                            hipMemcpyDeviceToDevice, e->s));
    e->report(slot, rep);
    BCHK(e->release(slot));
    BHIP(hipStreamSynchronize(e->s));
    return 0;
}

N3P_API int n3p_engine_largest_free(const n3p_engine *e, size_t *bytes)
{
    if (!e || !bytes) return N3P_E_INVALID;
    *bytes = e->alloc.largest();
    return 0;
}

// Times the factorisation phase (Jacobian, leaves, rank-64 updates) of the
// requests currently admitted under each candidate (leaf grid, update grid,
// update K chunk) and keeps the fastest.  Requests must be admitted and not
// yet stepped (fresh); they are initialised here and stay admitted.
N3P_API int n3p_engine_autotune(n3p_engine *e, n3p_engine_config *chosen, float *ms_out,
                                int *n_candidates)
{
    if (!e) return N3P_E_INVALID;
    if (e->any_fresh) {
        BHIP(launch_b_fill_x0(e->d_desc, e->d_state, e->nslots(), e->s));
        BHIP(launch_b_residual(e->d_desc, e->d_state, e->nslots(), 1 << BP_FRESH, e->cfg.vec_grid, e->s));
        BHIP(launch_b_newton_check(e->d_desc, e->d_state, e->nslots(), 1 << BP_FRESH, e->prm, e->s));
        e->any_fresh = false;
    }
    BCHK(e->pull_states());
    int leaves = 0;
    for (int k = 0; k < e->nslots(); ++k)
        if (e->hstate[k].phase == BP_RUN) leaves = std::max(leaves, e->slot_np[k] / B_LEAF);
    if (leaves == 0) return N3P_E_INVALID;
    const int leaf_grids[] = {256, 512, 1024};
    const int gemm_grids[] = {512, 1024, 2048, 4096};
    const int kcs[] = {32, 64};
    hipEvent_t a = nullptr, b = nullptr;
    BHIP(hipEventCreate(&a));
    BHIP(hipEventCreate(&b));
    const n3p_engine_config keep = e->cfg;
    n3p_engine_config best = keep;
    float best_ms = 1e30f;
    int cand = 0;
    for (int lg : leaf_grids)
        for (int gg : gemm_grids)
            for (int kc : kcs) {
                e->cfg.leaf_grid = lg;
                e->cfg.gemm_grid = gg;
                e->cfg.gemm_kc = kc;
                float tot = 0.0f;
                for (int rep = 0; rep < 3; ++rep) {
                    BHIP(hipEventRecord(a, e->s));
                    BHIP(launch_b_jac(e->cfg.lu_prec, e->d_desc, e->d_state, e->nslots(),
                                      e->prm.target_log2, e->cfg.vec_grid, e->s));
                    for (int l = 0; l < leaves; ++l) {
                        BHIP(launch_b_leaf(e->cfg.lu_prec, e->d_desc, e->d_state, e->nslots(), l, lg, e->s));
                        BHIP(launch_b_gemm(e->cfg.lu_prec, e->d_desc, e->d_state, e->nslots(), l, kc, gg, e->s));
                    }
                    BHIP(hipEventRecord(b, e->s));
                    BHIP(hipEventSynchronize(b));
                    float ms = 0.0f;
                    BHIP(hipEventElapsedTime(&ms, a, b));
                    if (rep > 0) tot += ms;  // the first run warms up
                }
                const float ms = tot / 2.0f;
                if (ms_out) ms_out[cand] = ms;
                ++cand;
                if (ms < best_ms) {
                    best_ms = ms;
                    best = e->cfg;
                }
            }
    bool ok = hipEventDestroy(a) == hipSuccess;
    ok &= hipEventDestroy(b) == hipSuccess;
    // graphs captured with the old grid sizes are stale: all are released
    // (and forgotten) before any failure is reported
    for (auto &kv : e->g_factor) ok &= hipGraphExecDestroy(kv.second) == hipSuccess;
    e->g_factor.clear();
    if (!ok) return N3P_E_HIP;
    e->cfg = best;
    if (chosen) *chosen = best;
    if (n_candidates) *n_candidates = cand;
    (void)keep;
    return 0;
}

// Continuous batching over a stream of H-equation requests (arrival times in
// seconds from the start, non-decreasing).  Between engine steps every
// request that has arrived is admitted in arrival order while a slot and
// pool memory are free; finished requests are copied out (x to
// x_out + x_off[i], FP64 device) and their memory released.
N3P_API int n3p_serve(const n3p_engine_config *cfg, const n3p_options *opt, void *pool,
                      size_t pool_bytes, int count, const int64_t *n, const double *c,
                      const double *arrival_s, double *x_out, const int64_t *x_off, int *its,
                      int *status, double *latency_ms, n3p_serve_stats *stats, void *stream)
{
    if (count < 0 || (count > 0 && (!n || !c || !arrival_s))) return N3P_E_INVALID;
    for (int i = 1; i < count; ++i)
        if (arrival_s[i] < arrival_s[i - 1]) return N3P_E_INVALID;
    n3p_engine *e = nullptr;
    BCHK(n3p_engine_create(&e, cfg, opt, pool, pool_bytes, stream));
    std::vector<int> req_of(e->nslots(), -1);
    std::vector<double> done_t(count, 0.0);
    using clk = std::chrono::steady_clock;
    const auto t0 = clk::now();
    auto now_s = [&] { return std::chrono::duration<double>(clk::now() - t0).count(); };
    int next = 0, finished = 0, active = 0, max_active = 0, steps = 0, st = 0;
    while (finished < count) {
        // admit everything that has arrived, in order, while it fits
        const double t = now_s();
        while (next < count && arrival_s[next] <= t) {
            int slot = -1;
            const int a = e->admit(n[next], c[next], &slot);
            if (a == N3P_E_NOMEM) {
                if (active == 0) { st = N3P_E_NOMEM; break; }  // can never fit
                break;
            }
            if (a) { st = a; break; }
            req_of[slot] = next++;
            ++active;
        }
        if (st) break;
        max_active = std::max(max_active, active);
        if (active == 0) {  // idle until the next arrival
            if (next >= count) break;
            const double wait = arrival_s[next] - now_s();
            if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(wait));
            continue;
        }
        int nd = 0;
        if ((st = e->step(&nd))) break;
        ++steps;
        if (nd) {
            const double tf = now_s();
            for (int k = 0; k < e->nslots(); ++k) {
                if (e->hstate[k].phase != BP_DONE) continue;
                const int r = req_of[k];
                n3p_report rep;
                if ((st = n3p_engine_collect(e, k, x_out && x_off ? x_out + x_off[r] : nullptr, &rep))) break;
                if (its) its[r] = rep.its;
                if (status) status[r] = rep.status;
                done_t[r] = tf;
                if (latency_ms) latency_ms[r] = (tf - arrival_s[r]) * 1e3;
                req_of[k] = -1;
                --active;
                ++finished;
            }
            if (st) break;
        }
    }
    const double makespan = now_s();
    n3p_engine_destroy(e);
    if (st) return st;
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        std::vector<double> lat(count);
        for (int i = 0; i < count; ++i) lat[i] = (done_t[i] - arrival_s[i]) * 1e3;
        std::sort(lat.begin(), lat.end());
        auto pct = [&](double p) {
            if (lat.empty()) return 0.0;
            const size_t k = (size_t)std::min<double>(lat.size() - 1, std::ceil(p * lat.size()) - 1);
            return lat[k];
        };
        double sum = 0;
        for (double v : lat) sum += v;
        stats->p50_ms = pct(0.50);
        stats->p99_ms = pct(0.99);
        stats->mean_ms = count ? sum / count : 0.0;
        stats->max_ms = lat.empty() ? 0.0 : lat.back();
        stats->makespan_s = makespan;
        stats->solves_per_s = makespan > 0 ? count / makespan : 0.0;
        stats->max_active = max_active;
        stats->steps = steps;
    }
    return 0;
}

}  // extern "C"
