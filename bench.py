"""Benchmark: three-precision Newton time-to-solution on one MI355X.

One step = one full solve of the midpoint-rule H-equation (eq. (3.2) of
Kelley, "Newton's Method in Three Precisions"), N = 16384, c = 0.99, from
x0 = ones to ||F|| <= 1e-10 ||F(x0)||, with the residual in FP64, the
Jacobian stored in FP32 and an FP16 LU reused by iterative refinement
(Algorithm 2.1).  Inputs are resident on the GPU before timing starts.

Printed (one JSON line): time per solve, the same solve with an FP64 LU
(Newton with a double-precision factorisation) on the same GPU, the
factorisation's fraction of the FP16 matrix-core peak, and the CPU oracle
timed on a bounded sample on this host's cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP16_TFLOPS = 2516.6   # MI355X dense FP16/BF16 matrix peak (no sparsity)
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--c", type=float, default=0.99)
    ap.add_argument("--prec", default="FP16", choices=["FP16", "BF16", "FP32", "FP64"])
    ap.add_argument("--solver", default="IR", choices=["IR", "GMRES_IR", "DIRECT"])
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-LU Newton comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-n", type=int, default=6144, help="oracle sample size (about 10-20 s of host work)")
    ap.add_argument("--no-mf", action="store_true",
                    help="skip the FFT / matrix-free comparison solve")
    ap.add_argument("--copy-calib", action="store_true",
                    help="run one plain 256 MiB device copy first (calibrates HBM byte counters)")
    ap.add_argument("--serve", action="store_true",
                    help="serving benchmark: seeded Poisson stream through the batched engine")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--rate", type=float, default=1000.0, help="arrivals per second")
    ap.add_argument("--slots", type=int, default=64)
    ap.add_argument("--pool-gib", type=float, default=8.0, help="HBM budget for admitted requests")
    return ap.parse_args()


def serve_bench(args):
    """Config: 2000 H-equation requests, Poisson arrivals, N uniform over
    {128, ..., 2048}, c uniform on [0.5, 0.999]; FP16 LU + IR in the batched
    engine; admission by a fixed HBM budget; latency from arrival to result."""
    import numpy as np
    import torch
    import paper_2307_16051_amd as n3p
    from workloads import serving_stream

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    pool = torch.empty(int(args.pool_gib * 2 ** 30), dtype=torch.uint8, device=dev)
    cfg = n3p.EngineConfig.default(max_slots=args.slots, max_n=2048)
    # autotune the factorisation kernels on a representative batch
    eng = n3p.Engine(pool, cfg)
    mix = [128, 256, 512, 1024, 2048] * 6
    slots = [eng.admit(n, 0.9) for n in mix]
    tuned, cand_ms = eng.autotune()
    for _ in range(40):
        if all(eng.state(s)[0] == n3p.PHASE_DONE for s in slots):
            break
        eng.step()
    for s in slots:
        eng.collect(s, None)
    eng.close()
    # warm-up stream (graph capture, first-call costs), then the measured stream
    warm = serving_stream(count=100, rate_per_s=args.rate, seed=3)
    n3p.serve([r.n for r in warm], [r.c for r in warm], [r.arrival_s for r in warm], pool, tuned)
    reqs = serving_stream(count=args.requests, rate_per_s=args.rate, seed=7)
    torch.cuda.synchronize()
    its, status, lat, stats = n3p.serve([r.n for r in reqs], [r.c for r in reqs],
                                        [r.arrival_s for r in reqs], pool, tuned)
    ok = sum(1 for s in status if s == 0)
    by_n = {}
    for r, l in zip(reqs, lat):
        by_n.setdefault(r.n, []).append(l)
    out = {
        "metric": "serving: solves/s with p50/p99 latency (arrival to result)",
        "value": stats["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
        "steps": stats["steps"], "warmup": 100, "ms_per_step": stats["makespan_s"] * 1e3 / max(stats["steps"], 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp16",
        "data": "synthetic",
        "config": {"workload": "%d H-equation requests, Poisson arrivals %.0f/s, N uniform over "
                               "{128,256,512,1024,2048}, c uniform [0.5,0.999], FP16 LU + IR, "
                               "batched engine, %d slots, %.1f GiB pool" % (
                                   args.requests, args.rate, args.slots, args.pool_gib),
                   "requests": args.requests, "rate_per_s": args.rate},
        "p50_ms": stats["p50_ms"], "p99_ms": stats["p99_ms"], "mean_ms": stats["mean_ms"],
        "max_ms": stats["max_ms"], "makespan_s": stats["makespan_s"],
        "max_active": stats["max_active"], "ok": ok, "mean_its": float(np.mean(its)),
        "p50_ms_by_n": {str(k): float(np.median(v)) for k, v in sorted(by_n.items())},
        "autotuned": {k: tuned.as_dict()[k] for k in ("leaf_grid", "gemm_grid", "gemm_kc")},
        "autotune_ms_range": [min(cand_ms), max(cand_ms)],
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(n_sample: int, n_target: int, c: float):
    """Oracle FP64 Newton on a bounded sample, scaled to the target size by N^3."""
    from oracle import oracle as O
    t0 = time.perf_counter()
    r = O.newton_heq(n_sample, c, floor=False)
    dt = time.perf_counter() - t0
    scale = (n_target / n_sample) ** 3
    return {"value": dt * 1e3 * scale, "unit": "ms", "cores": O.num_threads(), "kind": "oracle",
            "sample": "oracle FP64 Newton (own LU), H-equation N=%d c=%g, %d iterations, %.2f s "
                      "measured, scaled by (%d/%d)^3 to N=%d" % (
                          n_sample, c, r.its, dt, n_target, n_sample, n_target)}


def measured_mfma_peak(n3p, torch, prec, blocks=2048, iters=256):
    """The matrix-core rate on this device (TFLOP/s): back-to-back 32x32x16
    MFMA chains on register operands, timed with events on the current stream."""
    n3p.mfma_rate_probe(prec, blocks, 8)  # warm-up (code load)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    out, flops = n3p.mfma_rate_probe(prec, blocks, iters)
    e1.record()
    torch.cuda.synchronize()
    if not bool((out == 2.0 * iters).all()):
        raise RuntimeError("matrix-core rate probe returned wrong sums")
    return flops / (e0.elapsed_time(e1) * 1e-3) / 1e12


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported "
              "(independent solves shard one per GPU)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    if args.serve:
        serve_bench(args)
        return
    import numpy as np
    import torch
    import paper_2307_16051_amd as n3p

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calib:  # 256 MiB read + 256 MiB written by one copy kernel
        src = torch.ones(2 ** 26, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    n, c = args.n, args.c
    prec, solver = getattr(n3p, args.prec), getattr(n3p, args.solver)
    opts = n3p.Options.default()
    ws = torch.empty(n3p.workspace_size(n, prec, solver, opts), dtype=torch.uint8, device=dev)
    x = torch.empty(n, dtype=torch.float64, device=dev)

    def one():
        x.fill_(1.0)
        _, rep = n3p.solve_heq(n, c, x=x, prec=prec, solver=solver, opts=opts, ws=ws)
        return rep

    for _ in range(args.warmup):
        one()
    torch.cuda.synchronize()
    reps = []
    step_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        reps.append(one())  # ends with the stopping test read on the host
        step_ms.append((time.perf_counter() - ts) * 1e3)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per = wall * 1e3 / args.steps
    rep = reps[-1]
    its = rep.its
    getrf_ms = float(np.median([r.ms_getrf / max(r.its, 1) for r in reps]))
    Np = ((n + 511) // 512) * 512
    getrf_flops = 2.0 / 3.0 * float(n) ** 3
    achieved = getrf_flops / (getrf_ms * 1e-3) / 1e12
    xs = x.cpu().numpy()
    alpha = 2.0 * (1.0 - np.sqrt(1.0 - c)) / c
    out = {
        "metric": "Newton time-to-||F||<=1e-10: 3-precision vs FP64-LU, N=16384; LU MFMA %peak",
        "value": ms_per, "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": args.prec.lower() if args.prec != "FP64" else "f64",
        "data": "synthetic",
        "config": {"workload": "H-equation midpoint rule N=%d c=%g x0=ones, %s LU + %s, "
                               "stop ||F||<=1e-10||F0||" % (n, c, args.prec, args.solver),
                   "n": n, "c": c, "lu_precision": args.prec, "linear_solver": args.solver},
        "newton_its": its, "final_rel_resid": rep.resid_rel[-1],
        "moment_identity_err": abs(float(xs.mean()) - alpha),
        "lin_its": rep.lin_its,
        "phase_ms_per_solve": {"jacobian": rep.ms_jac, "getrf": rep.ms_getrf,
                               "linear_solve": rep.ms_solve, "residual": rep.ms_resid},
        "ms_per_step_median": float(np.median(step_ms)), "step_ms": step_ms,
        "getrf_ms": getrf_ms, "getrf_tflops": achieved,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP16_TFLOPS
                     if args.prec in ("FP16", "BF16") else PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / (PEAK_FP16_TFLOPS if args.prec in
                                                          ("FP16", "BF16") else PEAK_FP64_TFLOPS),
                     "traffic": measured_traffic(n, args.prec),
                     "kernel": "getrf (whole factorisation, (2/3)N^3 flop)", "padded_n": Np},
    }
    if args.prec in ("FP16", "BF16"):
        pk = measured_mfma_peak(n3p, torch, prec)
        out["roofline"]["peak_measured"] = pk
        out["roofline"]["frac_of_measured"] = achieved / pk if pk else None
    # the same solve with the O(N log N) residual and operator-based J v
    # (no stored FP32 Jacobian), for comparison
    if not args.no_mf:
        measure_matrix_free(n3p, torch, dev, n, c, prec, solver, x, ws, out)
    if not args.no_fp64:
        fp64_baseline(n3p, torch, dev, n, c, x, getrf_flops, ms_per, out)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_n, n, c)
    print(json.dumps(out), flush=True)


def measure_matrix_free(n3p, torch, dev, n, c, prec, solver, x, ws, out):
    opts_mf = n3p.Options.default(fft_residual=1, matrix_free=1)
    ws_mf = torch.empty(n3p.workspace_size(n, prec, solver, opts_mf), dtype=torch.uint8, device=dev)
    x.fill_(1.0)
    n3p.solve_heq(n, c, x=x, prec=prec, solver=solver, opts=opts_mf, ws=ws_mf)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x.fill_(1.0)
    _, rep_mf = n3p.solve_heq(n, c, x=x, prec=prec, solver=solver, opts=opts_mf, ws=ws_mf)
    torch.cuda.synchronize()
    out["fft_matrix_free"] = {"ms": (time.perf_counter() - t0) * 1e3, "its": rep_mf.its,
                              "linear_solve_ms": rep_mf.ms_solve, "residual_ms": rep_mf.ms_resid,
                              "workspace_gib": ws_mf.numel() / 2 ** 30,
                              "workspace_gib_stored_J": ws.numel() / 2 ** 30}
    del ws_mf


def fp64_baseline(n3p, torch, dev, n, c, x, getrf_flops, ms_per, out):
    """FP64-LU Newton (the FP64 Jacobian factored in FP64, one solve per step)."""
    opts64 = n3p.Options.default()
    ws64 = torch.empty(n3p.workspace_size(n, n3p.FP64, n3p.DIRECT, opts64), dtype=torch.uint8,
                       device=dev)
    x.fill_(1.0)
    n3p.solve_heq(n, c, x=x, prec=n3p.FP64, solver=n3p.DIRECT, opts=opts64, ws=ws64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x.fill_(1.0)
    _, rep64 = n3p.solve_heq(n, c, x=x, prec=n3p.FP64, solver=n3p.DIRECT, opts=opts64, ws=ws64)
    torch.cuda.synchronize()
    ms64 = (time.perf_counter() - t0) * 1e3
    g64 = rep64.ms_getrf / max(rep64.its, 1)
    out["fp64_lu_newton"] = {"ms": ms64, "its": rep64.its, "getrf_ms": g64,
                             "getrf_tflops": getrf_flops / (g64 * 1e-3) / 1e12,
                             "speedup_3p_vs_fp64": ms64 / ms_per}
    del ws64
    # vendor FP64 LU for context (rocSOLVER through torch), one factorisation
    try:
        A = torch.randn(n, n, dtype=torch.float64, device=dev) + n * torch.eye(
            n, dtype=torch.float64, device=dev)
        torch.linalg.lu_factor(A)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        torch.linalg.lu_factor(A)
        torch.cuda.synchronize()
        out["fp64_lu_newton"]["rocsolver_getrf_ms"] = (time.perf_counter() - t0) * 1e3
        del A
    except Exception as e:  # context only
        out["fp64_lu_newton"]["rocsolver_getrf_ms"] = "unavailable: %s" % type(e).__name__


def factor_source_sha(root=ROOT):
    """SHA-256 over what decides the factorisation's memory traffic: the
    kernel sources (k_getrf.hip, k_panel.hip) and the launch schedules
    (getrf_spec, getrf_spec_top)."""
    import hashlib
    csrc = os.path.join(root, "paper_2307_16051_amd", "csrc")
    api = open(os.path.join(csrc, "n3p_api.cpp")).read()
    h = hashlib.sha256()
    for src in ("k_getrf.hip", "k_panel.hip"):
        h.update(open(os.path.join(csrc, src), "rb").read())
    for fn in ("int getrf_spec(", "int getrf_spec_top("):
        i = api.index(fn)
        h.update(api[i:api.index("\n}\n", i)].encode())
    return h.hexdigest()


def measured_traffic(n, prec):
    """HBM bytes per factorisation from the committed rocprofv3 counter runs
    (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy of known size), only if
    the factorisation's kernels and launch schedule are unchanged since they
    were taken."""
    path = os.path.join(ROOT, "profiles", "getrf_traffic_n%d_%s.json" % (n, prec.lower()))
    try:
        rec = json.load(open(path))
        sha = factor_source_sha()
    except (OSError, ValueError):
        return None
    return rec.get("bytes_per_factorisation") if rec.get("factor_source_sha256") == sha else None

if __name__ == "__main__":
    main()
