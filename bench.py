"""Benchmark: three-precision Newton time-to-solution on one MI355X.

One step = one full solve of the midpoint-rule H-equation (eq. (3.2) of
Kelley, "Newton's Method in Three Precisions"), N = 16384, c = 0.99, from
x0 = ones to ||F|| <= 1e-10 ||F(x0)||, with the residual in FP64, the
Jacobian stored in FP32 and an FP16 LU reused by iterative refinement
(Algorithm 2.1).  Inputs are resident on the GPU before timing starts.

Printed (one JSON line): time per solve, the same solve with an FP64 LU
(Newton with a double-precision factorisation) on the same GPU, the
factorisation's fraction of the FP16 matrix-core peak, and the CPU oracle
timed on two bounded samples on this host's cores.

Other modes: --serve (the batched engine on a seeded request stream) and
--precision (the LU precisions compared on the paper's workloads against
the stored oracle results; one JSON line per run, optionally a markdown
table).
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
    ap.add_argument("--cpu-n", type=int, default=6144,
                    help="larger oracle sample size (about 10-20 s of host work); the smaller "
                         "sample is 2/3 of it")
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
    ap.add_argument("--precision", action="store_true",
                    help="LU precision comparison on the H-equation and dense tanh workloads")
    ap.add_argument("--precision-only", choices=["all", "heq", "dense"], default="all")
    ap.add_argument("--precision-quick", action="store_true",
                    help="N=4096 H-equation and N=1024 dense only")
    ap.add_argument("--precision-md", default=None, help="also write the table as markdown here")
    ap.add_argument("--dense-conds", default="100,10000,1000000",
                    help="dense tanh workload: condition numbers (comma-separated)")
    ap.add_argument("--dense-combos", default="FP16:IR,FP16:GMRES_IR,BF16:IR,BF16:GMRES_IR",
                    help="dense tanh workload: prec:solver runs besides the FP64-LU reference")
    ap.add_argument("--dense-no-fp64", action="store_true",
                    help="dense tanh workload: skip the FP64-LU reference run")
    ap.add_argument("--reps", type=int, default=3, help="timed solves per precision run")
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


def precision_bench(args):
    """The LU precisions compared on the paper's workloads (one JSON line per
    run, and optionally a markdown table).

    * H-equation (eq. (3.2)), x0 = ones: FP16 / BF16 / FP32 LU with IR and
      the FP64-LU Newton at N = 4096 and 16384, c in {0.5, 0.9, 0.99}; the
      ill-conditioned N = 8192, c in {0.9999, 0.99999} with GMRES-IR and IR.
      References are the stored oracle results (tests/golden/oracle_heq_*):
      its FP64 Newton count, and its iterate sampled at 257 points (error =
      max over the samples of |x - x_ref| / max|x_ref|).
    * Dense tanh system F(x) = A x + 0.1 tanh(x) - b with cond(A) in
      {1e2, 1e4, 1e6}: x* = 1 exactly (error = max |x - 1|); the count is
      set against the FP64-LU Newton on the same matrix.
    """
    import numpy as np
    import torch
    import paper_2307_16051_amd as n3p
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    import golden_heq as G
    from workloads import dense_tanh_system, dense_tanh_system_torch

    rows = []

    def emit(row):
        rows.append(row)
        print(json.dumps(row), flush=True)

    def timed(fn):
        """Median time of args.reps solves after an untimed first one; a first
        solve over 2 s (non-converging runs) is reported as it is."""
        def once():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            return r, (time.perf_counter() - t0) * 1e3
        rep, ms0 = once()
        if ms0 > 2000.0:
            return rep, ms0
        ts = []
        for _ in range(args.reps):
            rep, ms = once()
            ts.append(ms)
        return rep, float(np.median(ts))

    def heq(n, c, combos):
        g = G.read(n, c)
        idx = torch.from_numpy(g["idx"]).cuda()
        alpha = 2.0 * (1.0 - np.sqrt(1.0 - c)) / c
        for prec, solver in combos:
            opts = n3p.Options.default()
            ws = torch.empty(n3p.workspace_size(n, getattr(n3p, prec), getattr(n3p, solver), opts),
                             dtype=torch.uint8, device="cuda")
            x = torch.empty(n, dtype=torch.float64, device="cuda")

            def go():
                x.fill_(1.0)
                return n3p.solve_heq(n, c, x=x, prec=getattr(n3p, prec),
                                     solver=getattr(n3p, solver), opts=opts, ws=ws)[1]
            rep, ms = timed(go)
            xs = x[idx].cpu().numpy()
            emit(dict(problem="heq", n=n, c=c, prec=prec, solver=solver, status=rep.status,
                      its=rep.its, its_ref=g["its"], its_ref_src="oracle FP64 Newton (stored)",
                      err=float(np.abs(xs - g["x"]).max() / np.abs(g["x"]).max()),
                      moment_err=abs(float(x.mean().item()) - alpha), ms=ms,
                      lin_its=rep.lin_its, final_rel_resid=rep.resid_rel[-1]))
            del ws, x

    def dense(n, cond, combos):
        if n <= 2048:
            A_np, b_np, _ = dense_tanh_system(n, cond)
            A = torch.from_numpy(np.ascontiguousarray(A_np.T)).cuda().t()
            b = torch.from_numpy(b_np).cuda()
        else:
            A, b, _ = dense_tanh_system_torch(n, cond, "cuda")
        its64 = None
        ref = [] if args.dense_no_fp64 else [("FP64", "DIRECT")]
        for prec, solver in ref + [cs for cs in combos if cs[0] != "FP64"]:
            opts = n3p.Options.default()
            ws = torch.empty(n3p.workspace_size(n, getattr(n3p, prec), getattr(n3p, solver), opts),
                             dtype=torch.uint8, device="cuda")
            x = torch.empty(n, dtype=torch.float64, device="cuda")

            def go():
                x.zero_()
                return n3p.solve_dense_tanh(A, b, x, prec=getattr(n3p, prec),
                                            solver=getattr(n3p, solver), opts=opts, ws=ws)[1]
            rep, ms = timed(go)
            if prec == "FP64":
                its64 = rep.its
            emit(dict(problem="dense_tanh", n=n, cond=cond, prec=prec, solver=solver,
                      status=rep.status, its=rep.its, its_ref=its64,
                      its_ref_src="FP64-LU Newton on the GPU (context)",
                      err=float((x - 1.0).abs().max().item()), ms=ms, lin_its=rep.lin_its,
                      pivoted=any(rep.pivoted), final_rel_resid=rep.resid_rel[-1]))
            del ws, x
        del A, b

    if args.precision_only in ("all", "heq"):
        ir_combos = [("FP16", "IR"), ("BF16", "IR"), ("FP32", "IR"), ("FP64", "DIRECT")]
        for n in ([4096] if args.precision_quick else [4096, 16384]):
            for c in (0.5, 0.9, 0.99):
                heq(n, c, ir_combos)
        if not args.precision_quick:
            for c in (0.9999, 0.99999):
                heq(8192, c, [("FP16", "GMRES_IR"), ("FP16", "IR"), ("BF16", "GMRES_IR"),
                              ("FP64", "DIRECT")])
    if args.precision_only in ("all", "dense"):
        dn = 1024 if args.precision_quick else 16384
        combos = [tuple(cs.split(":")) for cs in args.dense_combos.split(",") if cs]
        for cond in [float(c) for c in args.dense_conds.split(",") if c]:
            dense(dn, cond, combos)
    if args.precision_md:
        write_precision_md(rows, args.precision_md, " ".join(["python bench.py"] + sys.argv[1:]))


def write_precision_md(rows, path, cmd):
    lines = ["# LU precision comparison (measured on one MI355X)", "",
             "Command:", "", "```", cmd, "```", "",
             "H-equation error: max over the 257 stored samples of |x - x_ref| / max |x_ref|, "
             "x_ref the oracle's FP64 Newton iterate (tests/golden/oracle_heq_*.txt; at "
             "N = 16384 the iterate that meets the stopping rule, elsewhere the one driven to "
             "the rounding floor); reference count: that oracle run.  Dense tanh: x* = 1, "
             "error max |x - 1|; reference count: FP64-LU Newton on the GPU, for context.  "
             "Status 1 = not converged in 20 Newton steps.", "",
             "| problem | N | c / cond | LU | solver | status | its (ref) | error | "
             "ms / solve | linear its |", "|---|---|---|---|---|---|---|---|---|---|"]
    for r in rows:
        par = r.get("c", r.get("cond"))
        ref = "-" if r["its_ref"] is None else str(r["its_ref"])
        lines.append("| %s | %d | %g | %s | %s | %d | %d (%s) | %.2e | %.1f | %s |" % (
            r["problem"], r["n"], par, r["prec"], r["solver"], r["status"], r["its"], ref,
            r["err"], r["ms"], ",".join(str(v) for v in r["lin_its"])))
    lines += ["", "Raw rows (JSON):", "", "```"] + [json.dumps(r) for r in rows] + ["```", ""]
    with open(path, "w") as f:
        f.write("\n".join(lines))


def cpu_baseline(n_sample: int, n_target: int, c: float):
    """Oracle FP64 Newton on two bounded samples (2/3 n_sample and n_sample),
    extrapolated to the target size with the exponent fitted to the two
    measured times (the O(N^3) LU dominates, but cache and threading effects
    make the small-size exponent differ from 3)."""
    import math
    from oracle import oracle as O
    sizes = [int(round(n_sample * 2 / 3 / 64)) * 64, n_sample]
    samples = []
    for ns in sizes:
        t0 = time.perf_counter()
        r = O.newton_heq(ns, c, floor=False)
        samples.append({"n": ns, "s": time.perf_counter() - t0, "its": r.its})
    (a, b) = samples
    p = math.log(b["s"] / a["s"]) / math.log(b["n"] / a["n"])
    value = b["s"] * 1e3 * (n_target / b["n"]) ** p
    return {"value": value, "unit": "ms", "cores": O.num_threads(), "kind": "oracle",
            "samples": samples, "fitted_exponent": p,
            "value_cubic_scaling": b["s"] * 1e3 * (n_target / b["n"]) ** 3,
            "sample": "oracle FP64 Newton (own LU), H-equation c=%g: N=%d in %.2f s (%d its) and "
                      "N=%d in %.2f s (%d its); time ~ N^%.2f fitted to the two, extrapolated "
                      "to N=%d" % (c, a["n"], a["s"], a["its"], b["n"], b["s"], b["its"], p,
                                   n_target)}


def measured_mfma_peak(n3p, torch, prec, blocks=2048, min_ms=10.0):
    """The matrix-core rate on this device (TFLOP/s): back-to-back 32x32x16
    MFMA chains on register operands, timed with events on the current
    stream.  The chain length is raised until one run takes at least min_ms;
    the rate is the median of three such runs."""
    import numpy as np

    def run(iters):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        out, flops = n3p.mfma_rate_probe(prec, blocks, iters)
        e1.record()
        torch.cuda.synchronize()
        if not bool((out == 2.0 * iters).all()):
            raise RuntimeError("matrix-core rate probe returned wrong sums")
        return e0.elapsed_time(e1), flops

    run(8)  # warm-up (code load)
    iters = 256
    ms, _ = run(iters)
    while ms < min_ms and iters < (1 << 20):
        iters = min(1 << 20, int(iters * max(2.0, 1.2 * min_ms / max(ms, 1e-3))))
        ms, _ = run(iters)
    rates, times = [], []
    for _ in range(3):
        ms, flops = run(iters)
        rates.append(flops / (ms * 1e-3) / 1e12)
        times.append(ms)
    return float(np.median(rates)), {"iters": iters, "ms": times, "tflops": rates}


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
    if args.precision:
        precision_bench(args)
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
        pk, runs = measured_mfma_peak(n3p, torch, prec)
        out["roofline"]["peak_measured"] = pk
        out["roofline"]["peak_measured_runs"] = runs
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
