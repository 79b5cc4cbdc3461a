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
    ap.add_argument("--cpu-n", type=int, default=4096, help="oracle sample size")
    return ap.parse_args()


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


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported "
              "(independent solves shard one per GPU; see DESIGN.md)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_2307_16051_amd as n3p

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
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
    t0 = time.perf_counter()
    for _ in range(args.steps):
        reps.append(one())
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
        "getrf_ms": getrf_ms, "getrf_tflops": achieved,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP16_TFLOPS
                     if args.prec in ("FP16", "BF16") else PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / (PEAK_FP16_TFLOPS if args.prec in
                                                          ("FP16", "BF16") else PEAK_FP64_TFLOPS),
                     "traffic": None, "kernel": "getrf (whole factorisation, (2/3)N^3 flop)",
                     "padded_n": Np},
    }
    if not args.no_fp64:
        opts64 = n3p.Options.default()
        ws64 = torch.empty(n3p.workspace_size(n, n3p.FP64, n3p.DIRECT, opts64), dtype=torch.uint8,
                           device=dev)
        x.fill_(1.0)
        n3p.solve_heq(n, c, x=x, prec=n3p.FP64, solver=n3p.DIRECT, opts=opts64, ws=ws64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x.fill_(1.0)
        _, rep64 = n3p.solve_heq(n, c, x=x, prec=n3p.FP64, solver=n3p.DIRECT, opts=opts64,
                                 ws=ws64)
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
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_n, n, c)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
