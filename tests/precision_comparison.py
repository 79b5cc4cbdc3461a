"""Measured comparison of the LU precisions on the paper's workloads.

Runs the GPU library with the LU in FP16, BF16, FP32 and FP64 (and the three
linear solvers) on the H-equation (eq. (3.2), Section 3.1) and the dense tanh
system, and states for each run the final relative error against the oracle's
solution, the Newton iteration count next to the oracle's, and the time per
solve.  Reference solutions come from the CPU oracle only:

* H-equation: the fixed point of the oracle's Picard sweeps (an independent
  route to the discrete solution; it agrees with the oracle's Newton
  iterate at the rounding floor), and the oracle's FP64 Newton count, read
  from tests/golden/oracle_heq_*.txt when present, else computed.
* Dense tanh system: x* = 1 exactly by construction of b.  The iteration
  count reference is the oracle's FP64 Newton on the identical matrix at the
  sizes where the oracle is run (N <= 2048); at N = 16384 the GPU's FP64-LU
  Newton count is shown for context only.

Usage (GPU):  python tests/precision_comparison.py --only heq --json heq.json
              python tests/precision_comparison.py --only dense --reps 1 --json dense.json
       (CPU):  python tests/precision_comparison.py --assemble heq.json dense.json --out profiles/precision_comparison.md
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))

from oracle import oracle as O  # noqa: E402
import make_heq_large as G  # noqa: E402

PRECS = ["FP16", "BF16", "FP32", "FP64"]


JSON_OUT = None


def log(*a):
    print(*a, flush=True)


def emit(rows):
    log(json.dumps(rows[-1]))
    if JSON_OUT:
        with open(JSON_OUT, "a") as f:
            f.write(json.dumps(rows[-1]) + "\n")


def heq_reference(n, c):
    xr = O.heq_picard(n, c, tol=1e-15)
    try:
        g = G.read(n, c)
        its = g["its"]
        src = "golden"
        # the Picard fixed point and the stored Newton iterate must agree: to
        # the rounding floor (~1e-11 as c -> 1, where Picard's increment test
        # stops short) or, for stored rule iterates, to the stopping rule
        d = np.abs(xr[g["idx"]] - g["x"]).max() / np.abs(g["x"]).max()
        assert d < (1e-10 if g["kind"] == "floor" else 1e-8), (n, c, d)
    except FileNotFoundError:
        its = O.newton_heq(n, c, floor=False).its
        src = "oracle run"
    return xr, its, src


def timed_solve(fn, reps):
    import torch
    out = None
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    return out, float(np.median(ts))


def run_heq(n3p, torch, rows, n, c, combos, reps):
    xr, its_ref, src = heq_reference(n, c)
    nr = np.linalg.norm(xr)
    for prec, solver in combos:
        opts = n3p.Options.default()
        ws = torch.empty(n3p.workspace_size(n, getattr(n3p, prec), getattr(n3p, solver), opts),
                         dtype=torch.uint8, device="cuda")
        x = torch.empty(n, dtype=torch.float64, device="cuda")

        def go():
            x.fill_(1.0)
            return n3p.solve_heq(n, c, x=x, prec=getattr(n3p, prec),
                                 solver=getattr(n3p, solver), opts=opts, ws=ws)[1]
        rep, ms = timed_solve(go, reps)
        err = float(np.linalg.norm(x.cpu().numpy() - xr) / nr)
        rows.append(dict(problem="heq", n=n, c=c, prec=prec, solver=solver, status=rep.status,
                         its=rep.its, its_oracle=its_ref, its_src=src, rel_err=err, ms=ms,
                         lin_its=rep.lin_its, final_rel_resid=rep.resid_rel[-1]))
        emit(rows)
        del ws, x


def run_dense(n3p, torch, rows, n, cond, combos, reps):
    from workloads import dense_tanh_system, dense_tanh_system_torch
    its_ref, src = None, "GPU FP64-LU Newton (context)"
    if n <= 2048:
        A, b, x0 = dense_tanh_system(n, cond)
        its_ref = O.newton_dense_tanh(A, b, x0, floor=False).its
        src = "oracle run"
        At = torch.from_numpy(np.ascontiguousarray(A.T)).cuda().t()
        bt = torch.from_numpy(b).cuda()
    else:
        At, bt, _ = dense_tanh_system_torch(n, cond, "cuda")
    for prec, solver in combos:
        opts = n3p.Options.default()
        ws = torch.empty(n3p.workspace_size(n, getattr(n3p, prec), getattr(n3p, solver), opts),
                         dtype=torch.uint8, device="cuda")
        x = torch.empty(n, dtype=torch.float64, device="cuda")

        def go():
            x.zero_()
            return n3p.solve_dense_tanh(At, bt, x, prec=getattr(n3p, prec),
                                        solver=getattr(n3p, solver), opts=opts, ws=ws)[1]
        rep, ms = timed_solve(go, reps)
        err = float((x - 1.0).norm().item() / np.sqrt(n))
        if its_ref is None and prec == "FP64":
            its_ref = rep.its
        rows.append(dict(problem="dense_tanh", n=n, cond=cond, prec=prec, solver=solver,
                         status=rep.status, its=rep.its, its_oracle=its_ref, its_src=src,
                         rel_err=err, ms=ms, lin_its=rep.lin_its, pivoted=any(rep.pivoted),
                         final_rel_resid=rep.resid_rel[-1]))
        emit(rows)
        del ws, x
    del At, bt


def table(rows):
    out = ["| problem | N | c / cond | LU | solver | status | its (oracle) | "
           "rel. error vs oracle | ms / solve | linear its |",
           "|---|---|---|---|---|---|---|---|---|---|"]
    for r in rows:
        par = r.get("c", r.get("cond"))
        its_o = "-" if r["its_oracle"] is None else str(r["its_oracle"])
        out.append("| %s | %d | %g | %s | %s | %d | %d (%s) | %.2e | %.1f | %s |" % (
            r["problem"], r["n"], par, r["prec"], r["solver"], r["status"], r["its"], its_o,
            r["rel_err"], r["ms"], ",".join(str(v) for v in r["lin_its"])))
    return "\n".join(out)


def write_md(rows, out, cmds):
    md = table(rows)
    with open(out, "w") as f:
        f.write("# LU precision comparison (measured on one MI355X)\n\n")
        f.write("Commands:\n\n```\n%s\n```\n\n" % "\n".join(cmds))
        f.write("Relative error: ||x - x_ref||_2 / ||x_ref||_2 with x_ref the oracle's solution "
                "(H-equation: oracle Picard fixed point; dense tanh: x* = 1, error in max norm).  "
                "Iteration reference: oracle FP64 Newton with the stopping rule "
                "||F|| <= 1e-10 ||F(x0)|| (H-equation: stored oracle results; dense N = 16384: "
                "the GPU's FP64-LU Newton, for context).  Status 1 = not converged in 20 steps "
                "(reported, not gated: see the gating rule in tests/test_gpu_precision.py).\n\n")
        f.write(md + "\n\n")
        f.write("Raw rows (JSON):\n\n```\n")
        for r in rows:
            f.write(json.dumps(r) + "\n")
        f.write("```\n")
    return md


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None, help="markdown file for the table")
    ap.add_argument("--json", default=None, help="write the rows as JSON lines here")
    ap.add_argument("--only", choices=["all", "heq", "dense"], default="all")
    ap.add_argument("--assemble", nargs="*", default=None,
                    help="no GPU: read JSON-line files and write --out")
    ap.add_argument("--quick", action="store_true", help="N=4096 H-equation and N=1024 dense only")
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    if args.assemble is not None:
        rows = []
        for path in args.assemble:
            rows += [json.loads(l) for l in open(path) if l.strip()]
        print(write_md(rows, args.out, [
            "python tests/precision_comparison.py --only heq --json <heq.json>",
            "python tests/precision_comparison.py --only dense --reps 1 --json <dense.json>",
            "python tests/precision_comparison.py --assemble <heq.json> <dense.json> --out %s" % args.out]))
        return
    import torch
    import paper_2307_16051_amd as n3p
    assert torch.cuda.is_available()
    global JSON_OUT
    if args.json:
        JSON_OUT = args.json
        open(JSON_OUT, "w").close()
    rows = []
    if args.only in ("all", "heq"):
        ir_combos = [("FP16", "IR"), ("BF16", "IR"), ("FP32", "IR"), ("FP64", "DIRECT")]
        sizes = [4096] if args.quick else [4096, 16384]
        for n in sizes:
            for c in (0.5, 0.9, 0.99):
                log("# heq n=%d c=%g" % (n, c))
                run_heq(n3p, torch, rows, n, c, ir_combos, args.reps)
        if not args.quick:
            for c in (0.9999, 0.99999):
                log("# heq n=8192 c=%g" % c)
                run_heq(n3p, torch, rows, 8192, c,
                        [("FP16", "GMRES_IR"), ("FP16", "IR"), ("BF16", "GMRES_IR"),
                         ("FP64", "DIRECT")], args.reps)
    if args.only in ("all", "dense"):
        dense_combos = [("FP16", "IR"), ("FP16", "GMRES_IR"), ("BF16", "IR"), ("BF16", "GMRES_IR"),
                        ("FP64", "DIRECT")]
        dn = 1024 if args.quick else 16384
        for cond in (1e2, 1e4, 1e6):
            log("# dense n=%d cond=%g" % (dn, cond))
            run_dense(n3p, torch, rows, dn, cond, dense_combos, args.reps)
    if args.out:
        write_md(rows, args.out, ["python tests/precision_comparison.py --only %s --out %s" % (
            args.only, args.out)])
    print(table(rows), flush=True)


if __name__ == "__main__":
    main()
