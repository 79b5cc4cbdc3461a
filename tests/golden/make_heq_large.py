"""Writes the oracle's FP64 Newton results for the large H-equation cases.

For each (N, c) below this runs the CPU oracle (plain FP64 Newton on eq. (3.2)
with an analytic Jacobian and its own partially pivoted LU, Algorithm 2.1 with
FP64 throughout) from x0 = ones with tau_r = 1e-10, tau_a = 0, and stores:
the Newton iteration count of that rule, the relative residual history, and
the mean, the 2-norm and 257 evenly spaced entries of the iterate driven to
the rounding floor (at N = 16384: of the iterate that meets the rule).  Nothing here comes from the GPU library.

Run from the repository root:  python tests/golden/make_heq_large.py [N c ...]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import oracle as O  # noqa: E402
from golden_heq import path_for, read, sample_index  # noqa: E402,F401

CASES = [(4096, 0.5), (4096, 0.9), (4096, 0.99), (8192, 0.9999), (8192, 0.99999),
         (16384, 0.5), (16384, 0.9), (16384, 0.99)]


def write(n, c, floor=True):
    """floor=False (used at N=16384, where each oracle Newton step costs minutes)
    stores the iterate at which the stopping rule is met instead of the one
    driven to the rounding floor."""
    t0 = time.time()
    r = O.newton_heq(n, c, floor=floor)
    dt = time.time() - t0
    idx = sample_index(n)
    xs = r.x_floor if floor else r.x
    with open(path_for(n, c), "w") as f:
        f.write("# oracle FP64 Newton, H-equation eq. (3.2), N=%d c=%r, x0=ones, "
                "tau_r=1e-10 tau_a=0 (l2 norm)\n" % (n, c))
        f.write("# written by tests/golden/make_heq_large.py (oracle only), %.0f s on %d threads\n"
                % (dt, O.num_threads()))
        f.write("kind %s\n" % ("floor" if floor else "rule"))
        f.write("its %d\n" % r.its)
        f.write("rel_hist %s\n" % " ".join(repr(float(v)) for v in r.rel_hist))
        f.write("mean %r\n" % float(xs.mean()))
        f.write("norm2 %r\n" % float(np.linalg.norm(xs)))
        for i in idx:
            f.write("x %d %r\n" % (i, float(xs[i])))
    print("wrote %s (%.0f s, its %d)" % (path_for(n, c), dt, r.its), flush=True)



if __name__ == "__main__":
    args = sys.argv[1:]
    cases = [(int(args[i]), float(args[i + 1])) for i in range(0, len(args), 2)] if args else CASES
    for n, c in cases:
        write(n, c, floor=n < 16384)
