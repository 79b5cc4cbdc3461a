"""Reader of the stored oracle results for the large H-equation cases.

The files tests/golden/oracle_heq_n<N>_c<c>.txt are written by
make_heq_large.py, which runs only the CPU oracle.  This module parses them
and imports nothing else, so the benchmark can read the stored values
without loading the oracle.
"""
import os

import numpy as np

NSAMPLE = 257


def path_for(n, c):
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_heq_n%d_c%s.txt" % (n, repr(c)))


def sample_index(n):
    return np.unique(np.linspace(0, n - 1, NSAMPLE).round().astype(int))


def read(n, c):
    """Parsed golden file: dict(kind, its, rel_hist, mean, norm2, idx, x)."""
    out = {"idx": [], "x": [], "kind": "floor"}
    with open(path_for(n, c)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            key, *vals = line.split()
            if key == "kind":
                out["kind"] = vals[0]
            elif key == "its":
                out["its"] = int(vals[0])
            elif key == "rel_hist":
                out["rel_hist"] = np.array([float(v) for v in vals])
            elif key in ("mean", "norm2", "floor_mean", "floor_norm2"):
                out[key.replace("floor_", "")] = float(vals[0])
            elif key == "x":
                out["idx"].append(int(vals[0]))
                out["x"].append(float(vals[1]))
    out["idx"] = np.array(out["idx"])
    out["x"] = np.array(out["x"])
    return out

