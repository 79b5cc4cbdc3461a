"""Build the CPU oracle shared library (plain C, gcc, OpenMP).

Test infrastructure: the oracle is the independent reference the GPU library
is checked against; nothing in the GPU library links or calls it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "n3p_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


SANITIZE = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
            "-fno-sanitize-recover=undefined"]


def build(verbose: bool = False, out: str = LIB, sanitize: bool = False) -> str:
    """sanitize: an AddressSanitizer + UndefinedBehaviorSanitizer build (load
    it with gcc's libasan preloaded and N3P_ORACLE_LIB=<out>)."""
    opt = SANITIZE if sanitize else ["-O2"]
    cmd = ["gcc"] + opt + ["-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
                           "-o", out, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
