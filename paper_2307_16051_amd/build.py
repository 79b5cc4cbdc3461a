"""Build libn3p.so (HIP for gfx950) in-tree with hipcc.

Every source is compiled for gfx950 only, with packed-FP32 instruction
selection disabled, and linked into paper_2307_16051_amd/libn3p.so.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libn3p.so")
SOURCES = ["k_problem.hip", "k_getrf.hip", "k_panel.hip", "k_pivot.hip", "k_solve.hip", "k_fft.hip", "k_bench.hip", "n3p_api.cpp", "n3p_batch.cpp"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def common_flags():
    return ["-O3", "-fPIC", "-std=c++17", "--offload-arch=" + ARCH,
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-fvisibility=hidden", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
            "-Wno-unused-result", "-Wno-unused-command-line-argument"]


# Host-side AddressSanitizer / UndefinedBehaviorSanitizer flags (CPU code
# only: each applies to the host compilation, never to gfx950 code)
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
HOST_SOURCES = ["n3p_api.cpp", "n3p_batch.cpp"]


def _compile(src: str, verbose: bool, out_dir: str = BUILD, extra=()) -> str:
    obj = os.path.join(out_dir, os.path.basename(src) + ".o")
    cmd = [hipcc()] + common_flags() + list(extra) + ["-x", "hip", "-c", os.path.join(CSRC, src),
                                                      "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops' is not a recognized feature" not in l)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (src, out))
    if verbose and out.strip():
        print(out, flush=True)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(4, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def build_host_sanitized(out_dir: str, verbose: bool = False) -> str:
    """A copy of the library whose host driver code (HOST_SOURCES) is built
    with HOST_SANITIZE, linked with the kernel objects of the last build().
    Load it with the compiler's ASan runtime preloaded (N3P_LIB=<path>)."""
    objs = []
    for src in SOURCES:
        if src in HOST_SOURCES:
            objs.append(_compile(src, verbose, out_dir, HOST_SANITIZE))
        else:
            obj = os.path.join(BUILD, src + ".o")
            if not os.path.exists(obj):
                raise RuntimeError("build() first: %s is missing" % obj)
            objs.append(obj)
    lib = os.path.join(out_dir, "libn3p_host_asan.so")
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-shared-libsan",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-o", lib] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return lib


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
