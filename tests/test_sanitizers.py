"""The CPU code under AddressSanitizer and UndefinedBehaviorSanitizer.

* The oracle (n3p_oracle.c) built with -fsanitize=address,undefined runs the
  fast oracle pins.
* The library's host driver code (n3p_api.cpp, n3p_batch.cpp) built with the
  same sanitizers for the host only runs the host ABI tests (argument
  checks, workspace sizing, exports; no device work).
Each runs in a child process with the sanitizer runtime preloaded; any
report fails the test.  GPU code is never sanitized.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
REPORTS = ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer")


def _pytest_child(env, target, timeout=600):
    env = dict(os.environ, **env)
    env.setdefault("OMP_NUM_THREADS", "4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not slow and not gpu",
                        "-p", "no:cacheprovider", target], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=timeout)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    for rep in REPORTS:
        assert rep not in out, out[-4000:]
    return out


def test_oracle_pins_under_asan_ubsan(tmp_path):
    from oracle import build as ob
    lib = ob.build(out=str(tmp_path / "liboracle_asan.so"), sanitize=True)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True, check=True).stdout.strip()
    if not os.path.isabs(asan):
        pytest.skip("gcc has no shared AddressSanitizer runtime")
    out = _pytest_child({"LD_PRELOAD": asan, "N3P_ORACLE_LIB": lib,
                         "ASAN_OPTIONS": "detect_leaks=0",
                         "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"},
                        "tests/test_oracle_pins.py")
    assert " passed" in out


def test_sanitizer_harness_reports_a_planted_overflow(tmp_path):
    """The harness itself: an out-of-bounds write planted in a scrap C
    function built with the oracle's sanitizer flags is reported when the
    function is called through ctypes in a child with the runtime preloaded."""
    from oracle import build as ob
    src = tmp_path / "planted.c"
    src.write_text("void planted(int i) { int a[4]; volatile int *p = a; p[i] = 1; }\n")
    lib = tmp_path / "libplanted.so"
    subprocess.run(["gcc"] + ob.SANITIZE + ["-fPIC", "-shared", "-o", str(lib), str(src)],
                   check=True)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True, check=True).stdout.strip()
    if not os.path.isabs(asan):
        pytest.skip("gcc has no shared AddressSanitizer runtime")
    code = "import ctypes; ctypes.CDLL(%r).planted(6)" % str(lib)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                       env=dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0"))
    assert r.returncode != 0 and any(rep in r.stderr for rep in REPORTS), r.stderr[-2000:]


def test_host_abi_under_asan_ubsan(tmp_path):
    sys.path.insert(0, os.path.join(ROOT, "paper_2307_16051_amd"))
    import build as nb
    if not all(os.path.exists(os.path.join(nb.BUILD, s + ".o")) for s in nb.SOURCES):
        pytest.skip("the library's objects are not built (run __graft_entry__.build())")
    lib = nb.build_host_sanitized(str(tmp_path))
    rt = subprocess.run([nb.hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"],
                        capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(rt) or not os.path.exists(rt):
        import glob
        cands = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
        if not cands:
            pytest.skip("no shared clang AddressSanitizer runtime")
        rt = cands[0]
    env = {"LD_PRELOAD": rt, "N3P_LIB": lib, "ASAN_OPTIONS": "detect_leaks=0:protect_shadow_gap=0",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}
    # the child loads the sanitized build, not the in-tree library
    r = subprocess.run([sys.executable, "-c", "import paper_2307_16051_amd as n; print(n.lib_path)"],
                       cwd=ROOT, env=dict(os.environ, **env), capture_output=True, text=True)
    assert r.returncode == 0 and r.stdout.strip() == lib, r.stderr[-2000:]
    out = _pytest_child(env, "tests/test_abi_host.py")
    assert " passed" in out
