"""The C-ABI checks of test_abi.py again, against the library with its host
code built under AddressSanitizer and UndefinedBehaviorSanitizer (device
code unchanged), in a Python process started with the clang ASan runtime
preloaded: argument validation, error paths and handle bookkeeping run
without a GPU, and any out-of-bounds access, use after free or undefined
behaviour in them aborts that process.  The sanitized library is built here
if missing or older than the sources (about two minutes)."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _stale(lib):
    if not os.path.exists(lib):
        return True
    t = os.path.getmtime(lib)
    srcs = glob.glob(os.path.join(ROOT, "paper_2004_05197_amd", "csrc", "*")) + \
        glob.glob(os.path.join(ROOT, "include", "*.h"))
    return any(os.path.getmtime(f) > t for f in srcs)


@pytest.mark.slow
def test_abi_under_host_sanitizers():
    from paper_2004_05197_amd import build
    lib = build.SAN_LIB
    if _stale(lib):
        build.build_sanitized()
    # the host code is instrumented (calls into both sanitizer runtimes)
    syms = subprocess.run(["nm", "-D", "--undefined-only", lib], capture_output=True, text=True).stdout
    assert "__asan_report_load" in syms and "__ubsan_handle_" in syms
    env = dict(os.environ)
    env["LD_PRELOAD"] = build.sanitizer_runtime()
    # the interpreter itself is not instrumented: leaks of the process are
    # not ours to report; any other finding aborts with a non-zero status
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["CELLFFT_LIBRARY"] = lib
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert " passed" in r.stdout
