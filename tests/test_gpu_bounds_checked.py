"""Bounds-checked debug build (-DCELLFFT_BOUNDS_CHECK, built by
paper_2004_05197_amd/build.py build_checked()): its kernels compare every
field, spectrum, material and partial-sum access of the PCG iteration and
every reduction partial of the neo-Hookean and surrogate kernels with the
extent of the slot's buffer, skip an access out of range and count it.

tests/checked_cases.py runs solves through every kernel family (3D both
precisions on a ragged grid with its adjoint gradient, every FP32 and FP64
stencil tile with varied FFT-pass variants, operator and preconditioner
applications, 2D, an uneven batch, a neo-Hookean Newton solve, a surrogate
solve) once against the checked build and once against the normal build,
each in a child process.  The checked build must count no violation after
any case, and its results must equal the normal build's (the checks only
guard the accesses; the arithmetic is the same code).  The normal build
reports -1 (it checks nothing).
"""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CHECKED = os.path.join(ROOT, "paper_2004_05197_amd", "_build_checked", "libcellfft_checked.so")

pytestmark = pytest.mark.gpu


def run_cases(lib_path):
    env = dict(os.environ)
    env.pop("CELLFFT_LIBRARY", None)
    if lib_path:
        env["CELLFFT_LIBRARY"] = lib_path
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "checked_cases.py")], env=env,
                       capture_output=True, text=True, timeout=300)
    sys.stderr.write(r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]
    return json.loads(r.stdout.strip().splitlines()[-1])


def test_checked_build_counts_no_violation_and_matches_normal_build():
    if not os.path.exists(CHECKED):
        pytest.skip("bounds-checked library not built (python -m paper_2004_05197_amd.build --checked)")
    chk = run_cases(CHECKED)
    ref = run_cases(None)
    assert set(chk) == set(ref)
    for name in ref:
        assert ref[name]["viol"] == -1, name
        assert chk[name]["viol"] == 0, (name, chk[name]["viol"])
        for key, v in ref[name].items():
            if key == "viol":
                continue
            a, b = np.asarray(chk[name][key], dtype=float), np.asarray(v, dtype=float)
            scale = max(np.abs(b).max(), 1e-300)
            assert np.abs(a - b).max() <= 1e-12 * scale, (name, key, np.abs(a - b).max() / scale)
