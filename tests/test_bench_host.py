"""Host-side parts of bench.py (no GPU): the one-GPU refusal and the CPU
oracle baselines' fields on tiny sub-blocks."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2004_05197_amd import microstructures as ms  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _check(out, unit):
    assert out["unit"] == unit and out["kind"] == "oracle"
    assert np.isfinite(out["value"]) and out["value"] > 0
    assert out["cores"] >= 1 and isinstance(out["sample"], str)


def test_cpu_baselines_on_tiny_blocks():
    E, nu = ms.lognormal_field(16, 5, ell=4.0)
    _check(bench.cpu_baseline(E, nu, sub=8, iters=2), "DOF-CG-iterations/s")
    _check(bench.cpu_baseline_adjoint(E, nu, sub=4), "DOF-solves/s")
    _check(bench.cpu_baseline_surrogate(E, nu, 2, sub=4), "DOF-solves/s")
    _check(bench.cpu_baseline_hyper(E, nu, bench.hyper_loads()[0], sub=4), "DOF-Newton-iterations/s")
