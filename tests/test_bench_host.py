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


def test_cpu_baseline_uneven_on_tiny_cells():
    rng = np.random.default_rng(1)
    cells = [{"n": n, "E": rng.uniform(1.0, 5.0, (n, n, n)), "nu": np.full((n, n, n), 0.3)} for n in (8, 12, 64)]
    out = bench.cpu_baseline_uneven(cells, budget_s=0.0, max_n=12)
    _check(out, "DOF-CG-iterations/s")
    assert "first 1 cells" in out["sample"] and "8^3" in out["sample"]
    out = bench.cpu_baseline_uneven(cells, budget_s=1e9, max_n=12)
    assert "first 2 cells" in out["sample"] and "64^3" not in out["sample"]


def test_summarize_counters_derived_values(tmp_path):
    """Synthetic rocprofv3 counter CSV: 2 K-apply launches of a 16^3 grid
    with 3 loads (one solve of 2 iterations); the derived VALU figures follow
    from the counter values by hand."""
    import csv
    import json
    n = 16 ** 3
    line = {"metric": "m", "value": 1.0, "unit": "u", "ms_per_step": 1.0,
            "config": {"workload": "w", "voxels": n, "iters_per_step": [2, 2, 2], "schedule": [1, 64, 3, 0, 0, 0]}}
    bench_out = tmp_path / "bench.out"
    bench_out.write_text("[bench] progress\n" + json.dumps(line) + "\n")
    d = tmp_path / "pmc"
    d.mkdir()
    name = "void cellfft::k_stencil3t<float, float, 0, true, 32, 8>(cellfft::KArgs<float>, int, int, int, int)"
    rows = []
    for disp in (1, 2):
        for cn, v in (("SQ_WAVES", 200.0), ("SQ_INSTS_VALU", 96000.0), ("SQ_INSTS_LDS", 19200.0),
                      ("TCC_HIT_sum", 30.0), ("TCC_MISS_sum", 10.0)):
            rows.append({"Dispatch_Id": disp, "Kernel_Name": name, "Counter_Name": cn, "Counter_Value": v,
                         "Start_Timestamp": 0, "End_Timestamp": 1000})
    with open(d / "run_counter_collection.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)
    out = tmp_path / "c.md"
    bench.summarize_counters([str(d), "--bench-out", str(bench_out), "--out", str(out), "--title", "t",
                              "--commands", "cmd"])
    text = out.read_text()
    # per unit: one launch covers the 3 loads of the grid, 3 n units
    units = 3 * n
    valu_unit = 96000.0 * 64 / units
    busy = 96000.0 * bench.VALU_CYCLES / (bench.SIMDS * 1e-6 * bench.CLOCK_HZ)
    row = [r for r in text.splitlines() if r.startswith("| k_apply | 480")][0]
    assert f"| {valu_unit:.0f} |" in row and f"| {19200.0 * 64 / units:.1f} |" in row
    assert f"| {busy:.2f} |" in row and "| 0.75 |" in row
