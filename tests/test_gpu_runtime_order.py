"""The binding starts torch's HIP runtime before the library's: a program
that solves through the binding before it touches torch.cuda still finds
the GPU in torch afterwards (torch and the library each carry a HIP
runtime, and the one that initialises the device first keeps it).  Run in a
child process, since this test process has long started torch."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.gpu

SCRIPT = r'''
import sys
sys.path.insert(0, sys.argv[1])
import numpy as np
from paper_2004_05197_amd import binding as B
with B.Cell((8, 8, 8), precision=B.FP64, tol=1e-8) as c:
    c.set_material(np.full(512, 2.0), np.full(512, 0.3))
    C, info = c.effective_stiffness()
assert info["status"] == "CELL_OK"
import torch
assert torch.cuda.is_available(), "torch lost the GPU"
x = torch.ones(16, device="cuda", dtype=torch.float64)
assert float(x.sum()) == 16.0
print("ok")
'''


def test_library_first_then_torch():
    r = subprocess.run([sys.executable, "-c", SCRIPT, ROOT], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stderr[-3000:]
