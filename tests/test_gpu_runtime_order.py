"""The binding imports torch before it loads the library, so the library
binds to torch's bundled HIP runtime (same soname as the system one) and
the process has one runtime: a program that solves through the binding
before it touches torch.cuda still finds the GPU in torch afterwards, and
only torch's runtime libraries are mapped.  Run in a child process, since
this test process has long loaded torch."""
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
maps = open("/proc/self/maps").read()
libs = {l.split()[-1] for l in maps.splitlines() if "libamdhip64" in l}
assert len(libs) == 1, libs
print("ok")
'''


def test_library_first_then_torch():
    r = subprocess.run([sys.executable, "-c", SCRIPT, ROOT], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stderr[-3000:]


def test_handle_on_a_torch_stream(lib):
    # one runtime: a torch stream is a valid handle stream; device inputs
    # written by torch on that stream are consumed in order, and the
    # results equal those of a handle on its own stream bit for bit
    import numpy as np
    import torch
    shape = (24, 16, 12)
    n = int(np.prod(shape))
    rng = np.random.default_rng(5)
    E = np.exp(rng.normal(0.0, 1.0, n))
    nu = rng.uniform(0.2, 0.35, n)
    with lib.Cell(shape, precision=lib.FP64, tol=1e-10) as c:
        c.set_material(E, nu)
        C0, info0 = c.effective_stiffness()
        u0 = c.displacement(3)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        Ed = torch.tensor(E, dtype=torch.float64, device="cuda") * 1.0
        nud = torch.tensor(nu, dtype=torch.float64, device="cuda") * 1.0
    with lib.Cell(shape, precision=lib.FP64, tol=1e-10, stream=s) as c:
        c.set_material(Ed, nud)
        C1, info1 = c.effective_stiffness()
        u1 = c.displacement(3)
    assert info1["iters"] == info0["iters"]
    assert np.array_equal(C1, C0) and np.array_equal(u1, u0)
