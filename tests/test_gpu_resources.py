"""Device memory comes back: handles created, used through every path that
allocates (solves with captured graphs, residual history, adjoint, warm
starts, surrogate operator, neo-Hookean solve, autotuning, uneven batches)
and destroyed, again and again, leave the free device memory where it was
after the first round (which loads the kernels' code).  The library runs on
torch's HIP runtime (the binding loads torch first), so the driver's free
count that torch reports includes the library's allocations."""
import numpy as np
import pytest

from paper_2004_05197_amd import microstructures as ms

pytestmark = pytest.mark.gpu


def _round(lib):
    shape = (32, 32, 32)
    n = 32 ** 3
    # a smooth field (the surrogate interpolates the stencil between samples)
    E = np.exp(0.5 * ms.gaussian_random_field(shape, 6.0, 4)).ravel()
    nu = np.full(n, 0.3)
    with lib.Cell(shape, precision=lib.MIXED, tol=1e-6) as c:
        c.set_material(E, nu)
        c.autotune(force=True)
        C, _ = c.effective_stiffness()
        c.residual_history(0)
        c.adjoint(np.eye(6))
        c.set_initial_guess(0, c.displacement(0))
        c.solve(np.eye(6)[:1])
        c.set_surrogate(4, 3)
        c.effective_stiffness()
        c.set_surrogate(0)
    with lib.Cell((16, 16, 16), precision=lib.FP64, tol=1e-9) as c:
        c.set_material(E[:4096], nu[:4096])
        c.solve_hyper((np.eye(3) + 0.01 * np.diag([1.0, -0.5, 0.2]))[None])
    shapes = [(16, 16, 16), (24, 24, 24), (16, 16, 16)]
    with lib.Batch(shapes, precision=lib.MIXED, tol=1e-6) as b:
        for i, sh in enumerate(shapes):
            m, _, _ = ms.rsa_spheres(sh[0], 0.25, seed=30 + i, rmin=1.0, rmax=3.0)
            b.set_material(i, np.where(m, 10.0, 1.0).ravel(), np.full(m.size, 0.3))
        b.effective_stiffness()


def test_no_device_memory_leak(lib):
    import torch
    _round(lib)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(5):
        _round(lib)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    print("free device memory change over 5 rounds: %.1f MiB" % ((free1 - free0) / 2**20))
    assert free0 - free1 <= 8 * 2**20, (free0 - free1) / 2**20
    # the count does see the library's buffers: a live 64^3 six-load cell
    # holds well over 64 MiB
    n = 64 ** 3
    with lib.Cell((64, 64, 64), precision=lib.MIXED, tol=1e-6) as c:
        c.set_material(np.full(n, 2.0), np.full(n, 0.3))
        c.effective_stiffness()
        torch.cuda.synchronize()
        held = free1 - torch.cuda.mem_get_info()[0]
    print("a live 64^3 cell: %.1f MiB" % (held / 2**20))
    assert held >= 64 * 2**20
