"""PCG behaviour on the GPU: the breakdown status forced from the host, and
iteration counts that do not grow with the grid at fixed microstructure
statistics.

Breakdown: CELLFFT_DEBUG_NEGATE_Q=1 (read when a handle is created) makes
the linear K-apply write -K p, so the first p.Kp is negative.  Every kernel
of the iteration still runs to its normal end (the slot state turns to
breakdown in the finalize kernel and later launches skip the slot); the
solve must report CELL_E_BREAKDOWN and a handle created afterwards must
solve normally.

Iteration counts: for the preconditioned operator, the spectrum is bounded
by the local ratios of the material to the reference medium (K/K_0 and
mu/mu_0 per voxel), not by the grid, so the thresholded Gaussian random
field with correlation length 8 voxels and contrast 1:1000 needs the same
number of iterations at every resolution of the same statistics (within
+-20 %, the spread between samples of a small cell).
"""
import numpy as np
import pytest

from oracle import fem
from paper_2004_05197_amd import microstructures as ms

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [0, 1])
def test_breakdown_status_forced_from_host(lib, monkeypatch, prec):
    mask, _, _ = ms.rsa_spheres(16, 0.3, seed=2, rmin=1.0, rmax=2.0)
    E = np.where(mask, 20.0, 1.0)
    nu = np.full(E.shape, 0.3)
    monkeypatch.setenv("CELLFFT_DEBUG_NEGATE_Q", "1")
    with lib.Cell((16, 16, 16), precision=prec, tol=1e-10 if prec == 0 else 1e-7) as c:
        c.set_material(E.ravel(), nu.ravel())
        with pytest.raises(lib.CellError) as e:
            c.effective_stiffness()
        assert e.value.status == lib.CELL_E_BREAKDOWN
        assert "breakdown" in lib.last_error().lower()
        with pytest.raises(lib.CellError) as e:
            c.displacement(0)
        assert e.value.status == lib.CELL_E_STATE
    monkeypatch.delenv("CELLFFT_DEBUG_NEGATE_Q")
    Cref, _, _ = fem.effective_stiffness(fem.Grid((16, 16, 16)), E, nu)
    with lib.Cell((16, 16, 16), precision=0, tol=1e-10) as c:
        c.set_material(E.ravel(), nu.ravel())
        C, info = c.effective_stiffness()
    assert info["status"] == "CELL_OK"
    assert np.abs(C - Cref).max() < 1e-10 * np.abs(Cref).max()


def _mean_iters(lib, n, seed):
    E, nu = ms.two_phase_grf(n, seed)
    with lib.Cell((n, n, n), precision=lib.MIXED, tol=1e-6) as c:
        c.set_material(E.ravel(), nu.ravel())
        _, info = c.effective_stiffness()
    assert info["status"] == "CELL_OK"
    return float(np.mean(info["iters"]))


def test_iterations_independent_of_grid_size(lib):
    ref = _mean_iters(lib, 256, 3)
    small = {n: np.mean([_mean_iters(lib, n, s) for s in seeds])
             for n, seeds in ((32, range(10, 18)), (64, range(20, 24)), (128, (30, 31)))}
    print("mean PCG iterations per load:", {256: ref, **small})
    for n, it in small.items():
        assert abs(it - ref) <= 0.2 * ref, (n, it, ref)
