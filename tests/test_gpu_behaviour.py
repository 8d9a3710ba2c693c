"""PCG behaviour on the GPU: the breakdown status forced from the host, and
iteration counts that do not grow with the grid at fixed microstructure
statistics.

Breakdown: CELLFFT_DEBUG_NEGATE_Q=1 (read when a handle is created) makes
the linear K-apply write -K p, so the first p.Kp is negative.  Every kernel
of the iteration still runs to its normal end (the slot state turns to
breakdown in the finalize kernel and later launches skip the slot); the
solve must report CELL_E_BREAKDOWN and a handle created afterwards must
solve normally.

Stagnation: a tolerance below what the arithmetic can reach (1e-20) leaves
the true residual on a plateau; with CELLFFT_STAG_WINDOW=40 the solve
refreshes and restarts once, then ends the loads with CELL_NOT_CONVERGED
long before max_iter, keeping the best iterate (C* still equal to the
direct solve).  With the window off, the same solve runs to max_iter.  A
batch of two cell sizes ends the same way (both groups polled with the
same check).

Iteration counts: the Fourier preconditioner is spectrally equivalent to
the operator with bounds set by the local ratios of the material to the
reference medium (K/K_0 and mu/mu_0 per voxel), not by the voxel size, so
one microstructure resolved on finer and finer grids needs the same number
of PCG iterations.  The microstructure here is the thresholded Gaussian
random field of the 256^3 workload (correlation length 8 of its voxels,
contrast 1:1000), sampled at every k-th voxel for the coarser grids
(64^3 and 128^3: correlation length 2 and 4 of their voxels), within +-20 %
of the 256^3 count.  (Cells of fixed correlation length in voxels grow in
physical size with N instead; measured at tol 1e-6, their counts rise from
67 at 32^3 over 101 and 166 to 190 at 256^3, as a larger cell fills the
spectrum between the bounds.  That is the cell size, not the resolution.)
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


@pytest.mark.parametrize("prec", [0, 1])
def test_stagnation_ends_unreachable_tolerance(lib, monkeypatch, prec):
    mask, _, _ = ms.rsa_spheres(16, 0.3, seed=2, rmin=1.0, rmax=2.0)
    E = np.where(mask, 20.0, 1.0)
    nu = np.full(E.shape, 0.3)
    Cref, _, _ = fem.effective_stiffness(fem.Grid((16, 16, 16)), E, nu)
    monkeypatch.setenv("CELLFFT_STAG_WINDOW", "40")
    with lib.Cell((16, 16, 16), precision=prec, tol=1e-20, max_iter=3000) as c:
        c.set_material(E.ravel(), nu.ravel())
        C, info = c.effective_stiffness()
        msg = lib.last_error()
    print("stagnation:", prec, info["iters"], info["relres"], info["refinements"])
    assert info["status"] == "CELL_NOT_CONVERGED"
    assert "stagnated" in msg
    assert max(info["iters"]) < 1500
    assert max(info["relres"]) < (1e-13 if prec == 0 else 1e-9)
    assert np.abs(C - Cref).max() < (1e-10 if prec == 0 else 1e-8) * np.abs(Cref).max()
    monkeypatch.setenv("CELLFFT_STAG_WINDOW", "0")
    with lib.Cell((16, 16, 16), precision=prec, tol=1e-20, max_iter=200) as c:
        c.set_material(E.ravel(), nu.ravel())
        C, info = c.effective_stiffness()
    assert info["status"] == "CELL_NOT_CONVERGED"
    assert min(info["iters"]) >= 200
    monkeypatch.delenv("CELLFFT_STAG_WINDOW")


def test_stagnation_in_a_batch(lib, monkeypatch):
    # the batch polls every group with the same check: cells of two sizes
    # with an unreachable tolerance end early, the status is the worst one
    monkeypatch.setenv("CELLFFT_STAG_WINDOW", "40")
    shapes = [(16, 16, 16), (12, 12, 12)]
    with lib.Batch(shapes, precision=lib.MIXED, tol=1e-20, max_iter=3000) as b:
        for i, sh in enumerate(shapes):
            m, _, _ = ms.rsa_spheres(sh[0], 0.3, seed=20 + i, rmin=1.0, rmax=2.0)
            b.set_material(i, np.where(m, 20.0, 1.0).ravel(), np.full(m.size, 0.3))
        C, infos = b.effective_stiffness()
        msg = lib.last_error()
    monkeypatch.delenv("CELLFFT_STAG_WINDOW")
    print("batch stagnation:", [i["iters"] for i in infos], [max(i["relres"]) for i in infos])
    assert all(i["status"] == "CELL_NOT_CONVERGED" for i in infos)
    assert "stagnated" in msg
    for i in infos:
        assert max(i["iters"]) < 1500
        assert max(i["relres"]) < 1e-9
    for k, sh in enumerate(shapes):
        m, _, _ = ms.rsa_spheres(sh[0], 0.3, seed=20 + k, rmin=1.0, rmax=2.0)
        E = np.where(m, 20.0, 1.0)
        Cref, _, _ = fem.effective_stiffness(fem.Grid(sh), E, np.full(E.shape, 0.3))
        assert np.abs(C[k] - Cref).max() < 1e-8 * np.abs(Cref).max()


def _mean_iters(lib, g):
    n = g.shape[0]
    E = np.where(g >= 0.0, 1000.0, 1.0)
    nu = np.where(g >= 0.0, 0.35, 0.25)
    with lib.Cell((n, n, n), precision=lib.MIXED, tol=1e-6) as c:
        c.set_material(E.ravel(), nu.ravel())
        _, info = c.effective_stiffness()
    assert info["status"] == "CELL_OK"
    return float(np.mean(info["iters"]))


def test_iterations_independent_of_resolution(lib):
    g = ms.gaussian_random_field((256, 256, 256), 8.0, 3)
    its = {n: _mean_iters(lib, np.ascontiguousarray(g[::256 // n, ::256 // n, ::256 // n]))
           for n in (32, 64, 128, 256)}
    print("mean PCG iterations per load:", its)
    for n in (64, 128):
        assert abs(its[n] - its[256]) <= 0.2 * its[256], (n, its)
