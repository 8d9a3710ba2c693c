"""The strain-based projection variant on the GPU (cell_solve_projection)
against the oracle's (oracle/strainproj.py) and against the displacement
PCG: both iterate B u_k of the PCG with the same Fourier reference
preconditioner, so stopped on the same residual ||f - K u||_2 <= tol ||f||_2
they take the same number of iterations (up to one of rounding drift) and
reach the same discrete solution (mean stresses against the oracle's direct
solve: 1e-8 relative at tol 1e-10, first order in the solver error)."""
import numpy as np
import pytest

from oracle import fem, strainproj as spj
from paper_2004_05197_amd import microstructures as ms

pytestmark = pytest.mark.gpu


def relerr(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


@pytest.mark.parametrize("n,contrast", [(16, 30.0), (24, 100.0)])
def test_iteration_counts_match_projection_cg(lib, n, contrast):
    mask, _, _ = ms.rsa_spheres(n, 0.25, seed=2, rmin=2.0, rmax=4.0)
    E = np.where(mask, contrast, 1.0)
    nu = np.full(E.shape, 0.3)
    g = fem.Grid((n, n, n))
    C_ref, its = spj.effective_stiffness(g, E, nu, tol=1e-9)
    with lib.Cell((n, n, n), precision=lib.FP64, tol=1e-9) as c:
        c.set_material(E.ravel(), nu.ravel())
        C, info = c.effective_stiffness()
        S, pinfo = c.solve_projection(np.eye(6))
    assert all(abs(a - b) <= 1 for a, b in zip(info["iters"], its)), (info["iters"], its)
    assert all(abs(a - b) <= 1 for a, b in zip(pinfo["iters"], its)), (pinfo["iters"], its)
    assert np.abs(C - C_ref).max() < 1e-8 * np.abs(C_ref).max()
    assert relerr(S.T, C_ref) < 1e-7


@pytest.mark.parametrize("shape,lengths", [((12, 8, 8), (1.0, 0.8, 0.7)), ((16, 16, 12), None)])
def test_projection_solution_matches_direct(lib, shape, lengths):
    rng = np.random.default_rng(3)
    nshape = tuple(reversed(shape))
    E = rng.uniform(1.0, 20.0, nshape)
    nu = rng.uniform(0.1, 0.4, nshape)
    g = fem.Grid(shape, lengths=lengths)
    C_ref, _, _ = fem.effective_stiffness(g, E, nu)
    eb = np.array([[1e-2, 0, 0, 0, 0, 0], [0, 0.3, -0.1, 0.2, 0, 0.05]])
    with lib.Cell(shape, precision=lib.FP64, tol=1e-11, lengths=g.L) as c:
        c.set_material(E.ravel(), nu.ravel())
        S, info = c.solve_projection(eb)
        S2, info2 = c.solve(eb)
    assert info["status"] == "CELL_OK"
    assert max(info["relres"][:2]) <= 1e-11
    assert relerr(S, eb @ C_ref.T) < 1e-9
    assert relerr(S, S2) < 1e-9
    assert all(abs(a - b) <= 1 for a, b in zip(info["iters"][:2], info2["iters"][:2]))


def test_projection_errors(lib):
    with lib.Cell((8, 8)) as c:
        c.set_material(np.full(64, 2.0), np.full(64, 0.3))
        with pytest.raises(lib.CellError) as e:
            c.solve_projection(np.eye(3))
        assert e.value.status == lib.CELL_E_UNSUPPORTED
    with lib.Cell((8, 8, 8)) as c:
        with pytest.raises(lib.CellError) as e:
            c.solve_projection(np.eye(6))
        assert e.value.status == lib.CELL_E_STATE
        c.set_material(np.full(512, 2.0), np.full(512, 0.3))
        S, info = c.solve_projection(np.eye(6))  # homogeneous: f = 0, no iteration
    assert info["iters"] == [0] * 6
    lam, mu = fem.lame(np.array(2.0), np.array(0.3))
    assert relerr(S, fem.D_voigt(float(lam), float(mu), 3)) < 1e-14
