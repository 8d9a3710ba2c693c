"""Cross-check of the GPU PCG against the strain-based projection variant
(oracle): both reach the same discrete solution in the same number of
iterations when stopped on the same residual ||f - K u||_2 <= tol ||f||_2
(the projection CG iterates are B u_k of the PCG with the same Fourier
reference preconditioner), so the per-load iteration counts of the FP64 GPU
solve equal the oracle's up to one iteration of rounding drift."""
import numpy as np
import pytest

from oracle import fem, strainproj as spj
from paper_2004_05197_amd import microstructures as ms

pytestmark = pytest.mark.gpu


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
    assert all(abs(a - b) <= 1 for a, b in zip(info["iters"], its)), (info["iters"], its)
    assert np.abs(C - C_ref).max() < 1e-8 * np.abs(C_ref).max()
