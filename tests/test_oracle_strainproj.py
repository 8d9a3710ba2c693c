"""Pins of the strain-based projection variant (CPU): its CG iterates are
B u_k of the displacement PCG (same iteration count and residual history,
same final strains), and its effective stiffness equals the direct solve's."""
import numpy as np
import pytest

from oracle import fem, matfree, strainproj as spj
from paper_2004_05197_amd import microstructures as ms


def test_iterates_are_the_displacement_pcg_strains():
    g = fem.Grid((12, 12, 12))
    mask, _, _ = ms.rsa_spheres(12, 0.25, seed=1, rmin=1.5, rmax=3.0)
    E = np.where(mask, 30.0, 1.0)
    nu = np.full(E.shape, 0.3)
    el = spj._fields(g)
    for J in (0, 4):
        eb = np.eye(6)[J]
        hist_u = []
        u, it_u, _ = matfree.pcg(g, E, nu, eb, tol=1e-10, callback=lambda it, r: hist_u.append(r))
        e, it_e, hist = spj.projection_cg(g, E, nu, eb, tol=1e-10)
        assert it_e == it_u
        assert max(abs(a - b) / b for a, b in zip(hist_u, hist[1:])) < 1e-3
        Bu = spj.strains(g, el, u.ravel())
        scale = max(np.abs(b).max() for b in Bu)
        assert max(np.abs(a - b).max() for a, b in zip(e, Bu)) < 1e-9 * scale


@pytest.mark.parametrize("shape", [(6, 6, 6), (16, 12)])
def test_effective_stiffness_equals_direct(shape):
    rng = np.random.default_rng(4)
    g = fem.Grid(shape, lengths=[1.0 + 0.1 * a for a in range(len(shape))])
    E = rng.uniform(1.0, 20.0, g.nshape)
    nu = rng.uniform(0.15, 0.4, g.nshape)
    C, its = spj.effective_stiffness(g, E, nu, tol=1e-12)
    Cd, _, _ = fem.effective_stiffness(g, E, nu)
    assert np.abs(C - Cd).max() < 1e-10 * np.abs(Cd).max()
    assert all(i > 0 for i in its)
