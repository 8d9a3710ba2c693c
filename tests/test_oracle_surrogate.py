"""Pins of the surrogate-stencil oracle (CPU): the B-spline interpolation
against scipy's periodic splines and numpy's periodic linear interpolation,
M = 1 and homogeneous material reproduce K exactly, symmetry, the translation
kernel where the stencil blocks are symmetric, the energy-form upper bound
C~* - C* >= 0 with its quadratic size, convergence as M decreases, and the
per-node versions (stencil blocks from element matrices, interpolants and
rows of Kt p at chosen nodes) against the assembled sparse matrices."""
import numpy as np
import pytest
from scipy.interpolate import make_interp_spline

from oracle import fem, surrogate as sg


def smooth_field(shape, seed, amp=0.5):
    """exp(amp g), g a standardised sum of four low-frequency cosines."""
    rng = np.random.default_rng(seed)
    d = len(shape)
    grids = np.meshgrid(*[np.arange(N) / N for N in reversed(shape)], indexing="ij")
    g = np.zeros(grids[0].shape)
    for _ in range(4):
        kv = rng.integers(-2, 3, size=d)
        ph = rng.uniform(0, 2 * np.pi)
        g += np.cos(2 * np.pi * sum(kv[a] * grids[d - 1 - a] for a in range(d)) + ph)
    return np.exp(amp * g / g.std())


@pytest.mark.parametrize("Nc,M", [(6, 4), (5, 3), (2, 4), (1, 4)])
def test_bspline_interpolation_matches_libraries(Nc, M):
    rng = np.random.default_rng(Nc * 10 + M)
    v = rng.standard_normal(Nc)
    x = np.arange(Nc * M) / M
    cub = sg.evaluate(sg.interpolation_coefficients(v[None], 3, 1), 3, M, (Nc * M,))[0]
    if Nc >= 2:
        spl = make_interp_spline(np.arange(Nc + 1), np.append(v, v[0]), k=3, bc_type="periodic")
        assert np.abs(cub - spl(x)).max() < 1e-13
    else:
        assert np.abs(cub - v[0]).max() < 1e-14
    lin = sg.evaluate(sg.interpolation_coefficients(v[None], 1, 1), 1, M, (Nc * M,))[0]
    ref = np.interp(x, np.arange(Nc + 1), np.append(v, v[0]))
    assert np.abs(lin - ref).max() < 1e-14
    # both interpolate: the samples come back at the knots
    assert np.abs(cub[::M] - v).max() < 1e-13 and np.abs(lin[::M] - v).max() < 1e-15


def test_tensor_product_interpolation_2d():
    rng = np.random.default_rng(3)
    v = rng.standard_normal((3, 4))     # (y, x) lattice
    M = 2
    fine = sg.evaluate(sg.interpolation_coefficients(v[None], 3, 2), 3, M, (6, 8))[0]
    # separable: interpolate rows in x, then columns in y, with scipy
    sx = [make_interp_spline(np.arange(5), np.append(r, r[0]), k=3, bc_type="periodic")(np.arange(8) / M) for r in v]
    sx = np.array(sx)
    ref = np.array([make_interp_spline(np.arange(4), np.append(col, col[0]), k=3,
                                       bc_type="periodic")(np.arange(6) / M) for col in sx.T]).T
    assert np.abs(fine - ref).max() < 1e-13


@pytest.mark.parametrize("shape", [(4, 4, 3), (5, 4)])
@pytest.mark.parametrize("q", [1, 3])
def test_M1_reproduces_K(shape, q):
    rng = np.random.default_rng(1)
    g = fem.Grid(shape)
    E = rng.uniform(1, 5, g.nshape)
    nu = rng.uniform(0.1, 0.4, g.nshape)
    K = fem.assemble_K(g, E, nu)
    Kt = sg.surrogate_matrix(g, sg.surrogate_stencils(g, E, nu, 1, q, K=K))
    assert abs(Kt - K).max() < 1e-13 * abs(K).max()


@pytest.mark.parametrize("shape,M", [((4, 4, 4), 2), ((8, 4, 4), 4), ((6, 6), 3)])
@pytest.mark.parametrize("q", [1, 3])
def test_homogeneous_material_is_exact(shape, M, q):
    g = fem.Grid(shape, lengths=[1.0 + 0.2 * a for a in range(len(shape))])
    E, nu = np.full(g.nshape, 3.0), np.full(g.nshape, 0.3)
    K = fem.assemble_K(g, E, nu)
    Kt = sg.surrogate_matrix(g, sg.surrogate_stencils(g, E, nu, M, q, K=K))
    assert abs(Kt - K).max() < 1e-13 * abs(K).max()


def test_symmetry_and_translations():
    """Kt is symmetric for any field; K keeps the three translations in its
    kernel exactly, Kt up to the interpolation error of the blocks' skew
    parts."""
    g = fem.Grid((6, 6, 6))
    E = smooth_field(g.shape, 2)
    nu = np.full(g.nshape, 0.3)
    K = fem.assemble_K(g, E, nu)
    Kt = sg.surrogate_matrix(g, sg.surrogate_stencils(g, E, nu, 2, 3, K=K))
    assert abs(Kt - Kt.T).max() == 0.0
    for c in range(3):
        t = np.zeros(3 * g.n)
        t[c * g.n:(c + 1) * g.n] = 1.0
        assert np.abs(K @ t).max() < 1e-13 * abs(K).max()
        assert np.abs(Kt @ t).max() < 0.05 * abs(K).max()


@pytest.mark.parametrize("shape,Ms", [((48, 48), (8, 4, 2)), ((12, 12, 12), (4, 2))])
@pytest.mark.parametrize("q", [1, 3])
def test_consistency_error(shape, Ms, q):
    """C~* - C* is positive semidefinite (the exact energy of a non-optimal
    fluctuation), equals (u~ - u).K(u~ - u)/|Y| and shrinks with M; M = 1
    reproduces C*."""
    g = fem.Grid(shape)
    E = smooth_field(shape, 1)
    nu = np.full(g.nshape, 0.3)
    K = fem.assemble_K(g, E, nu)
    C, _, u = fem.effective_stiffness(g, E, nu, K=K)
    errs = []
    for M in Ms + (1,):
        Ct, ut = sg.effective_stiffness(g, E, nu, M, q)
        dC = Ct - C
        assert np.linalg.eigvalsh(0.5 * (dC + dC.T)).min() > -1e-12 * abs(C).max()
        du = ut - u
        quad = np.array([[du[I] @ (K @ du[J]) for J in range(g.nv)] for I in range(g.nv)]) / g.volume
        assert np.abs(dC - quad).max() < 1e-9 * abs(C).max()
        errs.append(abs(dC).max() / abs(C).max())
    assert errs[-1] < 1e-13
    assert all(a > b for a, b in zip(errs[:-1], errs[1:]))


@pytest.mark.parametrize("shape,M,q,lengths", [((6, 4, 4), 2, 3, None), ((8, 4, 6), 2, 1, (1.0, 0.8, 1.3)),
                                                ((4, 6, 4), 1, 3, None), ((6, 6), 3, 3, None)])
def test_per_node_versions_match_assembly(shape, M, q, lengths):
    """stencil_blocks_at against K read off the assembled matrix, and
    surrogate_blocks_at / apply_at against surrogate_stencils /
    surrogate_matrix @ p (sparse assembly) at random nodes."""
    rng = np.random.default_rng(11)
    g = fem.Grid(shape, lengths=lengths)
    E = rng.uniform(1, 3, g.nshape)
    nu = rng.uniform(0.2, 0.35, g.nshape)
    lam, mu = fem.lame(E.ravel(), nu.ravel())
    K = fem.assemble_K(g, E, nu)
    Sf = sg.stencil_functions(g, K)
    Sa = sg.stencil_blocks_at(g, lam, mu, np.arange(g.n))
    assert np.abs(np.moveaxis(Sa, 0, -1) - Sf).max() < 1e-14 * np.abs(Sf).max()
    St = sg.surrogate_stencils(g, E, nu, M, q, K=K)
    nodes = rng.choice(g.n, size=10, replace=False)
    Sb = sg.surrogate_blocks_at(g, E, nu, M, q, nodes)
    assert np.abs(np.moveaxis(Sb, 0, -1) - St[..., nodes]).max() < 1e-14 * np.abs(St).max()
    p = rng.standard_normal(g.d * g.n)
    ref = (sg.surrogate_matrix(g, St) @ p).reshape(g.d, g.n)[:, nodes].T
    assert np.abs(sg.apply_at(g, E, nu, M, q, p, nodes) - ref).max() < 1e-14 * np.abs(ref).max()
