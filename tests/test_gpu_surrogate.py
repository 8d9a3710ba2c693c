"""Surrogate stencil operator on the GPU against the oracle: the
interpolated stencil blocks, the operator, the constrained surrogate
solution and its C*, fewer load slots, sampled operator rows at the full
256^3 bench size, M = 1 and homogeneous material against the exact path,
the consistency error on a smooth field, and the error paths.

Tolerances: stencil blocks and the FP64 operator 1e-12 (the same sums in a
different order); FP32 operator 2e-5 (as the exact FP32 operator); C* of
FP64 solves at tol 1e-10: 1e-10, mixed at tol 1e-7: 1e-6."""
import numpy as np
import pytest

from oracle import fem, surrogate as sg

pytestmark = pytest.mark.gpu


def relerr(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


def smooth_field(shape, seed, amp=0.5):
    rng = np.random.default_rng(seed)
    d = len(shape)
    grids = np.meshgrid(*[np.arange(N) / N for N in reversed(shape)], indexing="ij")
    g = np.zeros(grids[0].shape)
    for _ in range(4):
        kv = rng.integers(-2, 3, size=d)
        ph = rng.uniform(0, 2 * np.pi)
        g += np.cos(2 * np.pi * sum(kv[a] * grids[d - 1 - a] for a in range(d)) + ph)
    return np.exp(amp * g / g.std())


# lattice sizes per axis from 1 (one sample: constant interpolant) to 6,
# both degrees, cubic and stretched cells; nx = 64 runs the FP32 operator
# with one wavefront per row (full tiles of 4 rows, and ny = 6: a partial
# tile)
CASES = [((8, 8, 8), 2, 1, None), ((8, 8, 8), 2, 3, None), ((12, 8, 4), 4, 3, (1.0, 1.1, 0.6)),
         ((12, 12, 6), 3, 1, (1.2, 1.0, 0.5)), ((8, 8, 8), 8, 3, None), ((24, 12, 12), 4, 3, None),
         ((64, 8, 4), 4, 3, None), ((64, 6, 4), 2, 1, (1.0, 0.7, 0.9))]


def case_data(shape, lengths, seed=1):
    g = fem.Grid(shape, lengths=lengths)
    rng = np.random.default_rng(seed)
    E = smooth_field(shape, seed) * rng.uniform(0.9, 1.1, g.nshape)
    nu = rng.uniform(0.2, 0.35, g.nshape)
    return g, E, nu


@pytest.mark.parametrize("case", range(len(CASES)))
def test_stencil_and_operator_match_oracle(lib, case):
    shape, M, q, lengths = CASES[case]
    g, E, nu = case_data(shape, lengths)
    K = fem.assemble_K(g, E, nu)
    St = sg.surrogate_stencils(g, E, nu, M, q, K=K)
    Kt = sg.surrogate_matrix(g, St)
    p = np.random.default_rng(2).standard_normal(3 * g.n)
    with lib.Cell(shape, precision=lib.MIXED, lengths=g.L) as c:
        c.set_material(E.ravel(), nu.ravel())
        c.set_surrogate(M, q)
        assert relerr(c.surrogate_stencil(), St) < 1e-12
        assert relerr(c.apply_operator(p, precision=lib.FP64), Kt @ p) < 1e-12
        assert relerr(c.apply_operator(p, precision=lib.MIXED), Kt @ p) < 2e-5


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("prec", [0, 1])
def test_solve_matches_oracle(lib, case, prec):
    shape, M, q, lengths = CASES[case]
    g, E, nu = case_data(shape, lengths)
    Cref, uref = sg.effective_stiffness(g, E, nu, M, q)
    with lib.Cell(shape, precision=prec, tol=1e-10 if prec == 0 else 1e-7, lengths=g.L) as c:
        c.set_material(E.ravel(), nu.ravel())
        c.set_surrogate(M, q)
        C, info = c.effective_stiffness()
        U = np.stack([c.displacement(J).ravel() for J in range(6)])
    assert info["status"] == "CELL_OK"
    assert relerr(C, Cref) < (1e-10 if prec == 0 else 1e-6)
    assert relerr(U, uref) < (1e-8 if prec == 0 else 1e-5)


@pytest.mark.parametrize("max_loads", [1, 2, 4])
def test_fewer_load_slots(lib, max_loads):
    """nx = 64 with fewer than six load slots (the unit loads solved in
    rounds): the FP32 operator computes all six slot positions and stores
    the unused ones over slot 0's output with slot 0's values; the surrogate
    solutions must match the oracle's as with six slots."""
    shape, M, q, lengths = CASES[6]
    g, E, nu = case_data(shape, lengths)
    _, uref = sg.effective_stiffness(g, E, nu, M, q)
    eb = fem.unit_loads(3)
    U = np.zeros_like(uref)
    with lib.Cell(shape, precision=lib.MIXED, tol=1e-7, max_loads=max_loads) as c:
        c.set_material(E.ravel(), nu.ravel())
        c.set_surrogate(M, q)
        for j0 in range(0, 6, max_loads):
            loads = eb[j0:j0 + max_loads]
            c.solve(loads)
            for k in range(len(loads)):
                U[j0 + k] = c.displacement(k).ravel()
    assert relerr(U, uref) < 1e-5


def test_M1_and_homogeneous_equal_the_exact_path(lib):
    shape = (8, 8, 8)
    g, E, nu = case_data(shape, None, seed=3)
    with lib.Cell(shape, precision=lib.FP64, tol=1e-11) as c:
        c.set_material(E.ravel(), nu.ravel())
        C0, _ = c.effective_stiffness()
        c.set_surrogate(1, 3)
        C1, _ = c.effective_stiffness()
        assert relerr(C1, C0) < 1e-10
        # homogeneous material: every stencil function is constant
        c.set_material(np.full(g.n, 4.0), np.full(g.n, 0.3))
        Ch, _ = c.effective_stiffness()
        c.set_surrogate(4, 1)
        Cs, _ = c.effective_stiffness()
        assert relerr(Cs, Ch) < 1e-12


def test_consistency_error_64(lib):
    """64^3 log-normal field (sigma 0.5, correlation length 12 voxels):
    C~*(M) - C* is positive semidefinite and shrinks as M decreases (q = 1
    and 3); the oracle cannot assemble this size, so the exact C* is the
    GPU's own exact path (checked against the oracle elsewhere)."""
    from paper_2004_05197_amd import microstructures as ms
    n = 64
    E, nu = ms.lognormal_field(n, 5, ell=12.0, sigma=0.5)
    with lib.Cell((n, n, n), precision=lib.MIXED, tol=1e-8) as c:
        c.set_material(E.ravel(), nu.ravel())
        C, _ = c.effective_stiffness()
        for q in (1, 3):
            errs = []
            for M in (8, 4, 2):
                c.set_surrogate(M, q)
                Ct, info = c.effective_stiffness()
                assert info["status"] == "CELL_OK"
                dC = 0.5 * (Ct - C + (Ct - C).T)
                assert np.linalg.eigvalsh(dC).min() > -1e-7 * np.abs(C).max()
                errs.append(np.abs(Ct - C).max() / np.abs(C).max())
            c.set_surrogate(0, 1)
            assert all(a > b for a, b in zip(errs[:-1], errs[1:])), errs
            assert errs[-1] < 1e-3


def test_full_size_sampled_rows(lib):
    """The 256^3 bench configuration (log-normal E, sigma 1, correlation
    length 32 voxels, seed 7; M 4, cubic): rows of the surrogate operator at
    40 nodes (box corners and tile edges among them) against the oracle's
    per-node evaluation.  FP32 operator (one wavefront per row) within 2e-5,
    FP64 operator within 1e-11 of the largest sampled value; p is FP32-exact
    so that both see the same direction."""
    from paper_2004_05197_amd import microstructures as ms
    n = 256
    E, nu = ms.lognormal_field(n, 7, ell=32.0, sigma=1.0)
    g = fem.Grid((n, n, n))
    rng = np.random.default_rng(3)
    p = rng.standard_normal(3 * g.n).astype(np.float32).astype(np.float64)
    special = [(0, 0, 0), (255, 255, 255), (0, 255, 128), (255, 0, 0), (63, 3, 17), (64, 4, 200), (127, 0, 255),
               (128, 255, 1), (191, 100, 0), (192, 7, 254)]
    nodes = np.array([x + n * (y + n * z) for x, y, z in special] + list(rng.choice(g.n, size=30, replace=False)))
    ref = sg.apply_at(g, E, nu, 4, 3, p, nodes)
    with lib.Cell((n, n, n), precision=lib.MIXED) as c:
        c.set_material(E.ravel(), nu.ravel())
        c.set_surrogate(4, 3)
        for prec, tol in ((lib.MIXED, 2e-5), (lib.FP64, 1e-11)):
            q = c.apply_operator(p, precision=prec).reshape(3, g.n)[:, nodes].T
            assert relerr(q, ref) < tol, (prec, relerr(q, ref))


@pytest.mark.parametrize("shape,M,q,lengths", [((192, 8, 6), 2, 3, None), ((128, 4, 12), 4, 1, (1.3, 0.9, 1.0))])
def test_sampled_rows_wide_grids(lib, shape, M, q, lengths):
    """Grids of 2 and 3 wavefront-wide tiles per row (the FP32 operator with
    one wavefront per row, tile seams at x = 63/64 and 127/128) and a
    stretched cell: 60 sampled rows of the surrogate operator against the
    oracle's per-node evaluation, FP32 2e-5 and FP64 1e-11 of the largest."""
    g, E, nu = case_data(shape, lengths, seed=4)
    rng = np.random.default_rng(5)
    p = rng.standard_normal(3 * g.n).astype(np.float32).astype(np.float64)
    nx, ny, nz = shape
    seams = [(x, y, z) for x in (0, 63, 64, 127, nx - 1) for y in (0, ny - 1) for z in (0, nz - 1) if x < nx]
    nodes = np.array([x + nx * (y + ny * z) for x, y, z in seams] + list(rng.choice(g.n, size=60 - len(seams),
                                                                                    replace=False)))
    ref = sg.apply_at(g, E, nu, M, q, p, nodes)
    with lib.Cell(shape, precision=lib.MIXED, lengths=g.L) as c:
        c.set_material(E.ravel(), nu.ravel())
        c.set_surrogate(M, q)
        for prec, tol in ((lib.MIXED, 2e-5), (lib.FP64, 1e-11)):
            got = c.apply_operator(p, precision=prec).reshape(3, g.n)[:, nodes].T
            assert relerr(got, ref) < tol, (prec, relerr(got, ref))


def test_surrogate_errors(lib):
    with lib.Cell((8, 8)) as c:
        c.set_material(np.full(64, 2.0), np.full(64, 0.3))
        with pytest.raises(lib.CellError) as e:
            c.set_surrogate(2, 1)
        assert e.value.status == lib.CELL_E_UNSUPPORTED
    with lib.Cell((8, 8, 8)) as c:
        with pytest.raises(lib.CellError) as e:
            c.set_surrogate(2, 1)
        assert e.value.status == lib.CELL_E_STATE
        c.set_material(np.full(512, 2.0), np.full(512, 0.3))
        for M, q in ((3, 1), (2, 2), (-1, 3)):
            with pytest.raises(lib.CellError) as e:
                c.set_surrogate(M, q)
            assert e.value.status == lib.CELL_E_ARG
        c.set_surrogate(2, 3)
        C, _ = c.effective_stiffness()
        with pytest.raises(lib.CellError) as e:
            c.adjoint(np.eye(6))
        assert e.value.status == lib.CELL_E_STATE
        # a new material switches the surrogate off
        c.set_material(np.full(512, 3.0), np.full(512, 0.3))
        with pytest.raises(lib.CellError) as e:
            c.surrogate_stencil()
        assert e.value.status == lib.CELL_E_STATE


def test_surrogate_off_drops_its_results(lib):
    """Switching the surrogate operator off (M = 0) after a surrogate solve
    leaves no result that could pass for the exact operator's: the adjoint,
    the displacement, residual and energy-matrix getters report CELL_E_STATE
    until the next exact solve, whose adjoint then works."""
    rng = np.random.default_rng(12)
    E = np.exp(0.3 * rng.standard_normal(512))
    nu = np.full(512, 0.3)
    with lib.Cell((8, 8, 8), precision=lib.FP64, tol=1e-10) as c:
        c.set_material(E, nu)
        c.set_surrogate(2, 3)
        c.effective_stiffness()
        c.set_surrogate(0)
        for call in (lambda: c.adjoint(np.eye(6)), lambda: c.displacement(0), lambda: c.residual(0),
                     lambda: c.energy_matrix(6)):
            with pytest.raises(lib.CellError) as e:
                call()
            assert e.value.status == lib.CELL_E_STATE
        C, _ = c.effective_stiffness()
        g = c.adjoint(np.eye(6))
    grid = fem.Grid((8, 8, 8))
    Cref, _, _ = fem.effective_stiffness(grid, E.reshape(8, 8, 8), nu.reshape(8, 8, 8))
    assert relerr(C, Cref) < 1e-10
    assert np.all(np.isfinite(g))
