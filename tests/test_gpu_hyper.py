"""Neo-Hookean cell problem on the GPU (Newton's method with the PCG inner
solves) against the oracle: mean stress, energy and fluctuation of the
direct-solve Newton on small grids, the exact laminate solution, the
homogeneous and small-strain limits, frame indifference and, at 64^3, the
oracle's residual of the GPU solution.

Tolerances: the Newton iteration stops at ||f|| <= 1e-11 of the load scale
(FP64 residuals in both precisions), so the mean stress agrees with the
oracle to ~1e-9 relative and the fluctuation to ~1e-8.
"""
import numpy as np
import pytest

from oracle import fem, hyper
from paper_2004_05197_amd import microstructures as ms
from closed_forms import laminate_neohooke

pytestmark = pytest.mark.gpu


def relerr(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


def rand_case(shape, seed, amp=0.08):
    rng = np.random.default_rng(seed)
    nshape = tuple(reversed(shape))
    E = rng.uniform(1.0, 10.0, nshape)
    nu = rng.uniform(0.1, 0.4, nshape)
    d = len(shape)
    F = [np.eye(d) + amp * rng.standard_normal((d, d)) for _ in range(2)]
    return E, nu, np.stack(F)


STEP_CASES = [((4, 4, 4), None), ((8, 6, 4), None), ((8, 6), None), ((12, 8), None), ((12, 4, 6), None),
              ((32, 16, 12), None), ((16, 32, 24), None), ((32, 32, 16), (1.0, 1.0, 0.5))]


@pytest.mark.parametrize("case", range(len(STEP_CASES)))
@pytest.mark.parametrize("prec", [0, 1])
def test_steps_match_oracle(lib, case, prec):
    """One residual (FP64) and one tangent product (in the handle's
    precision) at a random state against the oracle's f(u), Pi(u), the
    stress sum and the assembled K_T(u) p.  Grids whose x and y sizes are
    multiples of 16 run the tiled kernels (several x, y and z tiles, a
    ragged last z tile; the last case has equal spacings, the uniform-grid
    variant), the others the node-centric ones.  The state moves nodes by
    ~0.05 h, so every simplex keeps J >~ 0.5: there a float32 evaluation of
    the same formulas stays within 2e-7 of FP64 (checked with numpy), and
    3e-6 leaves room for the hardware reciprocal and logarithm."""
    shape, lengths = STEP_CASES[case]
    d = len(shape)
    E, nu, Fb = rand_case(shape, 5, amp=0.1)
    grid = fem.Grid(shape, lengths=lengths or [1.0 + 0.1 * a for a in range(d)])
    rng = np.random.default_rng(6)
    u = 0.05 * min(grid.h) * rng.standard_normal((d, grid.n))
    p = rng.standard_normal((d, grid.n))
    with lib.Cell(shape, precision=prec, lengths=grid.L) as c:
        c.set_material(E.ravel(), nu.ravel())
        f, sums = c.hyper_residual(Fb[0], u)
        q = c.hyper_tangent(Fb[0], u, p)
    fo = hyper.residual(grid, E, nu, u, Fb[0])
    assert relerr(f.reshape(d, -1), fo) < 1e-12
    assert abs(sums[0] - hyper.total_energy(grid, E, nu, u, Fb[0])) < 1e-12 * abs(sums[0])
    Ps = sums[1:].reshape(3, 3)[:d, :d]
    assert relerr(Ps, hyper.mean_piola(grid, E, nu, u, Fb[0]) * grid.volume) < 1e-12
    qo = hyper.assemble_tangent(grid, E, nu, u, Fb[0]) @ p.ravel()
    assert relerr(q, qo) < (1e-12 if prec == 0 else 3e-6)


@pytest.mark.parametrize("shape", [(4, 4, 4), (8, 6, 4), (8, 6), (12, 8)])
@pytest.mark.parametrize("prec", [0, 1])
def test_newton_matches_oracle(lib, shape, prec):
    E, nu, Fb = rand_case(shape, 1)
    grid = fem.Grid(shape, lengths=[1.0 + 0.1 * a for a in range(len(shape))])
    with lib.Cell(shape, precision=prec, tol=1e-10 if prec == 0 else 1e-6, lengths=grid.L) as c:
        c.set_material(E.ravel(), nu.ravel())
        P, info = c.solve_hyper(Fb, tol=1e-11)
        U = [c.displacement(J) for J in range(2)]
    assert info["status"] == "CELL_OK"
    for J in range(2):
        ref = hyper.newton(grid, E, nu, Fb[J], tol=1e-13)
        assert relerr(P[J], ref["P_mean"]) < 1e-9, J
        assert abs(info["energy"][J] - ref["energy"]) < 1e-10 * abs(ref["energy"])
        assert relerr(U[J], ref["u"]) < 1e-7, J
        assert info["newton_iters"][J] <= ref["iterations"] + 2
        assert info["resnorm"][J] <= 1e-11


@pytest.mark.parametrize("prec", [0, 1])
def test_indefinite_tangent(lib, prec):
    """F_bar with det 0.52: K_T(0) has negative eigenvalues (the oracle's
    assembled tangent, checked here), so the first inner PCG meets
    p.K_T p <= 0 and stops; Newton still reaches the oracle's minimiser
    (K_T positive definite there)."""
    shape = (8, 6)
    E, nu, Fb = rand_case(shape, 1, amp=0.15)
    grid = fem.Grid(shape, lengths=[1.0, 1.1])
    K0 = hyper.assemble_tangent(grid, E, nu, np.zeros((2, grid.n)), Fb[0]).toarray()
    assert np.linalg.eigvalsh(K0)[0] < -0.1
    ref = hyper.newton(grid, E, nu, Fb[0], tol=1e-13)
    Kf = hyper.assemble_tangent(grid, E, nu, ref["u"], Fb[0]).toarray()
    assert np.linalg.eigvalsh(Kf)[2] > 0.1
    with lib.Cell(shape, precision=prec, tol=1e-10 if prec == 0 else 1e-6, lengths=grid.L) as c:
        c.set_material(E.ravel(), nu.ravel())
        P, info = c.solve_hyper(Fb[:1], tol=1e-11)
        u = c.displacement(0)
    assert info["status"] == "CELL_OK"
    assert info["indefinite_steps"][0] >= 1
    assert relerr(P[0], ref["P_mean"]) < 1e-9
    assert relerr(u, ref["u"]) < 1e-7


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("shape", [(24, 4, 4), (48, 16, 16), (24, 6)])
def test_laminate_exact(lib, shape, prec):
    """Layers normal to x under a general F_bar: the exact solution is
    piecewise homogeneous (the scalar-per-layer closed form).  (48, 16, 16)
    runs the tiled kernels (tangent, FP64 residual and energy)."""
    d = len(shape)
    nx = shape[0]
    thick = [nx // 3, nx - nx // 3]
    Eph, nuph = [1.0, 20.0], [0.25, 0.35]
    nshape = tuple(reversed(shape))
    E = np.broadcast_to(np.concatenate([np.full(t, e) for t, e in zip(thick, Eph)]), nshape).copy()
    nu = np.broadcast_to(np.concatenate([np.full(t, v) for t, v in zip(thick, nuph)]), nshape).copy()
    Fb = np.eye(d)
    Fb[0, 0] = 1.3
    Fb[1, 0] = 0.25
    Fb[0, 1] = -0.15
    with lib.Cell(shape, precision=prec, tol=1e-10 if prec == 0 else 1e-6) as c:
        c.set_material(E.ravel(), nu.ravel())
        P, info = c.solve_hyper(Fb[None], tol=1e-12)
    phases = [tuple(float(x) for x in fem.lame(e, v)) for e, v in zip(Eph, nuph)]
    Pex, Wex = laminate_neohooke(phases, [t / nx for t in thick], Fb)
    assert relerr(P[0], Pex) < 1e-9
    assert abs(info["energy"][0] - Wex) < 1e-9 * abs(Wex)
    assert info["newton_iters"][0] >= 2


def test_homogeneous_and_small_strain(lib):
    shape = (16, 16, 16)
    grid = fem.Grid(shape)
    nshape = tuple(reversed(shape))
    with lib.Cell(shape, precision=lib.FP64, tol=1e-12) as c:
        c.set_material(np.full(grid.n, 3.0), np.full(grid.n, 0.3))
        Fb = np.eye(3) + 0.1 * np.random.default_rng(2).standard_normal((3, 3))
        P, info = c.solve_hyper(Fb[None])
        lam, mu = fem.lame(3.0, 0.3)
        Pex = hyper.piola(Fb[None], np.array([lam]), np.array([mu]))[0]
        assert info["newton_iters"][0] == 0
        assert relerr(P[0], Pex) < 1e-12
        # small strain: P / eps -> C* sym(H) of the linear GPU solve
        mask, _, _ = ms.rsa_spheres(16, 0.25, seed=3, rmin=2.0, rmax=3.0)
        E = np.where(mask, 15.0, 1.0)
        c.set_material(E.ravel(), np.full(grid.n, 0.3))
        C, _ = c.effective_stiffness()
        H = np.random.default_rng(4).standard_normal((3, 3))
        Hs = 0.5 * (H + H.T)
        pairs = fem.voigt_pairs(3)
        ev = np.array([Hs[a, b] if a == b else 2 * Hs[a, b] for a, b in pairs])
        S = np.zeros((3, 3))
        for v, (a, b) in zip(C @ ev, pairs):
            S[a, b] = S[b, a] = v
        eps = 1e-5
        P, info = c.solve_hyper((np.eye(3) + eps * H)[None], tol=1e-12)
        assert relerr(P[0] / eps, S) < 50 * eps
        # the linear results are invalid after a nonlinear solve
        with pytest.raises(lib.CellError) as e:
            c.energy_matrix(6)
        assert e.value.status == lib.CELL_E_STATE


def test_spheres64_frame_indifference_and_oracle_residual(lib):
    """64^3 RSA spheres (vf 0.3, E 1:10): uniaxial stretch 1.15 and a
    rotated copy in one batched Newton solve; R P equals the rotated stress,
    the energies agree, and the oracle's residual of the GPU fluctuation
    (full 64^3 grid, FP64 numpy) is below the stopping tolerance."""
    n = 64
    E, nu, _ = ms.spheres_cell(n, 0.3, seed=2, contrast=10.0)
    grid = fem.Grid((n, n, n))
    c_, s_ = np.cos(0.4), np.sin(0.4)
    R = np.array([[c_, -s_, 0], [s_, c_, 0], [0, 0, 1.0]])
    F0 = np.diag([1.15, 1.0, 1.0])
    Fb = np.stack([F0, R @ F0])
    with lib.Cell((n, n, n), precision=lib.MIXED, tol=1e-6) as c:
        c.set_material(E.ravel(), nu.ravel())
        P, info = c.solve_hyper(Fb, tol=1e-10)
        u = c.displacement(0)
    assert info["status"] == "CELL_OK"
    assert relerr(R @ P[0], P[1]) < 1e-8
    assert abs(info["energy"][0] - info["energy"][1]) < 1e-9 * info["energy"][0]
    f = hyper.residual(grid, E, nu, u, F0)
    lam, mu = fem.lame(E.ravel(), nu.ravel())
    scale = grid.volume * float(np.max(np.abs(lam) + 2 * mu)) * 1.15
    assert np.linalg.norm(f) <= 2e-10 * scale
    # stress bounded by the phase stresses of the homogeneous deformation
    Ps = [hyper.piola(F0[None], *[np.array([x]) for x in fem.lame(e, 0.3)])[0] for e in (1.0, 10.0)]
    assert Ps[0][0, 0] < P[0][0, 0] < Ps[1][0, 0]


def test_hyper256_bench_configuration(lib):
    """The neo-Hookean workload of the benchmark at full size: 256^3 grf3d
    geometry (E 1:10, nu .25/.35), six 5 % stretch and shear loads, mixed
    inner solves, Newton tol 1e-8.  At 64 sampled nodes per load the
    oracle's residual of the GPU fluctuation is below the stopping level,
    and the GPU's own FP64 residual (tiled kernel) equals it."""
    n = 256
    E, nu = ms.two_phase_grf(n, seed=3, E_hard=10.0)
    Fb = np.tile(np.eye(3), (6, 1, 1))
    for a in range(3):
        Fb[a, a, a] += 0.05
    for J, (a, b) in enumerate([(1, 2), (0, 2), (0, 1)]):
        Fb[3 + J, a, b] = 0.05
    grid = fem.Grid((n, n, n))
    lam, mu = fem.lame(E.ravel(), nu.ravel())
    scale = grid.volume * float(np.max(np.abs(lam) + 2 * mu)) * 1.05
    nodes = np.random.default_rng(7).choice(grid.n, 64, replace=False)
    with lib.Cell((n, n, n), precision=lib.MIXED, tol=1e-6) as c:
        c.set_material(E.ravel(), nu.ravel())
        P, info = c.solve_hyper(Fb, tol=1e-8)
        assert info["status"] == "CELL_OK", info
        U = [c.displacement(J) for J in range(6)]  # (a single-step call ends the solve's results)
        for J in range(6):
            u = U[J]
            fo = hyper.residual_at_nodes(grid, E, nu, u, Fb[J], nodes)
            assert np.abs(fo).max() <= 2e-8 * scale, (J, np.abs(fo).max() / scale)
            fg, _ = c.hyper_residual(Fb[J], u)
            fg = fg.reshape(3, -1)[:, nodes].T
            assert np.abs(fg - fo).max() <= 1e-12 * scale
    assert all(k <= 6 for k in info["newton_iters"])


def test_hyper_errors(lib):
    with lib.Cell((8, 8, 8)) as c:
        with pytest.raises(lib.CellError) as e:
            c.solve_hyper(np.eye(3)[None])
        assert e.value.status == lib.CELL_E_STATE
        c.set_material(np.full(512, 2.0), np.full(512, 0.3))
        with pytest.raises(lib.CellError) as e:
            c.solve_hyper(np.diag([1.0, 1.0, -1.0])[None])
        assert e.value.status == lib.CELL_E_ARG
        with pytest.raises(lib.CellError) as e:
            c.solve_hyper(np.eye(3)[None], tol=-1.0)
        assert e.value.status == lib.CELL_E_ARG
        for bad in (np.zeros((0, 3, 3)), np.tile(np.eye(3), (7, 1, 1)), np.full((1, 3, 3), np.nan)):
            with pytest.raises(lib.CellError) as e:
                c.solve_hyper(bad)
            assert e.value.status == lib.CELL_E_ARG
        # a Newton iteration cap that is too small reports CELL_NOT_CONVERGED
        # with the iterate reached, and the linear results stay unavailable
        E = np.where(np.arange(512) % 3 == 0, 10.0, 1.0)
        c.set_material(E, np.full(512, 0.3))
        P, info = c.solve_hyper(np.diag([1.2, 1.0, 1.0])[None], tol=1e-12, max_newton=1)
        assert info["status"] == "CELL_NOT_CONVERGED" and info["newton_iters"][0] == 1
        assert np.all(np.isfinite(P))
