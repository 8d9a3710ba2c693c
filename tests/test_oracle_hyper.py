"""Pins of the neo-Hookean oracle (CPU): derivatives by central differences,
the homogeneous solution, the small-strain limit against the linear oracle,
the exact laminate solution (an independent nonlinear system per layer),
and frame indifference."""
import numpy as np
import pytest

from oracle import fem, hyper
from closed_forms import laminate_neohooke

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def rand_case(shape, seed, amp=0.15):
    rng = np.random.default_rng(seed)
    nshape = tuple(reversed(shape))
    E = rng.uniform(1.0, 5.0, nshape)
    nu = rng.uniform(0.1, 0.4, nshape)
    d = len(shape)
    Fbar = np.eye(d) + amp * rng.standard_normal((d, d))
    u = 0.02 * rng.standard_normal((d, int(np.prod(shape))))
    return E, nu, Fbar, u


@pytest.mark.parametrize("shape", [(3, 3, 2), (4, 3)])
def test_residual_is_minus_energy_gradient(shape):
    grid = fem.Grid(shape, lengths=[1.0 + 0.1 * a for a in range(len(shape))])
    E, nu, Fbar, u = rand_case(shape, 1)
    f = hyper.residual(grid, E, nu, u, Fbar).ravel()
    rng = np.random.default_rng(2)
    h = 1e-6
    for k in rng.choice(u.size, 12, replace=False):
        e = np.zeros(u.size)
        e[k] = h
        fd = (hyper.total_energy(grid, E, nu, u.ravel() + e, Fbar) -
              hyper.total_energy(grid, E, nu, u.ravel() - e, Fbar)) / (2 * h)
        assert abs(fd + f[k]) <= 1e-6 * (abs(f[k]) + np.abs(f).max() * 1e-3), k


@pytest.mark.parametrize("shape", [(3, 3, 2), (4, 3)])
def test_tangent_is_residual_derivative(shape):
    grid = fem.Grid(shape)
    E, nu, Fbar, u = rand_case(shape, 3)
    K = hyper.assemble_tangent(grid, E, nu, u, Fbar)
    assert abs(K - K.T).max() <= 1e-12 * abs(K).max()
    rng = np.random.default_rng(4)
    du = rng.standard_normal(u.size)
    h = 1e-6
    fd = -(hyper.residual(grid, E, nu, u.ravel() + h * du, Fbar) -
           hyper.residual(grid, E, nu, u.ravel() - h * du, Fbar)).ravel() / (2 * h)
    Kd = K @ du
    assert np.abs(fd - Kd).max() <= 1e-6 * np.abs(Kd).max()


@pytest.mark.parametrize("shape", [(4, 3, 5), (5, 4)])
def test_sampled_residual_equals_full(shape):
    """The per-node gather used for spot checks of large fields equals the
    full scatter evaluation at every node."""
    grid = fem.Grid(shape, lengths=[1.0 + 0.1 * a for a in range(len(shape))])
    E, nu, Fbar, u = rand_case(shape, 11)
    f = hyper.residual(grid, E, nu, u, Fbar)
    fs = hyper.residual_at_nodes(grid, E, nu, u, Fbar, np.arange(grid.n))
    assert np.abs(fs.T - f).max() < 1e-14 * np.abs(f).max()


def test_material_law_closed_forms():
    """P and A at F = I reduce to the linear law; P by differences of W."""
    lam, mu = np.array([1.3]), np.array([0.7])
    A = hyper.tangent(np.eye(3)[None], lam, mu)[0]
    I = np.eye(3)
    A_lin = (lam[0] * np.einsum("ab,ce->abce", I, I) + mu[0] * (np.einsum("ac,be->abce", I, I) +
                                                              np.einsum("ae,bc->abce", I, I)))
    assert np.abs(A - A_lin).max() < 1e-14
    assert np.abs(hyper.piola(np.eye(3)[None], lam, mu)).max() < 1e-15
    rng = np.random.default_rng(5)
    F = np.eye(3) + 0.3 * rng.standard_normal((3, 3))
    P = hyper.piola(F[None], lam, mu)[0]
    h = 1e-6
    for a in range(3):
        for b in range(3):
            dF = np.zeros((3, 3))
            dF[a, b] = h
            fd = (hyper.energy_density((F + dF)[None], lam, mu) - hyper.energy_density((F - dF)[None], lam, mu)) / (2 * h)
            assert abs(fd[0] - P[a, b]) < 1e-7


def test_energy_density_closed_values():
    """W itself at deformations with a closed value (Sec. 2.2, eq.
    NeoHookeanEnergy): zero at F = I; pure dilation F = s I with J = s^d,
    W = lam/2 (d ln s)^2 - mu d ln s + mu/2 d (s^2 - 1); simple shear
    F = I + g e_1 (x) e_2 with J = 1, W = mu g^2 / 2 (only the trace term);
    uniaxial stretch F = diag(s, 1, ..) with J = s, W = lam/2 ln^2 s - mu ln s
    + mu/2 (s^2 - 1); no admissible value for det F <= 0.  Dropping or
    changing any of the three terms, or the tr I constant, fails one of them."""
    lam, mu = np.array([1.7]), np.array([0.6])
    for d in (2, 3):
        I = np.eye(d)[None]
        assert hyper.energy_density(I, lam, mu)[0] == 0.0
        for s in (0.8, 1.25, 2.0):
            W = hyper.energy_density(s * I, lam, mu)[0]
            Wc = 0.5 * lam[0] * (d * np.log(s)) ** 2 - mu[0] * d * np.log(s) + 0.5 * mu[0] * d * (s * s - 1.0)
            assert abs(W - Wc) < 1e-14 * max(1.0, abs(Wc))
            F = np.eye(d)
            F[0, 0] = s
            W = hyper.energy_density(F[None], lam, mu)[0]
            Wc = 0.5 * lam[0] * np.log(s) ** 2 - mu[0] * np.log(s) + 0.5 * mu[0] * (s * s - 1.0)
            assert abs(W - Wc) < 1e-14 * max(1.0, abs(Wc))
        for g in (0.1, -0.7):
            F = np.eye(d)
            F[0, 1] = g
            assert abs(hyper.energy_density(F[None], lam, mu)[0] - 0.5 * mu[0] * g * g) < 1e-15
        F = np.eye(d)
        F[0, 0] = -1.0
        assert np.isnan(hyper.energy_density(F[None], lam, mu)[0])


@pytest.mark.parametrize("shape", [(4, 4, 4), (6, 6)])
def test_homogeneous_cell(shape):
    grid = fem.Grid(shape)
    nshape = tuple(reversed(shape))
    E = np.full(nshape, 2.0)
    nu = np.full(nshape, 0.3)
    d = len(shape)
    Fbar = np.eye(d) + 0.2 * np.random.default_rng(6).standard_normal((d, d))
    out = hyper.newton(grid, E, nu, Fbar)
    lam, mu = fem.lame(2.0, 0.3)
    assert out["iterations"] == 0
    P = hyper.piola(Fbar[None], np.array([lam]), np.array([mu]))[0]
    assert np.abs(out["P_mean"] - P).max() < 1e-12 * np.abs(P).max()
    W = hyper.energy_density(Fbar[None], np.array([lam]), np.array([mu]))[0]
    assert abs(out["energy"] - W) < 1e-12 * abs(W)


@pytest.mark.parametrize("shape", [(4, 4, 4), (6, 6)])
def test_small_strain_limit_is_linear_cstar(shape):
    """F_bar = I + eps H: P_mean / eps -> C* sym(H) of the linear oracle."""
    grid = fem.Grid(shape)
    d = len(shape)
    E, nu, _, _ = rand_case(shape, 7)
    Clin, _, _ = fem.effective_stiffness(grid, E, nu)
    pairs = fem.voigt_pairs(d)
    rng = np.random.default_rng(8)
    H = rng.standard_normal((d, d))
    Hs = 0.5 * (H + H.T)
    ev = np.array([Hs[a, b] if a == b else 2 * Hs[a, b] for a, b in pairs])
    sig = Clin @ ev
    S = np.zeros((d, d))
    for v, (a, b) in zip(sig, pairs):
        S[a, b] = S[b, a] = v
    eps = 1e-5
    out = hyper.newton(grid, E, nu, np.eye(d) + eps * H, tol=1e-13)
    err = np.abs(out["P_mean"] / eps - S).max() / np.abs(S).max()
    assert err < 50 * eps, err


@pytest.mark.parametrize("shape", [(6, 2, 2), (8, 3)])
def test_laminate_exact_solution(shape):
    d = len(shape)
    nx = shape[0]
    thick = [nx // 3, nx - nx // 3]
    Eph, nuph = [1.0, 8.0], [0.2, 0.35]
    Ex = np.concatenate([np.full(t, e) for t, e in zip(thick, Eph)])
    nux = np.concatenate([np.full(t, v) for t, v in zip(thick, nuph)])
    nshape = tuple(reversed(shape))
    E = np.broadcast_to(Ex, nshape).copy()
    nu = np.broadcast_to(nux, nshape).copy()
    grid = fem.Grid(shape)
    Fbar = np.eye(d)
    Fbar[0, 0] = 1.25
    Fbar[1, 0] = 0.2
    Fbar[0, 1] = -0.1
    out = hyper.newton(grid, E, nu, Fbar, tol=1e-14)
    phases = [tuple(float(x) for x in fem.lame(e, v)) for e, v in zip(Eph, nuph)]
    P, W = laminate_neohooke(phases, [t / nx for t in thick], Fbar)
    assert np.abs(out["P_mean"] - P).max() < 1e-10 * np.abs(P).max()
    assert abs(out["energy"] - W) < 1e-10 * abs(W)
    assert out["iterations"] >= 2


def test_frame_indifference():
    shape = (4, 3, 3)
    grid = fem.Grid(shape)
    E, nu, Fbar, _ = rand_case(shape, 9, amp=0.1)
    c, s = np.cos(0.5), np.sin(0.5)
    R = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]])
    a = hyper.newton(grid, E, nu, Fbar)
    b = hyper.newton(grid, E, nu, R @ Fbar)
    assert abs(a["energy"] - b["energy"]) < 1e-10 * abs(a["energy"])
    assert np.abs(R @ a["P_mean"] - b["P_mean"]).max() < 1e-9 * np.abs(a["P_mean"]).max()
