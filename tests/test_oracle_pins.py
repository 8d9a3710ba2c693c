"""Pins of the CPU oracle against facts fixed by mathematics, not by itself.

Each test would fail for a plausible mistake in the oracle (dropped term,
wrong sign or index, transposed operand, wrong shear convention):

  * brute force: the stiffness and load vector recovered from a separate
    energy evaluation (tensor strains from a least-squares plane fit on each
    simplex, W = lambda/2 tr(eps)^2 + mu eps:eps of Sec. 2.2) on tiny grids;
  * homogeneous material: zero load, zero fluctuation, C* = D exactly;
  * laminates: exact Backus averages (the continuum solution lies in the
    P1 space), normal along every axis, 2D and 3D;
  * Voigt/Reuss bounds, symmetry, Hill-Mandel energy equality;
  * invariances: periodic roll, axis permutation, central inversion,
    modulus scaling;
  * operator structure: symmetry, translation kernel (Sec. 3.4 zero row
    sums, vector form), rank, element rigid-body modes (Sec. 3.4 remark);
  * Fourier preconditioner = exact inverse of the assembled homogeneous K;
  * derivative of C* w.r.t. E: central finite differences, Euler identity
    for the 1-homogeneous map E -> C*, sign.
"""
import itertools

import numpy as np
import pytest

from oracle import fem, matfree
from paper_2004_05197_amd import microstructures as ms
from closed_forms import backus


def rand_material(grid, seed, Emin=1.0, Emax=10.0):
    rng = np.random.default_rng(seed)
    E = rng.uniform(Emin, Emax, grid.nshape)
    nu = rng.uniform(0.05, 0.45, grid.nshape)
    return E, nu


# --------------------------------------------------------------------------
# brute force through an independent energy evaluation
# --------------------------------------------------------------------------

def energy_bruteforce(grid, E, nu, u, eps_bar_tensor):
    """Total energy sum_s |s| W(eps_bar + sym grad u_h) evaluated directly.

    The gradient of the P1 interpolant on each simplex is obtained by a
    least-squares affine fit through the vertex values (exact for affine
    data); W uses tensor strains, no Voigt notation.
    """
    d = grid.d
    lam, mu = fem.lame(np.ravel(E), np.ravel(nu))
    mi = grid.multi_index()
    u = u.reshape(d, grid.n)
    total = 0.0
    h = np.asarray(grid.h)
    for V in fem.kuhn_simplices(d):
        X = V * h[None, :]
        A = np.hstack([np.ones((d + 1, 1)), X])
        vol = abs(np.linalg.det(A)) / np.prod(np.arange(1, d + 1))
        nodes = [grid.flat([mi[a] + V[j, a] for a in range(d)]) for j in range(d + 1)]
        for v in range(grid.n):
            vals = np.array([[u[c, nodes[j][v]] for c in range(d)] for j in range(d + 1)])
            coef, *_ = np.linalg.lstsq(A, vals, rcond=None)
            G = coef[1:, :].T  # G[c, a] = d u_c / d x_a
            eps = eps_bar_tensor + 0.5 * (G + G.T)
            W = 0.5 * lam[v] * np.trace(eps) ** 2 + mu[v] * np.sum(eps * eps)
            total += vol * W
    return total


def voigt_to_tensor(e, d):
    T = np.zeros((d, d))
    for k, (a, b) in enumerate(fem.voigt_pairs(d)):
        if a == b:
            T[a, a] = e[k]
        else:
            T[a, b] = T[b, a] = 0.5 * e[k]
    return T


@pytest.mark.parametrize("shape", [(3, 2), (2, 3, 2)])
def test_bruteforce_stiffness_and_load(shape):
    grid = fem.Grid(shape, lengths=[1.0 + 0.3 * k for k in range(len(shape))])
    E, nu = rand_material(grid, 11)
    K = fem.assemble_K(grid, E, nu).toarray()
    N = grid.d * grid.n
    zero = np.zeros((grid.d, grid.d))
    Pi = lambda u, eb=zero: energy_bruteforce(grid, E, nu, u, eb)
    diag = np.array([Pi(np.eye(N)[i]) for i in range(N)])
    Kb = np.zeros((N, N))
    for i in range(N):
        for j in range(i, N):
            if i == j:
                Kb[i, i] = 2.0 * diag[i]
            else:
                Kb[i, j] = Kb[j, i] = Pi(np.eye(N)[i] + np.eye(N)[j]) - diag[i] - diag[j]
    assert np.allclose(K, Kb, rtol=0, atol=1e-10 * np.abs(K).max())
    # load vector: Pi(eb, u) = 1/2 u^T K u - f^T u + Pi(eb, 0)
    rng = np.random.default_rng(3)
    e = rng.standard_normal(grid.nv)
    ebt = voigt_to_tensor(e, grid.d)
    f = fem.assemble_rhs(grid, E, nu, e[None, :])[0]
    P0 = Pi(np.zeros(N), ebt)
    fb = np.array([-(Pi(np.eye(N)[i], ebt) - P0 - 0.5 * Kb[i, i]) for i in range(N)])
    assert np.allclose(f, fb, rtol=0, atol=1e-10 * np.abs(f).max())
    # homogenized energy density with u = 0 is the voxel average of W(eps_bar)
    C = fem.homogenize(grid, E, nu, np.zeros((1, N)), e[None, :])["C_energy"][0, 0]
    assert np.isclose(0.5 * C, P0 / grid.volume, rtol=1e-12)


# --------------------------------------------------------------------------
# homogeneous material
# --------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(5, 4), (4, 5, 6)])
def test_homogeneous_exact(shape):
    grid = fem.Grid(shape)
    E = np.full(grid.nshape, 7.0)
    nu = np.full(grid.nshape, 0.27)
    f = fem.assemble_rhs(grid, E, nu, fem.unit_loads(grid.d))
    assert np.abs(f).max() < 1e-13
    C, Cs, u = fem.effective_stiffness(grid, E, nu)
    lam, mu = fem.lame(7.0, 0.27)
    D = fem.D_voigt(lam, mu, grid.d)
    assert np.abs(C - D).max() < 1e-12 * np.abs(D).max()
    assert np.abs(Cs - D).max() < 1e-12 * np.abs(D).max()
    assert np.abs(u).max() < 1e-12


# --------------------------------------------------------------------------
# laminates (Backus averaging is exact for P1 here)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("d,shape", [(2, (6, 5)), (3, (4, 5, 6))])
def test_laminates_exact(d, shape):
    rng = np.random.default_rng(5)
    for normal in range(d):
        N = shape[normal]
        nph = 2 + normal % 3
        cuts = np.sort(rng.choice(np.arange(1, N), nph - 1, replace=False))
        th = np.diff(np.concatenate([[0], cuts, [N]]))
        Es = rng.uniform(1, 50, nph)
        nus = rng.uniform(0.1, 0.45, nph)
        E, nu = ms.laminate(shape, normal, Es, nus, th)
        grid = fem.Grid(shape)
        C, Cs, _ = fem.effective_stiffness(grid, E, nu)
        lam, mu = fem.lame(Es, nus)
        Cb = backus(lam, mu, th / N, d, normal)
        assert np.abs(C - Cb).max() < 1e-11 * np.abs(Cb).max(), (normal, C, Cb)
        assert np.abs(Cs - Cb).max() < 1e-11 * np.abs(Cb).max()


# --------------------------------------------------------------------------
# bounds, symmetry, Hill-Mandel
# --------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(6, 7), (4, 4, 5)])
def test_bounds_symmetry_hill_mandel(shape):
    grid = fem.Grid(shape)
    E, nu = rand_material(grid, 21, 1.0, 100.0)
    K = fem.assemble_K(grid, E, nu)
    C, Cs, u = fem.effective_stiffness(grid, E, nu, K=K)
    lam, mu = fem.lame(np.ravel(E), np.ravel(nu))
    Ds = [fem.D_voigt(l, m, grid.d) for l, m in zip(lam, mu)]
    voigt = np.mean(Ds, axis=0)
    reuss = np.linalg.inv(np.mean([np.linalg.inv(D) for D in Ds], axis=0))
    tol = 1e-10 * np.abs(C).max()
    assert np.linalg.eigvalsh(voigt - C).min() >= -tol
    assert np.linalg.eigvalsh(C - reuss).min() >= -tol
    assert np.abs(Cs - Cs.T).max() < 1e-10 * np.abs(C).max()
    assert np.abs(C - Cs).max() < 1e-10 * np.abs(C).max()
    gap = fem.hill_mandel_gap(grid, E, nu, u, fem.unit_loads(grid.d), K=K)
    assert np.abs(gap).max() < 1e-12 * np.abs(C).max()
    # C* is SPD
    assert np.linalg.eigvalsh(C).min() > 0


# --------------------------------------------------------------------------
# invariances
# --------------------------------------------------------------------------

def voigt_perm(perm, d):
    """Voigt index map for the axis relabeling a -> perm[a]."""
    pairs = fem.voigt_pairs(d)
    idx = {}
    for k, (a, b) in enumerate(pairs):
        idx[(a, b)] = k
        idx[(b, a)] = k
    return np.array([idx[(perm[a], perm[b])] for (a, b) in pairs])


@pytest.mark.parametrize("shape", [(5, 5), (4, 4, 4)])
def test_invariances(shape):
    grid = fem.Grid(shape)
    d = grid.d
    E, nu = rand_material(grid, 31)
    C0, _, u0 = fem.effective_stiffness(grid, E, nu)
    tol = 1e-11 * np.abs(C0).max()
    # (i) periodic roll
    Er = np.roll(E, (1, 2) if d == 2 else (1, 2, 3), axis=tuple(range(d)))
    nur = np.roll(nu, (1, 2) if d == 2 else (1, 2, 3), axis=tuple(range(d)))
    assert np.abs(fem.effective_stiffness(grid, Er, nur)[0] - C0).max() < tol
    # (ii) axis permutations: material axes relabeled -> C* indices relabeled
    for perm in itertools.permutations(range(d)):
        # new field F(x) = old(x') with x'_{perm[a]} = x_a; numpy axes are reversed
        np_axes = [d - 1 - perm[d - 1 - k] for k in range(d)]
        Ep = np.transpose(E, np_axes)
        nup = np.transpose(nu, np_axes)
        Cp = fem.effective_stiffness(fem.Grid(tuple(shape[perm[a]] for a in range(d))), Ep, nup)[0]
        P = voigt_perm(perm, d)
        assert np.abs(Cp - C0[np.ix_(P, P)]).max() < tol, perm
    # (iii) central inversion (all axes reversed at once)
    Ei = E[(slice(None, None, -1),) * d]
    nui = nu[(slice(None, None, -1),) * d]
    assert np.abs(fem.effective_stiffness(grid, Ei, nui)[0] - C0).max() < tol
    # (iv) scaling E -> sE scales C*, leaves u unchanged
    C2, _, u2 = fem.effective_stiffness(grid, 3.5 * E, nu)
    assert np.abs(C2 - 3.5 * C0).max() < 3.5 * tol
    assert np.abs(u2 - u0).max() < 1e-10 * np.abs(u0).max()


def test_single_axis_reflection_is_not_an_invariance():
    # the Kuhn split has a preferred diagonal: mirroring one axis changes
    # the discrete C* (this guards against a symmetric-by-accident oracle)
    grid = fem.Grid((5, 5))
    E, nu = rand_material(grid, 41, 1.0, 100.0)
    C0 = fem.effective_stiffness(grid, E, nu)[0]
    Cm = fem.effective_stiffness(grid, E[:, ::-1], nu[:, ::-1])[0]
    # mirror x: the shear coupling entries flip sign, the rest stays close
    assert np.abs(Cm - C0).max() > 1e-6 * np.abs(C0).max()


# --------------------------------------------------------------------------
# operator structure
# --------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(4, 5), (3, 4, 3)])
def test_operator_structure(shape):
    grid = fem.Grid(shape)
    E, nu = rand_material(grid, 51)
    K = fem.assemble_K(grid, E, nu).toarray()
    assert np.abs(K - K.T).max() < 1e-13 * np.abs(K).max()
    for c in range(grid.d):
        t = np.zeros(grid.d * grid.n)
        t[c * grid.n:(c + 1) * grid.n] = 1.0
        assert np.abs(K @ t).max() < 1e-12 * np.abs(K).max()
    ev = np.linalg.eigvalsh(K)
    assert np.sum(ev < 1e-10 * ev.max()) == grid.d  # rank = d n - d
    assert ev.min() > -1e-12 * ev.max()             # PSD
    # element matrices: kernel = rigid-body modes (3 in 2D, 6 in 3D)
    m = fem.voigt_m(grid.d)
    S = np.diag(fem.voigt_s(grid.d))
    nc = 2 ** grid.d
    Ke = np.zeros((grid.d * nc, grid.d * nc))
    for V, vol, B in fem.element_data(grid):
        corner = [int(sum(V[j, a] << a for a in range(grid.d))) for j in range(grid.d + 1)]
        P = np.zeros((grid.d * (grid.d + 1), grid.d * nc))
        for c in range(grid.d):
            for j in range(grid.d + 1):
                P[c * (grid.d + 1) + j, c * nc + corner[j]] = 1.0
        Bc = B @ P
        Ke += vol * Bc.T @ (1.3 * np.outer(m, m) + 0.7 * S) @ Bc
    eve = np.linalg.eigvalsh(Ke)
    assert np.sum(eve < 1e-10 * eve.max()) == (3 if grid.d == 2 else 6)


# --------------------------------------------------------------------------
# Fourier reference preconditioner
# --------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(6, 4), (4, 6, 5)])
def test_fourier_preconditioner_is_exact_inverse(shape):
    grid = fem.Grid(shape, lengths=[1.0 + 0.2 * a for a in range(len(shape))])
    lam0, mu0 = 2.3, 0.9
    Kref = fem.assemble_K(grid, *_lame_inverse(lam0, mu0, grid.nshape)).toarray()
    P = matfree.FourierPreconditioner(grid, lam0, mu0)
    rng = np.random.default_rng(61)
    r = rng.standard_normal((grid.d,) + grid.nshape)
    r -= r.reshape(grid.d, -1).mean(axis=1).reshape((grid.d,) + (1,) * grid.d)
    z = P(r)
    assert np.abs(z.reshape(grid.d, -1).mean(axis=1)).max() < 1e-13
    assert np.abs(Kref @ z.ravel() - r.ravel()).max() < 1e-10 * np.abs(r).max()


def _lame_inverse(lam, mu, nshape):
    """(E, nu) arrays reproducing the given Lame pair."""
    nu = lam / (2 * (lam + mu))
    E = mu * 2 * (1 + nu)
    return np.full(nshape, E), np.full(nshape, nu)


@pytest.mark.parametrize("shape", [(8, 6), (6, 4, 8)])
def test_pcg_matches_direct(shape):
    grid = fem.Grid(shape)
    E, nu = rand_material(grid, 71, 1.0, 100.0)
    eb = fem.unit_loads(grid.d)
    ud = fem.solve_direct(grid, E, nu, eb)
    for J in range(eb.shape[0]):
        x, it, rr = matfree.pcg(grid, E, nu, eb[J], tol=1e-13)
        assert rr <= 1e-13
        assert np.abs(x.ravel() - ud[J]).max() < 1e-10 * np.abs(ud[J]).max()
    h1 = fem.homogenize(grid, E, nu, ud, eb)
    h2 = matfree.homogenize(grid, E, nu, ud.reshape((eb.shape[0], grid.d) + grid.nshape), eb)
    assert np.abs(h1["C_energy"] - h2["C_energy"]).max() < 1e-13 * np.abs(h1["C_energy"]).max()


# --------------------------------------------------------------------------
# derivative with respect to E
# --------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(4, 5), (3, 4, 3)])
def test_gradient_fd_euler_sign(shape):
    grid = fem.Grid(shape)
    E, nu = rand_material(grid, 81, 1.0, 5.0)
    eb = fem.unit_loads(grid.d)
    C, _, u = fem.effective_stiffness(grid, E, nu)
    G = fem.dC_dE(grid, E, nu, u, eb)  # (nv, nv, n)
    # Euler: C* is 1-homogeneous in E at fixed nu
    assert np.abs(np.einsum("ijv,v->ij", G, np.ravel(E)) - C).max() < 1e-12 * np.abs(C).max()
    # diagonal entries are non-decreasing in every E_v
    for I in range(grid.nv):
        assert G[I, I].min() >= -1e-14
    # central differences on a few voxels
    rng = np.random.default_rng(82)
    step = 1e-5
    for v in rng.choice(grid.n, 4, replace=False):
        Ep = np.ravel(E).copy()
        Em = np.ravel(E).copy()
        Ep[v] += step
        Em[v] -= step
        Cp = fem.effective_stiffness(grid, Ep.reshape(grid.nshape), nu)[0]
        Cm = fem.effective_stiffness(grid, Em.reshape(grid.nshape), nu)[0]
        fd = (Cp - Cm) / (2 * step)
        assert np.abs(fd - G[:, :, v]).max() < 1e-7 * np.abs(G[:, :, v]).max() + 1e-12


# --------------------------------------------------------------------------
# generators
# --------------------------------------------------------------------------

def test_generators():
    E, nu = ms.circle2d(32)
    assert int((E == 10.0).sum()) == 208
    mask, avf, sph = ms.rsa_spheres(32, 0.2, seed=7)
    assert avf >= 0.2
    for i in range(len(sph)):
        for j in range(i):
            dv = sph[i][0] - sph[j][0]
            dv -= 32 * np.round(dv / 32)
            assert np.linalg.norm(dv) >= sph[i][1] + sph[j][1] - 1e-12
    g = ms.gaussian_random_field((16, 16, 16), 3.0, seed=3)
    assert abs(g.mean()) < 1e-12 and abs(g.std() - 1) < 1e-12
    g2 = ms.gaussian_random_field((16, 16, 16), 3.0, seed=3)
    assert np.array_equal(g, g2)


@pytest.mark.parametrize("shape", [(5, 4), (4, 3, 5)])
def test_residual_at_nodes_matches_assembled(shape):
    grid = fem.Grid(shape, lengths=[1.0 + 0.1 * a for a in range(len(shape))])
    E, nu = rand_material(grid, 91)
    rng = np.random.default_rng(92)
    u = rng.standard_normal(grid.d * grid.n)
    e = rng.standard_normal(grid.nv)
    K = fem.assemble_K(grid, E, nu)
    r = fem.assemble_rhs(grid, E, nu, e[None, :])[0] - K @ u
    nodes = rng.choice(grid.n, 7, replace=False)
    rl = fem.residual_at_nodes(grid, E, nu, u, e, nodes)
    ref = np.stack([r[c * grid.n + nodes] for c in range(grid.d)], axis=1)
    assert np.abs(rl - ref).max() < 1e-12 * np.abs(r).max()
