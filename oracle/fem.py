"""Explicit P1 finite-element assembly and direct solve (CPU, FP64).

Test infrastructure only (see the package docstring).

Problem (static, periodic special case of the elastic system of Sec. 2.1,
eq. TimeHarmonicSystem with k = 0): find the periodic displacement
fluctuation u~ minimizing

    Pi(u~) = sum_{voxels v} sum_{simplices s in v} |s| * W(eps_bar + eps(u~))

with the linear-elastic energy W(eps) = lambda/2 tr(eps)^2 + mu eps:eps of
Sec. 2.2 (eq. LinearElastEnergy), Lame parameters from (E, nu) as in
Sec. 6.3, and P1 (linear) displacement on every simplex of the Kuhn
subdivision.  Nodes sit at voxel corners and wrap periodically; node and
voxel multi-indices are flattened colexicographically (x fastest), as in
Sec. 3.1.

Voigt order is (11, 22, 33, 23, 13, 12) in 3D and (11, 22, 12) in 2D, with
engineering shear strains.  2D is plane strain.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

# --------------------------------------------------------------------------
# material law
# --------------------------------------------------------------------------


def lame(E, nu):
    """Lame parameters from Young's modulus and Poisson ratio (Sec. 6.3)."""
    E = np.asarray(E, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    lam = nu * E / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def voigt_pairs(d):
    """Tensor index pairs of the Voigt components."""
    if d == 2:
        return [(0, 0), (1, 1), (0, 1)]
    return [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]


def voigt_m(d):
    """Voigt vector of the identity tensor (trace extractor)."""
    return np.array([1.0 if a == b else 0.0 for (a, b) in voigt_pairs(d)])


def voigt_s(d):
    """Diagonal of the Voigt matrix of eps:eps*2 with engineering shear.

    W = lambda/2 (m.e)^2 + mu * sum_normal e_i^2 + mu/2 * sum_shear g_i^2,
    so W = 1/2 e^T D e with D = lambda m m^T + mu diag(s),
    s = 2 on normal and 1 on shear components.
    """
    return np.array([2.0 if a == b else 1.0 for (a, b) in voigt_pairs(d)])


def D_voigt(lam, mu, d):
    """Voigt stiffness D = lambda m m^T + mu diag(s) for one voxel."""
    m = voigt_m(d)
    return lam * np.outer(m, m) + mu * np.diag(voigt_s(d))


# --------------------------------------------------------------------------
# grid and simplices
# --------------------------------------------------------------------------


class Grid:
    """Periodic node/voxel grid on the box prod [0, L_a)."""

    def __init__(self, shape_xyz, lengths=None):
        self.shape = tuple(int(s) for s in shape_xyz)
        self.d = len(self.shape)
        if self.d not in (2, 3):
            raise ValueError("2D or 3D grids only")
        if min(self.shape) < 2:
            raise ValueError("every grid size must be >= 2")
        self.L = tuple(float(x) for x in (lengths or (1.0,) * self.d))
        self.h = tuple(L / N for L, N in zip(self.L, self.shape))
        self.n = int(np.prod(self.shape))
        self.volume = float(np.prod(self.L))
        self.nv = 3 if self.d == 2 else 6
        self.nshape = tuple(reversed(self.shape))

    def multi_index(self):
        """Per-voxel (i_x, i_y[, i_z]) for flat colexicographic indices."""
        idx = np.arange(self.n)
        out = []
        for N in self.shape:
            out.append(idx % N)
            idx = idx // N
        return out

    def flat(self, comps):
        """Colexicographic flat index of (possibly out-of-range) indices."""
        f = np.zeros_like(comps[0])
        stride = 1
        for c, N in zip(comps, self.shape):
            f = f + (c % N) * stride
            stride *= N
        return f


def kuhn_simplices(d):
    """Kuhn (Freudenthal) subdivision of the unit cube.

    One simplex per permutation p of the axes: v_0 = 0, v_j = v_{j-1} + e_{p_j}.
    All d! simplices share the main diagonal from 0 to (1,...,1).
    Returns a list of (d+1, d) integer vertex arrays.
    """
    out = []
    for perm in itertools.permutations(range(d)):
        v = [np.zeros(d, dtype=np.int64)]
        for a in perm:
            w = v[-1].copy()
            w[a] += 1
            v.append(w)
        out.append(np.array(v))
    return out


def p1_gradients(X):
    """Gradients of the barycentric (P1 hat) functions of a simplex.

    X: (d+1, d) vertex coordinates.  phi_k(x) = c_k + g_k . x with
    phi_k(x_j) = delta_kj, i.e. [1 X] [c; g]_k = e_k.  Returns (g, volume).
    """
    d = X.shape[1]
    A = np.hstack([np.ones((d + 1, 1)), X])
    C = np.linalg.inv(A)
    grads = C[1:, :].T  # (d+1, d): row k = grad phi_k
    vol = abs(np.linalg.det(A)) / math.factorial(d)
    return grads, vol


def simplex_B(grads, d):
    """Voigt strain operator of one simplex: (nv, d*(d+1)).

    Column index = comp * (d+1) + vertex.  Normal rows give u_a,a; shear
    rows give u_a,b + u_b,a (engineering shear).
    """
    pairs = voigt_pairs(d)
    nvert = d + 1
    B = np.zeros((len(pairs), d * nvert))
    for row, (a, b) in enumerate(pairs):
        for j in range(nvert):
            if a == b:
                B[row, a * nvert + j] += grads[j, a]
            else:
                B[row, a * nvert + j] += grads[j, b]
                B[row, b * nvert + j] += grads[j, a]
    return B


def element_data(grid):
    """Per simplex: vertex corner offsets, volume and strain operator B."""
    out = []
    for V in kuhn_simplices(grid.d):
        X = V * np.asarray(grid.h)[None, :]
        grads, vol = p1_gradients(X)
        out.append((V, vol, simplex_B(grads, grid.d)))
    return out


def simplex_dofs(grid, V):
    """Global dof indices (n, d*(d+1)) of the vertices of one simplex type.

    Global dof = comp * n + node (component-major), node colexicographic.
    """
    mi = grid.multi_index()
    nodes = [grid.flat([mi[a] + V[j, a] for a in range(grid.d)])
             for j in range(V.shape[0])]
    cols = []
    for c in range(grid.d):
        for j in range(V.shape[0]):
            cols.append(c * grid.n + nodes[j])
    return np.stack(cols, axis=1)


# --------------------------------------------------------------------------
# assembly
# --------------------------------------------------------------------------


def assemble_K(grid, E, nu):
    """Sparse periodic stiffness K = sum_v sum_s |s| B_s^T D_v B_s (CSR)."""
    lam, mu = lame(np.ravel(E), np.ravel(nu))
    m = voigt_m(grid.d)
    S = np.diag(voigt_s(grid.d))
    rows, cols, vals = [], [], []
    for V, vol, B in element_data(grid):
        Kl = vol * (B.T @ np.outer(m, m) @ B)
        Km = vol * (B.T @ S @ B)
        dofs = simplex_dofs(grid, V)
        k = dofs.shape[1]
        rows.append(np.repeat(dofs, k, axis=1).ravel())
        cols.append(np.tile(dofs, (1, k)).ravel())
        vals.append((lam[:, None, None] * Kl[None] + mu[:, None, None] * Km[None]).ravel())
    N = grid.d * grid.n
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N)).tocsr()
    K.sum_duplicates()
    return K


def assemble_rhs(grid, E, nu, eps_bar):
    """Load vectors f^J = -sum_v sum_s |s| B_s^T D_v eps_bar^J.

    eps_bar: (nload, nv) Voigt macro strains.  Returns (nload, d*n).
    """
    eps_bar = np.atleast_2d(np.asarray(eps_bar, dtype=np.float64))
    lam, mu = lame(np.ravel(E), np.ravel(nu))
    m = voigt_m(grid.d)
    s = voigt_s(grid.d)
    N = grid.d * grid.n
    f = np.zeros((eps_bar.shape[0], N))
    for V, vol, B in element_data(grid):
        dofs = simplex_dofs(grid, V)
        for J, e in enumerate(eps_bar):
            sig = lam[:, None] * (m @ e) * m[None, :] + mu[:, None] * (s * e)[None, :]
            contrib = -vol * sig @ B  # (n, d*(d+1))
            f[J] += np.bincount(dofs.ravel(), weights=contrib.ravel(), minlength=N)
    return f


def simplex_strains(grid, u, eps_bar):
    """Total strains eps_bar + B_s u on every (voxel, simplex).

    u: (d*n,), eps_bar: (nv,).  Returns list over simplices of (n, nv) and
    the simplex volumes.
    """
    out, vols = [], []
    for V, vol, B in element_data(grid):
        dofs = simplex_dofs(grid, V)
        out.append(eps_bar[None, :] + u[dofs] @ B.T)
        vols.append(vol)
    return out, vols


# --------------------------------------------------------------------------
# solve and homogenized quantities
# --------------------------------------------------------------------------


def unit_loads(d):
    """Unit Voigt macro strains e_J (engineering shear: gamma = 1)."""
    nv = 3 if d == 2 else 6
    return np.eye(nv)


def solve_direct(grid, E, nu, eps_bar, K=None):
    """Direct sparse solve of K u = f for each macro strain.

    K is singular with kernel = the d constant translations (the vector
    analogue of the zero row-sum property, Sec. 3.4 eq. RowSumProperty),
    so node 0 is pinned (its d dofs removed), the reduced SPD system is
    factorized once, and the nodal mean of each component is subtracted.
    Returns u (nload, d*n) mean-zero per component.
    """
    if K is None:
        K = assemble_K(grid, E, nu)
    f = assemble_rhs(grid, E, nu, eps_bar)
    N = grid.d * grid.n
    pinned = np.array([c * grid.n for c in range(grid.d)])
    keep = np.setdiff1d(np.arange(N), pinned)
    Kr = K[keep][:, keep].tocsc()
    lu = spla.splu(Kr)
    u = np.zeros_like(f)
    for J in range(f.shape[0]):
        u[J, keep] = lu.solve(f[J, keep])
        for c in range(grid.d):
            blk = u[J, c * grid.n:(c + 1) * grid.n]
            blk -= blk.mean()
    return u


def homogenize(grid, E, nu, u, eps_bar):
    """Effective quantities from solved fluctuations.

    Returns dict with
      C_energy[I,J] = (1/|Y|) sum |s| (eps^I)^T D (eps^J)   (energy form)
      mean_stress[J] = (1/|Y|) sum |s| D eps^J              (mean-stress form)
    with eps^J = eps_bar^J + B u^J.
    """
    lam, mu = lame(np.ravel(E), np.ravel(nu))
    m = voigt_m(grid.d)
    s = voigt_s(grid.d)
    nl = eps_bar.shape[0]
    strains = []
    vols = None
    for J in range(nl):
        st, vols = simplex_strains(grid, u[J], eps_bar[J])
        strains.append(st)
    C = np.zeros((nl, nl))
    sbar = np.zeros((nl, grid.nv))
    for k, vol in enumerate(vols):
        sig = []
        for J in range(nl):
            e = strains[J][k]
            sig.append(lam[:, None] * (e @ m)[:, None] * m[None, :] + mu[:, None] * e * s[None, :])
        for J in range(nl):
            sbar[J] += vol * sig[J].sum(axis=0)
            for I in range(nl):
                C[I, J] += vol * np.sum(strains[I][k] * sig[J])
    return dict(C_energy=C / grid.volume, mean_stress=sbar / grid.volume)


def effective_stiffness(grid, E, nu, K=None):
    """C* by direct solve for the unit loads; also the mean-stress form."""
    eb = unit_loads(grid.d)
    u = solve_direct(grid, E, nu, eb, K=K)
    h = homogenize(grid, E, nu, u, eb)
    return h["C_energy"], h["mean_stress"].T, u


def hill_mandel_gap(grid, E, nu, u, eps_bar, K=None):
    """<sigma:eps> - sigma_bar:eps_bar, which equals -(u^T r)/|Y| with
    r = f - K u; zero at the exact discrete solution."""
    if K is None:
        K = assemble_K(grid, E, nu)
    f = assemble_rhs(grid, E, nu, eps_bar)
    out = []
    for J in range(f.shape[0]):
        r = f[J] - K @ u[J]
        out.append(-(u[J] @ r) / grid.volume)
    return np.array(out)


def dC_dE(grid, E, nu, u, eps_bar):
    """Derivative of C*_IJ with respect to the Young's modulus of each voxel.

    C*_JJ is the minimum of the total energy, so by the envelope theorem its
    derivative is the partial derivative of the energy at the fixed
    minimizer; the off-diagonal entries follow by polarization.  At fixed nu
    the voxel stiffness is linear in E, so D_v / E_v is the derivative.
    Returns (nload, nload, n):  (1/|Y|) sum_s |s| (eps^I)^T (D_v/E_v) eps^J.
    """
    E = np.ravel(E)
    lam1, mu1 = lame(np.ones_like(E), np.ravel(nu))
    m = voigt_m(grid.d)
    s = voigt_s(grid.d)
    nl = eps_bar.shape[0]
    strains = []
    vols = None
    for J in range(nl):
        st, vols = simplex_strains(grid, u[J], eps_bar[J])
        strains.append(st)
    G = np.zeros((nl, nl, grid.n))
    for k, vol in enumerate(vols):
        for J in range(nl):
            e = strains[J][k]
            sigJ = lam1[:, None] * (e @ m)[:, None] * m[None, :] + mu1[:, None] * e * s[None, :]
            for I in range(nl):
                G[I, J] += vol * np.sum(strains[I][k] * sigJ, axis=1)
    return G / grid.volume


def residual_at_nodes(grid, E, nu, u, eps_bar, nodes):
    """Residual r = f - K u = -sum_v sum_s |s| B_s^T D_v (eps_bar + B_s u) at
    selected nodes only (for spot checks of fields too large to assemble).

    A node is vertex j of simplex s in the voxel at node - V_s[j]; summing the
    vertex-j rows of -|s| B_s^T sigma over all (s, j) collects every element
    term of that node.  u: (d*n,), eps_bar: (nv,), nodes: flat node indices.
    Returns (len(nodes), d).
    """
    d = grid.d
    nodes = np.asarray(nodes, dtype=np.int64)
    lam, mu = lame(np.ravel(E), np.ravel(nu))
    m = voigt_m(d)
    s = voigt_s(d)
    comps = []
    idx = nodes.copy()
    for N in grid.shape:
        comps.append(idx % N)
        idx = idx // N
    out = np.zeros((len(nodes), d))
    eb = np.asarray(eps_bar, dtype=np.float64)
    for V, vol, B in element_data(grid):
        nvert = d + 1
        for j in range(nvert):
            vox = [comps[a] - V[j, a] for a in range(d)]
            vflat = grid.flat(vox)
            ue = np.zeros((len(nodes), d * nvert))
            for k in range(nvert):
                nk = grid.flat([vox[a] + V[k, a] for a in range(d)])
                for c in range(d):
                    ue[:, c * nvert + k] = u[c * grid.n + nk]
            e = eb[None, :] + ue @ B.T
            sig = lam[vflat][:, None] * (e @ m)[:, None] * m[None, :] + mu[vflat][:, None] * e * s[None, :]
            contrib = -vol * sig @ B
            for c in range(d):
                out[:, c] += contrib[:, c * nvert + j]
    return out
