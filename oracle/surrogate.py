"""Surrogate stencil functions for the periodic voxel P1 elasticity matrix
(CPU, FP64).

Test infrastructure only (see the package docstring).

Stencil functions (Sec. 3.2, eqs. DefinitionOfStencilFunction and
StencilRoughDefinition): the block of K coupling node x_i with node
x_i + delta, seen as a function of x_i, K_delta(x_i) = K[i, i + delta]
(d x d, dofs component-major as in ``fem``).  On the Kuhn subdivision two
nodes share a simplex exactly when their index offset is a nonzero 0/1
vector or its negative, so the off-diagonal offsets are +-delta with delta
in the 2^d - 1 nonzero 0/1 vectors (7 in 3D, 3 in 2D).

Surrogate stencil functions (Sec. 3.3, eq. SurrogateRoughDefinition):
K_delta is sampled at every M-th node along each axis and interpolated with
uniform B-splines of degree q whose knots are the sample points.  On the
periodic cell every node is interior; the surrogate matrix follows the
symmetric, kernel-preserving definition of Sec. 3.4 (eq.
DefinitionOfSurrogateMatrixSymmetricKernel):

    Kt[i, i + delta] = Kt_delta(x_i),  Kt[i + delta, i] = Kt_delta(x_i)^T
    (delta in the 7 (3D) / 3 (2D) nonzero 0/1 offsets),
    Kt[i, i] = - sym( sum_{j != i} Kt[i, j] ).

Reading for the vector problem (the paper's Remark on vector-valued problems
leaves it open): the off-diagonal stencil blocks of elasticity are not
symmetric where the material varies, and their interpolants' block row sums
need not be symmetric either, so "minus the row sum" and symmetry cannot
both hold exactly; we keep K symmetric (CG needs it) and take the symmetric
part of the row sum.  The translations (one per component) then stay in the
kernel up to the interpolation error of the blocks' skew parts, and the
surrogate solution is the minimiser of 1/2 u.Kt u - f.u over fluctuations
with zero nodal mean per component (a bordered direct solve here).  Further
readings: q is the B-spline degree, q in {1, 3} (odd, so that interpolation
at the knots is a circulant system); M divides every grid size (periodic
sample lattice); every grid size is at least 3 (i + delta != i - delta).

The load vectors stay exact, and the effective stiffness of a surrogate
solution u~ is the energy form of the exact material law on its strain
field (``fem.homogenize``), which exceeds C* by (u~ - u).K(u~ - u)/|Y|.

For grids too large to assemble, ``stencil_blocks_at``, ``evaluate_at`` and
``apply_at`` compute the same quantities at chosen nodes only: the stencil
blocks from the element matrices of the simplices holding both nodes, the
interpolants from the same coefficients, and rows of Kt p from their
definition above.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem


def offsets(d):
    """The nonzero 0/1 offsets (x fastest), in the order (x, y, z, xy, yz, xz, xyz) / (x, y, xy)."""
    if d == 3:
        return [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (0, 1, 1), (1, 0, 1), (1, 1, 1)]
    return [(1, 0), (0, 1), (1, 1)]


def shifted(grid, delta):
    """Flat index of node i + delta for every node i (periodic)."""
    mi = grid.multi_index()
    return grid.flat([mi[a] + delta[a] for a in range(grid.d)])


def stencil_functions(grid, K):
    """K_delta(x_i) for every offset and node: array (noff, d, d, n), with
    [k, a, b, i] = K[a n + i, b n + (i + delta_k)]."""
    d, n = grid.d, grid.n
    Kc = K.tocsr()
    idx = np.arange(n)
    out = []
    for delta in offsets(d):
        j = shifted(grid, delta)
        blk = np.zeros((d, d, n))
        for a in range(d):
            for b in range(d):
                blk[a, b] = np.asarray(Kc[a * n + idx, b * n + j]).ravel()
        out.append(blk)
    return np.stack(out)


# --------------------------------------------------------------------------
# periodic cardinal B-splines of odd degree
# --------------------------------------------------------------------------


def bspline(q, x):
    """Centred cardinal B-spline of degree q in {1, 3} (support |x| < (q+1)/2)."""
    ax = np.abs(np.asarray(x, dtype=np.float64))
    if q == 1:
        return np.maximum(0.0, 1.0 - ax)
    if q == 3:
        return np.where(ax < 1.0, 2.0 / 3.0 - ax ** 2 + 0.5 * ax ** 3,
                        np.where(ax < 2.0, (2.0 - ax) ** 3 / 6.0, 0.0))
    raise ValueError("degree must be 1 or 3")


def interpolation_coefficients(values, q, d):
    """Coefficients c on a periodic lattice (the last d axes of `values`)
    with sum_j c_j B_q(k - j) = values_k at every lattice point k: the
    circulant system along each axis is diagonal in the DFT (library FFT as
    a step)."""
    c = np.asarray(values, dtype=np.float64)
    nd = c.ndim
    for ax in range(nd - d, nd):
        Nc = c.shape[ax]
        if Nc == 1 or q == 1:
            # q = 1: B_1 is the Kronecker delta on the lattice; a single
            # point: the periodic sum of B_q(k - j) over all shifts is 1
            continue
        ker = np.zeros(Nc)
        for s in range(-2, 3):
            ker[s % Nc] += bspline(q, s)
        sym = np.fft.fft(ker)
        c = np.real(np.fft.ifft(np.fft.fft(c, axis=ax) / np.expand_dims(sym, tuple(i for i in range(nd) if i != ax)),
                                axis=ax))
    return c


def evaluate(coef, q, M, fine_shape):
    """Value at every fine node of the B-spline with coefficients `coef` on
    the lattice of every M-th node; fine_shape and coef's last axes are in
    (z, y, x) array order (x fastest in memory)."""
    d = len(fine_shape)
    lead = coef.shape[:-d]
    # separable: weights along each axis, (fine, coarse) matrices
    mats = []
    for ax in range(d):
        N = fine_shape[ax]
        Nc = coef.shape[len(lead) + ax]
        W = np.zeros((N, Nc))
        for i in range(N):
            t = i / M
            for j in range(int(np.floor(t)) - 2, int(np.floor(t)) + 3):
                W[i, j % Nc] += bspline(q, t - j)
        mats.append(W)
    out = coef
    for ax in range(d):
        out = np.moveaxis(np.tensordot(mats[ax], np.moveaxis(out, len(lead) + ax, 0), axes=(1, 0)), 0, len(lead) + ax)
    return out


# --------------------------------------------------------------------------
# the surrogate matrix and its solution
# --------------------------------------------------------------------------


def surrogate_stencils(grid, E, nu, M, q, K=None):
    """Kt_delta(x_i): the stencil functions sampled at every M-th node and
    interpolated (Sec. 3.3).  Returns (noff, d, d, n)."""
    if any(N % M for N in grid.shape):
        raise ValueError("M must divide every grid size")
    if min(grid.shape) < 3:
        raise ValueError("grid sizes >= 3 (distinct +-delta neighbours)")
    if K is None:
        K = fem.assemble_K(grid, E, nu)
    S = stencil_functions(grid, K)                          # (noff, d, d, n)
    nshape = grid.nshape                                     # (z, y, x)
    Sg = S.reshape(S.shape[:3] + nshape)
    samp = Sg[(Ellipsis,) + tuple(slice(None, None, M) for _ in range(grid.d))]
    coef = interpolation_coefficients(samp, q, grid.d)
    St = evaluate(coef, q, M, nshape)
    return St.reshape(S.shape)


def surrogate_matrix(grid, St):
    """Kt from the surrogate stencil functions: off-diagonal blocks at
    +-delta (transposes for -delta), diagonal blocks = minus the block row
    sums of the off-diagonal ones (eq. DefinitionOfSurrogateMatrixSymmetricKernel)."""
    d, n = grid.d, grid.n
    idx = np.arange(n)
    rows, cols, vals = [], [], []
    diag = np.zeros((d, d, n))
    for k, delta in enumerate(offsets(d)):
        j = shifted(grid, delta)
        for a in range(d):
            for b in range(d):
                v = St[k, a, b]
                rows += [a * n + idx, b * n + j]          # (i, i+delta) and its transpose (i+delta, i)
                cols += [b * n + j, a * n + idx]
                vals += [v, v]
                diag[a, b] -= v                           # row i: sum over b-columns of block (i, i+delta)
                # row i+delta gets block (i+delta, i) = St^T: entry [b, a] at node i+delta
                np.add.at(diag[b, a], j, -v)
    for a in range(d):
        for b in range(d):
            rows.append(a * n + idx)
            cols.append(b * n + idx)
            vals.append(0.5 * (diag[a, b] + diag[b, a]))
    N = d * n
    Kt = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N)).tocsr()
    Kt.sum_duplicates()
    return Kt


def solve(grid, E, nu, eps_bar, Kt):
    """min 1/2 u.Kt u - f.u subject to zero nodal mean of every component:
    the bordered system [[Kt, C^T], [C, 0]] [u; l] = [f; 0] (exact f)."""
    f = fem.assemble_rhs(grid, E, nu, eps_bar)
    d, n = grid.d, grid.n
    C = sp.csr_matrix((np.ones(d * n), (np.repeat(np.arange(d), n), np.arange(d * n))), shape=(d, d * n))
    A = sp.bmat([[Kt, C.T], [C, None]]).tocsc()
    lu = spla.splu(A)
    u = np.zeros_like(f)
    for J in range(f.shape[0]):
        u[J] = lu.solve(np.concatenate([f[J], np.zeros(d)]))[:d * n]
    return u, f


def effective_stiffness(grid, E, nu, M, q):
    """C* of the surrogate solutions for the unit loads (exact energy form
    on their strain fields) and the solutions u~ (nv, d n)."""
    eb = fem.unit_loads(grid.d)
    St = surrogate_stencils(grid, E, nu, M, q)
    Kt = surrogate_matrix(grid, St)
    u, _ = solve(grid, E, nu, eb, Kt)
    return fem.homogenize(grid, E, nu, u, eb)["C_energy"], u


# --------------------------------------------------------------------------
# the same quantities at chosen nodes (grids too large to assemble)
# --------------------------------------------------------------------------


def node_multi_index(grid, nodes):
    """(i_x, i_y[, i_z]) of flat node indices."""
    idx = np.asarray(nodes, dtype=np.int64)
    out = []
    for N in grid.shape:
        out.append(idx % N)
        idx = idx // N
    return out


def stencil_blocks_at(grid, lam, mu, nodes):
    """K_delta(x_i) = K[i, i + delta] for chosen nodes: (len(nodes), noff, d, d).

    Node i and node i + delta share a simplex exactly where they are vertices
    j < k of it with V_k - V_j = delta (the vertices of a Kuhn simplex follow
    a monotone path); the block entry (a, b) collects |s| (lam B^T m m^T B +
    mu B^T S B) at rows (a, vertex j), columns (b, vertex k) over those
    simplices, with the (lam, mu) of the voxel at i - V_j.  lam, mu: per voxel
    (n,)."""
    d = grid.d
    offs = [tuple(o) for o in offsets(d)]
    comps = node_multi_index(grid, nodes)
    m = fem.voigt_m(d)
    S = np.diag(fem.voigt_s(d))
    nv1 = d + 1
    out = np.zeros((len(comps[0]), len(offs), d, d))
    for V, vol, B in fem.element_data(grid):
        Kl = vol * (B.T @ np.outer(m, m) @ B)
        Km = vol * (B.T @ S @ B)
        for j in range(nv1):
            vflat = grid.flat([comps[a] - V[j, a] for a in range(d)])
            lv, mv = lam[vflat], mu[vflat]
            for k in range(j + 1, nv1):
                di = offs.index(tuple(int(x) for x in V[k] - V[j]))
                for a in range(d):
                    for b in range(d):
                        out[:, di, a, b] += lv * Kl[a * nv1 + j, b * nv1 + k] + mv * Km[a * nv1 + j, b * nv1 + k]
    return out


def evaluate_at(coef, q, M, fine_shape, nodes_multi):
    """The B-spline of ``evaluate`` at chosen fine nodes only.  coef: (..., coarse
    lattice in (z, y, x) order); nodes_multi: (i_x, i_y[, i_z]) arrays.
    Returns (len(nodes), ...)."""
    d = len(fine_shape)
    lead = coef.shape[:-d]
    coarse = coef.shape[len(lead):]           # (z, y, x)
    n_nodes = len(nodes_multi[0])
    out = np.zeros((n_nodes,) + lead)
    for t in range(n_nodes):
        # per axis in (z, y, x) order: lattice indices and weights
        taps = []
        for ax in range(d):
            i = int(nodes_multi[d - 1 - ax][t])
            Nc = coarse[ax]
            x = i / M
            js = range(int(np.floor(x)) - 2, int(np.floor(x)) + 3)
            taps.append([(j % Nc, bspline(q, x - j)) for j in js if bspline(q, x - j) != 0.0])
        val = np.zeros(lead)
        for combo in itertools.product(*taps):
            w = 1.0
            for _, wa in combo:
                w *= wa
            val = val + w * coef[(Ellipsis,) + tuple(j for j, _ in combo)]
        out[t] = val
    return out


def surrogate_blocks_at(grid, E, nu, M, q, nodes):
    """Kt_delta(x_i) at chosen nodes: stencil blocks sampled on the lattice of
    every M-th node, their interpolation coefficients, the interpolant at the
    nodes.  Returns (len(nodes), noff, d, d)."""
    if any(N % M for N in grid.shape):
        raise ValueError("M must divide every grid size")
    lam, mu = fem.lame(np.ravel(E), np.ravel(nu))
    d = grid.d
    cshape = tuple(N // M for N in grid.shape)                       # (x, y[, z])
    cgrid = np.meshgrid(*[np.arange(Nc) * M for Nc in reversed(cshape)], indexing="ij")  # (z, y, x)
    cm = [cgrid[d - 1 - a].ravel() for a in range(d)]                # i_x, i_y[, i_z]
    cflat = grid.flat(cm)
    Sc = stencil_blocks_at(grid, lam, mu, cflat)                     # (nc, noff, d, d)
    samp = np.moveaxis(Sc, 0, -1).reshape(Sc.shape[1:] + tuple(reversed(cshape)))
    coef = interpolation_coefficients(samp, q, d)
    return evaluate_at(coef, q, M, grid.nshape, node_multi_index(grid, nodes))


def apply_at(grid, E, nu, M, q, p, nodes):
    """Rows of Kt p at chosen nodes (the matrix of ``surrogate_matrix``):
    (Kt p)_i = sum_delta [Kt_delta(x_i) p_{i+delta} + Kt_delta(x_{i-delta})^T p_{i-delta}]
               - sym(R_i) p_i,  R_i = sum_delta [Kt_delta(x_i) + Kt_delta(x_{i-delta})^T].
    p: (d n,) component-major.  Returns (len(nodes), d)."""
    d, n = grid.d, grid.n
    offs = offsets(d)
    nodes = np.asarray(nodes, dtype=np.int64)
    mi = node_multi_index(grid, nodes)
    minus = [grid.flat([mi[a] - o[a] for a in range(d)]) for o in offs]
    plus = [grid.flat([mi[a] + o[a] for a in range(d)]) for o in offs]
    allnodes = np.concatenate([nodes] + minus)
    blocks = surrogate_blocks_at(grid, E, nu, M, q, allnodes)
    nn = len(nodes)
    A = blocks[:nn]                                                  # Kt_delta(x_i)
    P = p.reshape(d, n)
    out = np.zeros((nn, d))
    R = np.zeros((nn, d, d))
    for k in range(len(offs)):
        Bm = blocks[nn * (k + 1):nn * (k + 2), k]                    # Kt_delta(x_{i-delta})
        out += np.einsum("tab,bt->ta", A[:, k], P[:, plus[k]])
        out += np.einsum("tba,bt->ta", Bm, P[:, minus[k]])
        R += A[:, k] + np.transpose(Bm, (0, 2, 1))
    Rs = 0.5 * (R + np.transpose(R, (0, 2, 1)))
    out -= np.einsum("tab,bt->ta", Rs, P[:, nodes])
    return out
