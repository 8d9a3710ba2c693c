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
"""
from __future__ import annotations

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
