"""Matrix-free operator, Fourier reference preconditioner and PCG (CPU, FP64).

Test infrastructure only (see the package docstring).

The operator is the same sum over voxels and Kuhn simplices as in ``fem``
(sum_v sum_s |s| B_s^T D_v B_s), applied with whole-array numpy shifts so
that grids too large to assemble (32^3 and up) can still be solved and
timed.  Fields are arrays of numpy shape (d, N_z, N_y, N_x) (3D) or
(d, N_y, N_x) (2D), C-order, i.e. colexicographic with x fastest (Sec. 3.1).

Preconditioner: for a homogeneous reference medium every stencil function
is constant (Sec. 3.2: the matrix entries depend only on the offset), so the
reference operator is a block convolution and the DFT diagonalizes it.  Its
3x3 (2x2) symbol is taken *numerically*: apply the reference operator to a
unit impulse in each component and DFT the response.  No closed form is
used here.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft as sfft

from .fem import Grid, element_data, lame, voigt_m, voigt_s

WORKERS = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()


def _shift(f, offset_xyz):
    """g[..., i] = f[..., i + offset] with periodic wrap (x is the last axis)."""
    d = len(offset_xyz)
    shifts = tuple(-int(o) for o in reversed(offset_xyz))
    axes = tuple(range(f.ndim - d, f.ndim))
    return np.roll(f, shifts, axis=axes)


def _unshift(f, offset_xyz):
    """Inverse of _shift: g[..., i + offset] = f[..., i]."""
    d = len(offset_xyz)
    shifts = tuple(int(o) for o in reversed(offset_xyz))
    axes = tuple(range(f.ndim - d, f.ndim))
    return np.roll(f, shifts, axis=axes)


def neg_divergence_stress(grid: Grid, lam, mu, u, eps_bar):
    """r = -sum_v sum_s |s| B_s^T D_v (eps_bar + B_s u).

    With eps_bar = 0 this is -K u; with u = 0 it is the load vector f; in
    general it is the residual f - K u of the cell problem.
    lam, mu: per-voxel arrays of numpy shape grid.nshape.
    u: (d,) + grid.nshape.  eps_bar: (nv,).
    """
    d = grid.d
    m = voigt_m(d)
    s = voigt_s(d)
    out = np.zeros((d,) + grid.nshape)
    for V, vol, B in element_data(grid):
        nvert = d + 1
        # strain on this simplex in every voxel
        e = np.zeros((grid.nv,) + grid.nshape)
        e += np.asarray(eps_bar, dtype=np.float64).reshape((-1,) + (1,) * d)
        for j in range(nvert):
            uj = _shift(u, V[j])
            for c in range(d):
                col = B[:, c * nvert + j]
                for row in range(grid.nv):
                    if col[row] != 0.0:
                        e[row] += col[row] * uj[c]
        tr = np.tensordot(m, e, axes=(0, 0))
        sig = lam[None] * tr[None] * m.reshape((-1,) + (1,) * d) + mu[None] * e * s.reshape((-1,) + (1,) * d)
        for j in range(nvert):
            contrib = np.zeros((d,) + grid.nshape)
            for c in range(d):
                col = B[:, c * nvert + j]
                for row in range(grid.nv):
                    if col[row] != 0.0:
                        contrib[c] += col[row] * sig[row]
            out -= vol * _unshift(contrib, V[j])
    return out


def apply_K(grid, lam, mu, u):
    """K u (matrix-free)."""
    zero = np.zeros(grid.nv)
    return -neg_divergence_stress(grid, lam, mu, u, zero)


def reference_medium(E, nu, d):
    """Homogeneous reference medium used by the preconditioner.

    Bulk modulus K and shear modulus mu are the geometric means of their
    extreme values over the voxels (3D bulk K = lambda + 2 mu / 3; 2D plane
    strain in-plane bulk K = lambda + mu).  Any SPD choice gives the same
    solution; only the iteration count depends on it.
    """
    lam, mu = lame(E, nu)
    bulk = lam + (2.0 * mu / 3.0 if d == 3 else mu)
    K0 = np.sqrt(bulk.min() * bulk.max())
    mu0 = np.sqrt(mu.min() * mu.max())
    lam0 = K0 - (2.0 * mu0 / 3.0 if d == 3 else mu0)
    return lam0, mu0


def reference_symbol(grid, lam0, mu0):
    """Fourier symbol of the homogeneous reference operator, numerically.

    K_hat[c, e](k) = rfftn(response_e[c])(k), response_e = K_ref applied to a
    unit impulse in component e at node 0.  Because K_ref is translation
    invariant, K_ref u = sum_e response_e (*) u_e (circular convolution),
    hence rfftn((K_ref u)_c) = sum_e K_hat[c, e] rfftn(u_e).
    Returns complex array (d, d, rfft shape).
    """
    d = grid.d
    lam = np.full(grid.nshape, float(lam0))
    mu = np.full(grid.nshape, float(mu0))
    cols = []
    for e in range(d):
        imp = np.zeros((d,) + grid.nshape)
        imp[(e,) + (0,) * d] = 1.0
        resp = apply_K(grid, lam, mu, imp)
        cols.append(np.stack([sfft.rfftn(resp[c], workers=WORKERS) for c in range(d)]))
    return np.stack(cols, axis=1)  # [c, e, ...]


class FourierPreconditioner:
    """z = K_ref^{-1} r in Fourier space; the zero frequency is set to 0."""

    def __init__(self, grid, lam0, mu0):
        self.grid = grid
        Kh = reference_symbol(grid, lam0, mu0)
        d = grid.d
        spec_shape = Kh.shape[2:]
        M = np.moveaxis(Kh.reshape(d, d, -1), 2, 0)  # (nk, d, d)
        M[0] = np.eye(d)  # zero frequency: excluded below
        self.Minv = np.linalg.inv(M)
        self.spec_shape = spec_shape

    def __call__(self, r):
        g = self.grid
        d = g.d
        rh = np.stack([sfft.rfftn(r[c], workers=WORKERS).ravel() for c in range(d)], axis=1)
        zh = np.einsum("kab,kb->ka", self.Minv, rh)
        zh[0] = 0.0
        z = np.stack([sfft.irfftn(zh[:, c].reshape(self.spec_shape), s=g.nshape, workers=WORKERS)
                      for c in range(d)])
        return z


def pcg(grid, E, nu, eps_bar, tol=1e-12, maxit=2000, x0=None, precond=None,
        callback=None):
    """Preconditioned conjugate gradients (Hestenes-Stiefel) on K u = f.

    Stops when ||r||_2 <= tol ||f||_2 (unpreconditioned residual).
    Returns (u of shape (d,)+nshape, iterations, final relative residual).
    """
    E = np.asarray(E, dtype=np.float64).reshape(grid.nshape)
    nu = np.asarray(nu, dtype=np.float64).reshape(grid.nshape)
    lam, mu = lame(E, nu)
    if precond is None:
        precond = FourierPreconditioner(grid, *reference_medium(E, nu, grid.d))
    d = grid.d
    f = neg_divergence_stress(grid, lam, mu, np.zeros((d,) + grid.nshape), eps_bar)
    fn = np.sqrt(np.sum(f * f))
    x = np.zeros_like(f) if x0 is None else np.array(x0, dtype=np.float64)
    r = f - apply_K(grid, lam, mu, x)
    if fn == 0.0:
        return x, 0, 0.0
    rn = np.sqrt(np.sum(r * r))
    if rn <= tol * fn:
        return x, 0, rn / fn
    z = precond(r)
    p = z.copy()
    rz = np.sum(r * z)
    it = 0
    while it < maxit:
        q = apply_K(grid, lam, mu, p)
        alpha = rz / np.sum(p * q)
        x += alpha * p
        r -= alpha * q
        it += 1
        rn = np.sqrt(np.sum(r * r))
        if callback is not None:
            callback(it, rn / fn)
        if rn <= tol * fn:
            break
        z = precond(r)
        rz_new = np.sum(r * z)
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    for c in range(d):
        x[c] -= x[c].mean()
    return x, it, rn / fn


def homogenize(grid, E, nu, u, eps_bar):
    """Energy-form C* column data and mean stress from a matrix-free field.

    u: (nload, d) + nshape.  Returns dict like fem.homogenize.
    """
    E = np.asarray(E, dtype=np.float64).reshape(grid.nshape)
    nu = np.asarray(nu, dtype=np.float64).reshape(grid.nshape)
    lam, mu = lame(E, nu)
    d = grid.d
    m = voigt_m(d)
    s = voigt_s(d)
    nl = eps_bar.shape[0]
    C = np.zeros((nl, nl))
    sbar = np.zeros((nl, grid.nv))
    for V, vol, B in element_data(grid):
        nvert = d + 1
        strains = []
        for J in range(nl):
            e = np.zeros((grid.nv,) + grid.nshape)
            e += eps_bar[J].reshape((-1,) + (1,) * d)
            for j in range(nvert):
                uj = _shift(u[J], V[j])
                for c in range(d):
                    col = B[:, c * nvert + j]
                    for row in range(grid.nv):
                        if col[row] != 0.0:
                            e[row] += col[row] * uj[c]
            strains.append(e)
        sigs = []
        for J in range(nl):
            e = strains[J]
            tr = np.tensordot(m, e, axes=(0, 0))
            sigs.append(lam[None] * tr[None] * m.reshape((-1,) + (1,) * d)
                        + mu[None] * e * s.reshape((-1,) + (1,) * d))
        for J in range(nl):
            sbar[J] += vol * sigs[J].reshape(grid.nv, -1).sum(axis=1)
            for I in range(nl):
                C[I, J] += vol * np.sum(strains[I] * sigs[J])
    return dict(C_energy=C / grid.volume, mean_stress=sbar / grid.volume)
