"""Strain-based Fourier projection variant of the cell solve (CPU, FP64).

Test infrastructure only (see the package docstring).

Instead of iterating on nodal displacements, conjugate gradients iterate on
compatible strain fields (one Voigt strain per simplex): the unknown is
e = B u, the operator is the FE-gradient projection applied to the stress,
A e = B M^-1 B^T D e with M = B^T D0 B the reference operator (inverted in
Fourier space by ``matfree.FourierPreconditioner``), and the inner product
is <e, h>_0 = sum_s |s| e_s . D0 h_s.  On compatible fields A is
self-adjoint and positive for that inner product, and the CG iterates are
B u_k of the displacement PCG with preconditioner M^-1 (same alpha, beta:
<B z, B z>_0 = z.M z = r.z and <A B p, B p>_0 = p.K p), so the two reach
the same discrete solution in the same number of iterations when stopped
on the same residual, ||f - K u_k|| = ||B^T D (eps_bar + e_k)||.  It stores
d!(d(d+1)/2) strain values per voxel (36 in 3D) against d displacements per
node: a cross-check of the iteration, not a faster method.
"""
from __future__ import annotations

import numpy as np

from . import fem, matfree


def _fields(grid):
    """Per simplex type: (volume, B (nv, d(d+1)), dofs (n, d(d+1)))."""
    return [(vol, B, fem.simplex_dofs(grid, V)) for V, vol, B in fem.element_data(grid)]


def strains(grid, el, u):
    """B u per simplex type: list of (n, nv); u is (d n,)."""
    return [u[dofs] @ B.T for vol, B, dofs in el]


def stresses(grid, el, lam, mu, eps):
    """D_v e_s per simplex type (Voigt, engineering shear in e)."""
    m = fem.voigt_m(grid.d)
    s = fem.voigt_s(grid.d)
    return [lam[:, None] * (e @ m)[:, None] * m[None, :] + mu[:, None] * e * s[None, :] for e in eps]


def divergence(grid, el, sig):
    """sum_s |s| B_s^T sig_s as a nodal vector (d n,)."""
    N = grid.d * grid.n
    out = np.zeros(N)
    for (vol, B, dofs), sg in zip(el, sig):
        out += np.bincount(dofs.ravel(), weights=(vol * sg @ B).ravel(), minlength=N)
    return out


def inner0(grid, el, lam0, mu0, a, b):
    """<a, b>_0 = sum_s |s| a_s . D0 b_s."""
    n = grid.n
    sig = stresses(grid, el, np.full(n, lam0), np.full(n, mu0), b)
    return float(sum(vol * np.sum(x * y) for (vol, _, _), x, y in zip(el, a, sig)))


def projection_cg(grid, E, nu, eps_bar, tol=1e-12, maxit=2000):
    """CG on compatible strains for one macro strain (Voigt, (nv,)).

    Stops when ||B^T D (eps_bar + e)||_2 <= tol ||f||_2.  Returns (e as a
    list per simplex type of (n, nv), iterations, residual history)."""
    E = np.ravel(E)
    nu = np.ravel(nu)
    lam, mu = fem.lame(E, nu)
    d, n = grid.d, grid.n
    lam0, mu0 = matfree.reference_medium(E, nu, d)
    pre = matfree.FourierPreconditioner(grid, lam0, mu0)
    el = _fields(grid)

    def Minv(v):  # nodal (d n,) -> (d n,)
        return pre(v.reshape((d,) + grid.nshape)).ravel()

    ebar = [np.tile(np.asarray(eps_bar, dtype=np.float64), (n, 1)) for _ in el]
    f = -divergence(grid, el, stresses(grid, el, lam, mu, ebar))
    fn = np.linalg.norm(f)
    e = [np.zeros((n, grid.nv)) for _ in el]
    r = f.copy()
    hist = [1.0]
    if fn == 0.0:
        return e, 0, hist
    rho = strains(grid, el, Minv(r))
    p = [x.copy() for x in rho]
    gam = inner0(grid, el, lam0, mu0, rho, rho)
    it = 0
    while it < maxit:
        w = divergence(grid, el, stresses(grid, el, lam, mu, p))    # B^T D p
        Ap = strains(grid, el, Minv(w))                              # B M^-1 B^T D p
        alpha = gam / inner0(grid, el, lam0, mu0, Ap, p)
        e = [x + alpha * y for x, y in zip(e, p)]
        rho = [x - alpha * y for x, y in zip(rho, Ap)]
        r = r - alpha * w
        it += 1
        hist.append(np.linalg.norm(r) / fn)
        if hist[-1] <= tol:
            break
        gnew = inner0(grid, el, lam0, mu0, rho, rho)
        beta = gnew / gam
        gam = gnew
        p = [x + beta * y for x, y in zip(rho, p)]
    return e, it, hist


def effective_stiffness(grid, E, nu, tol=1e-12):
    """C* (energy form) from the strain CG of every unit load, and the
    iteration counts."""
    lam, mu = fem.lame(np.ravel(E), np.ravel(nu))
    el = _fields(grid)
    eb = fem.unit_loads(grid.d)
    tot, its = [], []
    for J in range(grid.nv):
        e, it, _ = projection_cg(grid, E, nu, eb[J], tol=tol)
        tot.append([x + eb[J][None, :] for x in e])
        its.append(it)
    C = np.zeros((grid.nv, grid.nv))
    for J in range(grid.nv):
        sig = stresses(grid, el, lam, mu, tot[J])
        for I in range(grid.nv):
            C[I, J] = sum(vol * np.sum(x * y) for (vol, _, _), x, y in zip(el, tot[I], sig))
    return C / grid.volume, its
