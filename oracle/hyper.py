"""Compressible neo-Hookean cell problem: explicit assembly, Newton's
method with direct sparse solves (CPU, FP64).

Test infrastructure only (see the package docstring).

Energy density (Sec. 2.2, eq. NeoHookeanEnergy), with J = det F:

    W(F) = lambda/2 (ln J)^2 - mu ln J + mu/2 (tr(F^T F) - tr I).

On the periodic cell the deformation gradient of simplex s is
F_s = F_bar + grad u~ on s, with the macroscopic gradient F_bar and the
periodic P1 fluctuation u~ on the Kuhn subdivision (the same mesh, node
numbering and dof layout as ``fem``: u is (d, n), component-major).  The
fluctuation minimises Pi(u~) = sum_v sum_s |s| W_v(F_s).  2D is plane
strain: F is the in-plane 2 x 2 block (F_33 = 1), so J = det F and
tr(F^T F) - tr I reads the same with tr I = 2.

Derivatives (standard continuum mechanics, written out):
    P(F)  = dW/dF = mu (F - F^-T) + lambda ln J F^-T,
    dP    = A(F) : dF
          = mu dF + (mu - lambda ln J) F^-T dF^T F^-T + lambda tr(F^-1 dF) F^-T.
The nodal residual is f = -sum |s| B^T P (f_{a,j} = -|s| sum_b P_ab g_jb
for the barycentric gradient g_j of vertex j), the tangent
K_T = sum |s| G^T A G.  Newton's method (Sec. 4, subsection on nonlinear
problems: the Jacobian is reassembled in each iteration) solves K_T du = f
with node 0 pinned and takes the largest step t in {1, 1/2, 1/4, ...} that
keeps every J > 0 and decreases Pi by at least 1e-4 t f.du (Armijo).  The
paper does not fix the step control; near the solution the decrease falls
below the rounding level of Pi (about 1e-13 |Y| max(|lambda| + 2 mu)
d (1 + |F_bar|^2)), and there a step is also taken when Pi does not grow by
more than that level and ||f|| falls by the factor 1 - 1e-4 t.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import Grid, kuhn_simplices, lame, p1_gradients  # noqa: F401


# --------------------------------------------------------------------------
# material law (vectorised over leading axes; F has shape (..., d, d))
# --------------------------------------------------------------------------


def energy_density(F, lam, mu):
    """W(F) of eq. NeoHookeanEnergy; nan where det F <= 0."""
    d = F.shape[-1]
    J = np.linalg.det(F)
    with np.errstate(invalid="ignore", divide="ignore"):
        lnJ = np.where(J > 0, np.log(np.where(J > 0, J, 1.0)), np.nan)
    trC = np.einsum("...ab,...ab->...", F, F)
    return 0.5 * lam * lnJ ** 2 - mu * lnJ + 0.5 * mu * (trC - d)


def piola(F, lam, mu):
    """First Piola-Kirchhoff stress P = dW/dF."""
    Finv = np.linalg.inv(F)
    FinvT = np.swapaxes(Finv, -1, -2)
    lnJ = np.log(np.linalg.det(F))
    return (mu[..., None, None] * (F - FinvT) + (lam * lnJ)[..., None, None] * FinvT)


def tangent(F, lam, mu):
    """A_{abce} = d P_ab / d F_ce, shape (..., d, d, d, d)."""
    d = F.shape[-1]
    Finv = np.linalg.inv(F)
    lnJ = np.log(np.linalg.det(F))
    I = np.eye(d)
    # mu dF_ab                        -> mu delta_ac delta_be
    # (mu - lam lnJ) (F^-T dF^T F^-T)_ab = (mu - lam lnJ) Finv_ea Finv_bc
    # lam tr(F^-1 dF) F^-T_ab            = lam Finv_ec Finv_ba
    A = mu[..., None, None, None, None] * np.einsum("ac,be->abce", I, I)
    A = A + (mu - lam * lnJ)[..., None, None, None, None] * np.einsum("...ea,...bc->...abce", Finv, Finv)
    A = A + lam[..., None, None, None, None] * np.einsum("...ec,...ba->...abce", Finv, Finv)
    return A


# --------------------------------------------------------------------------
# mesh quantities
# --------------------------------------------------------------------------


def simplex_data(grid):
    """Per simplex type: (vertex offsets V, volume, barycentric gradients
    (d+1, d), node indices (d+1, n) of its vertices in every voxel)."""
    out = []
    mi = grid.multi_index()
    for V in kuhn_simplices(grid.d):
        X = V * np.asarray(grid.h)[None, :]
        g, vol = p1_gradients(X)
        nodes = np.stack([grid.flat([mi[a] + V[j, a] for a in range(grid.d)]) for j in range(V.shape[0])])
        out.append((V, vol, g, nodes))
    return out


def deformation_gradients(grid, u, Fbar):
    """F_s = F_bar + grad u on every (simplex type, voxel): list of (n, d, d)."""
    u = np.asarray(u, dtype=np.float64).reshape(grid.d, grid.n)
    out = []
    for V, vol, g, nodes in simplex_data(grid):
        G = np.einsum("ajv,jb->vab", u[:, nodes], g)
        out.append(np.asarray(Fbar)[None] + G)
    return out


def total_energy(grid, E, nu, u, Fbar):
    """Pi(u) = sum_v sum_s |s| W_v(F_s) (nan if any J <= 0)."""
    lam, mu = lame(np.ravel(E), np.ravel(nu))
    tot = 0.0
    for (V, vol, g, nodes), F in zip(simplex_data(grid), deformation_gradients(grid, u, Fbar)):
        tot += vol * np.sum(energy_density(F, lam, mu))
    return tot


def residual(grid, E, nu, u, Fbar):
    """f = -sum |s| B^T P(F_s), shape (d, n)."""
    lam, mu = lame(np.ravel(E), np.ravel(nu))
    f = np.zeros((grid.d, grid.n))
    for (V, vol, g, nodes), F in zip(simplex_data(grid), deformation_gradients(grid, u, Fbar)):
        P = piola(F, lam, mu)
        for j in range(grid.d + 1):
            contrib = -vol * np.einsum("vab,b->av", P, g[j])
            for a in range(grid.d):
                f[a] += np.bincount(nodes[j], weights=contrib[a], minlength=grid.n)
    return f


def residual_at_nodes(grid, E, nu, u, Fbar, nodes):
    """f = -sum |s| B^T P(F_s) at selected nodes only (spot checks of fields
    too large for the full evaluation): node = vertex j of simplex type s in
    the voxel at node - V_s[j]; its row of -|s| P g_j, summed over (s, j).
    u: (d n,) or (d, n); nodes: flat indices.  Returns (len(nodes), d)."""
    d = grid.d
    u = np.asarray(u, dtype=np.float64).reshape(d, grid.n)
    nodes = np.asarray(nodes, dtype=np.int64)
    lam, mu = lame(np.ravel(E), np.ravel(nu))
    comps, idx = [], nodes.copy()
    for N in grid.shape:
        comps.append(idx % N)
        idx = idx // N
    out = np.zeros((len(nodes), d))
    for V in kuhn_simplices(d):
        X = V * np.asarray(grid.h)[None, :]
        g, vol = p1_gradients(X)
        for j in range(d + 1):
            vox = [comps[a] - V[j, a] for a in range(d)]
            vflat = grid.flat(vox)
            F = np.tile(np.asarray(Fbar, dtype=np.float64), (len(nodes), 1, 1))
            for k in range(d + 1):
                nk = grid.flat([vox[a] + V[k, a] for a in range(d)])
                F += np.einsum("av,b->vab", u[:, nk], g[k])
            P = piola(F, lam[vflat], mu[vflat])
            out -= vol * np.einsum("vab,b->va", P, g[j])
    return out


def assemble_tangent(grid, E, nu, u, Fbar):
    """Sparse K_T = sum |s| G^T A(F_s) G over the (d n) dofs (CSR)."""
    lam, mu = lame(np.ravel(E), np.ravel(nu))
    d, n = grid.d, grid.n
    rows, cols, vals = [], [], []
    for (V, vol, g, nodes), F in zip(simplex_data(grid), deformation_gradients(grid, u, Fbar)):
        A = tangent(F, lam, mu)
        # K[(a, j), (c, k)] = |s| sum_{b, e} g_jb A_abce g_ke
        Ke = vol * np.einsum("jb,vabce,ke->vajck", g, A, g)
        nv = d + 1
        dof = np.stack([a * n + nodes[j] for a in range(d) for j in range(nv)], axis=1)  # (n, d*nv)
        Ke = Ke.reshape(n, d * nv, d * nv)
        rows.append(np.repeat(dof, d * nv, axis=1).ravel())
        cols.append(np.tile(dof, (1, d * nv)).ravel())
        vals.append(Ke.ravel())
    N = d * n
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N)).tocsr()
    K.sum_duplicates()
    return K


def mean_piola(grid, E, nu, u, Fbar):
    """(1/|Y|) sum_v sum_s |s| P(F_s)."""
    lam, mu = lame(np.ravel(E), np.ravel(nu))
    Pm = np.zeros((grid.d, grid.d))
    for (V, vol, g, nodes), F in zip(simplex_data(grid), deformation_gradients(grid, u, Fbar)):
        Pm += vol * piola(F, lam, mu).sum(axis=0)
    return Pm / grid.volume


# --------------------------------------------------------------------------
# Newton's method
# --------------------------------------------------------------------------


def newton(grid, E, nu, Fbar, tol=1e-12, maxit=30, u0=None):
    """Minimise Pi over periodic fluctuations for the macro gradient F_bar.

    Returns dict(u (d, n) with zero nodal mean per component, P_mean,
    energy (Pi / |Y|), iterations, residual norms per iteration).
    Stops when ||f|| <= tol * max(||f_0||, |Y| max(mu) |F_bar|).
    """
    d, n = grid.d, grid.n
    Fbar = np.asarray(Fbar, dtype=np.float64)
    u = np.zeros((d, n)) if u0 is None else np.array(u0, dtype=np.float64).reshape(d, n)
    pinned = np.array([a * n for a in range(d)])
    keep = np.setdiff1d(np.arange(d * n), pinned)
    lam, mu = lame(np.ravel(E), np.ravel(nu))
    scale = grid.volume * float(np.max(mu)) * max(np.abs(Fbar).max(), 1.0)
    fmax = max(np.abs(Fbar).max(), 1.0)
    dE = 1e-13 * grid.volume * float(np.max(np.abs(lam) + 2 * mu)) * d * (1.0 + fmax ** 2)
    f = residual(grid, E, nu, u, Fbar)
    Pi = total_energy(grid, E, nu, u, Fbar)
    norms = [float(np.linalg.norm(f))]
    ref = max(norms[0], scale)
    it = 0
    while norms[-1] > tol * ref and it < maxit:
        K = assemble_tangent(grid, E, nu, u, Fbar)
        du = np.zeros(d * n)
        du[keep] = spla.spsolve(K[keep][:, keep].tocsc(), f.ravel()[keep])
        du = du.reshape(d, n)
        slope = float(np.sum(f * du))
        t = 1.0
        while True:
            ut = u + t * du
            Pt = total_energy(grid, E, nu, ut, Fbar)
            if np.isfinite(Pt) and Pt <= Pi - 1e-4 * t * slope:
                break
            if np.isfinite(Pt) and Pt - Pi <= dE:
                ft = np.linalg.norm(residual(grid, E, nu, ut, Fbar))
                if ft <= (1.0 - 1e-4 * t) * norms[-1]:
                    break
            t *= 0.5
            if t < 1e-10:
                raise RuntimeError("line search failed")
        u, Pi = ut, Pt
        f = residual(grid, E, nu, u, Fbar)
        norms.append(float(np.linalg.norm(f)))
        it += 1
    u = u - u.mean(axis=1, keepdims=True)
    return dict(u=u, P_mean=mean_piola(grid, E, nu, u, Fbar), energy=Pi / grid.volume, iterations=it,
                norms=norms)
