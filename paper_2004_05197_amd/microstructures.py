"""Seeded synthetic microstructures for the periodic voxel cell problem.

This module only draws material fields (per-voxel Young's modulus E and
Poisson ratio nu); it holds none of the solver's arithmetic, so both the
CPU oracle's tests and the GPU path use it to build identical inputs.

Conventions shared by every generator:
  * a grid of shape (N_x, N_y[, N_z]) on the unit cell, voxel i covers
    [i_a/N_a, (i_a+1)/N_a) along each axis;
  * returned arrays have numpy shape (N_z, N_y, N_x) in 3D and (N_y, N_x)
    in 2D, so a C-order ``ravel()`` is the colexicographic voxel order
    (x fastest) that the paper uses for multi-indices (Sec. 3.1);
  * all randomness comes from ``numpy.random.default_rng(seed)`` (PCG64).

The paper has no microstructure data for this problem; the recipes below
are the readings recorded in the design notes (circle, random sequential
addition of spheres, thresholded and log-normal Gaussian random fields,
laminates).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "circle2d", "rsa_spheres", "gaussian_random_field", "two_phase_grf",
    "lognormal_field", "laminate", "random_cells", "uneven_cell", "WORKLOADS",
]


def _centres(shape_xyz):
    """Voxel-centre coordinates in voxel units, numpy order (z, y, x)."""
    axes = [np.arange(n, dtype=np.float64) + 0.5 for n in reversed(shape_xyz)]
    return np.meshgrid(*axes, indexing="ij")


def circle2d(n: int = 32, radius: float = 0.25, E_matrix: float = 1.0,
             E_inclusion: float = 10.0, nu: float = 0.3):
    """Centred circular inclusion in a square pixel cell.

    A pixel belongs to the inclusion iff its centre lies strictly inside the
    circle of the given radius (in cell lengths) about the cell centre.
    Returns (E, nu) arrays of shape (n, n).
    """
    yc, xc = _centres((n, n))
    r2 = (xc / n - 0.5) ** 2 + (yc / n - 0.5) ** 2
    inside = r2 < radius * radius
    E = np.where(inside, E_inclusion, E_matrix).astype(np.float64)
    return E, np.full_like(E, nu)


def rsa_spheres(n: int, vf: float, seed: int, rmin: float = 4.0,
                rmax: float = 8.0, max_reject: int = 1_000_000,
                saturate: bool = False):
    """Random sequential addition of non-overlapping periodic spheres.

    Radii r ~ U[rmin, rmax] (voxel units), centres ~ U[0, n)^3.  A candidate
    is accepted iff its minimum-image distance to every accepted centre is at
    least the sum of the radii.  A voxel is inside a sphere iff the
    minimum-image distance from its centre to the sphere centre is < r.
    Spheres are added until the inclusion voxel fraction reaches ``vf``.
    After ``max_reject`` rejected candidates the process is saturated: with
    ``saturate`` the cell keeps the fraction reached, else it raises.
    Returns (mask[bool, (n, n, n)], achieved_vf, list_of_(centre, r)).
    """
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(seed)
    mask = np.zeros((n, n, n), dtype=bool)
    spheres = []
    cen = np.zeros((0, 3))
    rad = np.zeros(0)
    rejects = 0
    target = vf * n ** 3
    count = 0
    block = 64
    while count < target:
        # A block of candidates in the order of the sequential draws (r, then
        # the centre's x, y, z): the same stream as one candidate at a time.
        # Each candidate is tested against the spheres accepted before the
        # block at once (neighbours from a periodic k-d tree, the decision by
        # the minimum-image formula below), then one by one against the
        # block's own acceptances -- the outcome of testing sequentially.
        u = rng.random((block, 4))
        rb = rmin + (rmax - rmin) * u[:, 0]
        cb = n * u[:, 1:]
        nb = len(rad)
        clash = np.zeros(block, dtype=bool)
        if nb:
            kq = min(nb, 32)
            tree = cKDTree(cen % n, boxsize=n)
            dist, idx = tree.query(cb % n, k=kq)
            dist = dist.reshape(block, kq)
            idx = idx.reshape(block, kq)
            dv = cb[:, None, :] - cen[idx]
            dv -= n * np.round(dv / n)
            d2 = dv[..., 0] ** 2 + dv[..., 1] ** 2 + dv[..., 2] ** 2
            clash = np.any(d2 < (rb[:, None] + rad[idx]) ** 2, axis=1)
            # more than kq spheres may lie within reach: test those in full
            full = (~clash) & (kq < nb) & (dist[:, -1] < rb + rmax + 1e-6)
            for k in np.nonzero(full)[0]:
                dv = cb[k][None, :] - cen
                dv -= n * np.round(dv / n)
                d2 = dv[:, 0] ** 2 + dv[:, 1] ** 2 + dv[:, 2] ** 2
                clash[k] = np.any(d2 < (rb[k] + rad) ** 2)
        accepted_here = 0
        kend = block
        for k in np.nonzero(~clash)[0]:
            if count >= target:
                kend = k
                break
            r, c = rb[k], cb[k]
            ok = True
            if len(rad) > nb:
                dv = c[None, :] - cen[nb:]
                dv -= n * np.round(dv / n)
                d2 = dv[:, 0] ** 2 + dv[:, 1] ** 2 + dv[:, 2] ** 2
                ok = not np.any(d2 < (r + rad[nb:]) ** 2)
            if not ok:
                rejects += 1
                continue
            accepted_here += 1
            spheres.append((c, r))
            cen = np.vstack([cen, c[None, :]])
            rad = np.append(rad, r)
            # voxels in the bounding box, wrapped periodically
            lo = np.floor(c - r - 1).astype(int)
            hi = np.ceil(c + r + 1).astype(int)
            ix = np.arange(lo[0], hi[0])
            iy = np.arange(lo[1], hi[1])
            iz = np.arange(lo[2], hi[2])
            dx = (ix + 0.5) - c[0]
            dy = (iy + 0.5) - c[1]
            dz = (iz + 0.5) - c[2]
            d2 = dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2
            sel = d2 < r * r
            zz, yy, xx = np.nonzero(sel)
            flat = np.unique(((iz[zz] % n) * n + (iy[yy] % n)) * n + (ix[xx] % n))
            count += int(np.count_nonzero(~mask.ravel()[flat]))
            mask.ravel()[flat] = True
        rejects += int(np.count_nonzero(clash[:kend]))
        if rejects > max_reject:
            if saturate:
                break
            raise RuntimeError("rsa_spheres: too many rejections")
        # larger blocks once acceptances become rare
        if accepted_here <= 1:
            block = min(block * 2, 1 << 15)
    return mask, count / n ** 3, spheres


def gaussian_random_field(shape_xyz, ell: float, seed: int):
    """Standardized periodic Gaussian random field.

    White noise w ~ N(0,1) on the grid is filtered in Fourier space by
    exp(-ell^2 |xi|^2 / 4), xi_a = 2 pi k_a / N_a with signed k_a, which
    gives a covariance proportional to exp(-r^2 / (2 ell^2)) (r in voxels).
    The result is shifted/scaled to sample mean 0 and standard deviation 1.
    Returns an array of numpy shape reversed(shape_xyz).
    """
    rng = np.random.default_rng(seed)
    nshape = tuple(reversed(shape_xyz))
    w = rng.standard_normal(nshape)
    ks = [2.0 * np.pi * np.fft.fftfreq(m) for m in nshape]
    grids = np.meshgrid(*ks, indexing="ij")
    xi2 = sum(g * g for g in grids)
    g = np.fft.ifftn(np.fft.fftn(w) * np.exp(-ell * ell * xi2 / 4.0)).real
    g -= g.mean()
    g /= g.std()
    return g


def two_phase_grf(n: int, seed: int, ell: float = 8.0, E_soft: float = 1.0,
                  E_hard: float = 1000.0, nu_soft: float = 0.25,
                  nu_hard: float = 0.35):
    """Two-phase field from a GRF thresholded at 0 (g < 0 soft, g >= 0 hard)."""
    g = gaussian_random_field((n, n, n), ell, seed)
    hard = g >= 0.0
    E = np.where(hard, E_hard, E_soft).astype(np.float64)
    nu = np.where(hard, nu_hard, nu_soft).astype(np.float64)
    return E, nu


def lognormal_field(n: int, seed: int, ell: float = 6.0, mu: float = 0.0,
                    sigma: float = 1.0, nu: float = 0.3):
    """Log-normal Young's modulus E = exp(mu + sigma g), g a standardized GRF."""
    g = gaussian_random_field((n, n, n), ell, seed)
    E = np.exp(mu + sigma * g)
    return E, np.full_like(E, nu)


def laminate(shape_xyz, axis: int, layer_E, layer_nu, thickness):
    """Layered material: whole voxel slabs normal to ``axis`` (0 = x).

    ``thickness[k]`` voxels of phase k follow each other along ``axis``
    (their sum must equal the grid size along that axis).
    """
    thickness = list(thickness)
    if sum(thickness) != shape_xyz[axis]:
        raise ValueError("layer thicknesses must sum to the grid size")
    prof_E = np.repeat(np.asarray(layer_E, float), thickness)
    prof_nu = np.repeat(np.asarray(layer_nu, float), thickness)
    d = len(shape_xyz)
    nshape = tuple(reversed(shape_xyz))
    np_axis = d - 1 - axis
    bshape = [1] * d
    bshape[np_axis] = shape_xyz[axis]
    E = np.broadcast_to(prof_E.reshape(bshape), nshape).copy()
    nu = np.broadcast_to(prof_nu.reshape(bshape), nshape).copy()
    return E, nu


def uneven_cell(seed: int, sizes=(32, 48, 64, 96), nu: float = 0.3):
    """One cell of the uneven batch, all draws from ``seed``: size ~ U(sizes),
    vf ~ U[0.1, 0.4], contrast ~ U[10, 100], then the sphere seed; spheres
    with r ~ U[4, 8], E = contrast inside and 1 outside.  A target fraction
    the small cells cannot reach keeps the saturated fraction.  Returns a
    dict with keys n, vf, contrast, E, nu, achieved_vf."""
    rng = np.random.default_rng(seed)
    n = int(rng.choice(np.asarray(sizes)))
    vf = float(rng.uniform(0.1, 0.4))
    contrast = float(rng.uniform(10.0, 100.0))
    sub_seed = int(rng.integers(0, 2 ** 31 - 1))
    mask, avf, _ = rsa_spheres(n, vf, sub_seed, saturate=True)
    E = np.where(mask, contrast, 1.0).astype(np.float64)
    return dict(n=n, vf=vf, contrast=contrast, E=E, nu=np.full_like(E, nu), achieved_vf=avf)


def _uneven_cell_args(args):
    return uneven_cell(*args)


def random_cells(count: int, base_seed: int = 1000, sizes=(32, 48, 64, 96),
                 nu: float = 0.3, workers: int = 1):
    """Uneven batch of sphere microstructures: cell k is
    ``uneven_cell(base_seed + k)``.  With workers > 1 the cells are built in
    that many fresh (spawned) processes; the result does not depend on it."""
    args = [(base_seed + k, sizes, nu) for k in range(count)]
    if workers <= 1:
        for a in args:
            yield uneven_cell(*a)
        return
    import concurrent.futures as cf
    import multiprocessing as mp
    with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        yield from ex.map(_uneven_cell_args, args, chunksize=2)


def spheres_cell(n: int, vf: float, seed: int, contrast: float,
                 nu: float = 0.3, rmin: float = 4.0, rmax: float = 8.0):
    """Sphere microstructure with E = contrast in the spheres, 1 outside."""
    mask, avf, _ = rsa_spheres(n, vf, seed, rmin, rmax)
    E = np.where(mask, contrast, 1.0).astype(np.float64)
    return E, np.full_like(E, nu), avf


# Named workloads (synthetic stand-ins, sizes as used by tests and bench).
WORKLOADS = {
    "circle2d_32": dict(dim=2, n=32, desc="2D plane strain 32x32, centred "
                        "circle r=0.25L, E 1/10, nu 0.3, eps_xx=1e-2, FP64 tol 1e-10"),
    "spheres3d_64": dict(dim=3, n=64, desc="3D 64^3 RSA spheres r 4-8 vf 0.3 "
                         "seed 2, E 1:100, nu 0.3, 6 unit loads"),
    "grf3d_256": dict(dim=3, n=256, desc="3D 256^3 two-phase thresholded GRF "
                      "ell 8 seed 3, E 1:1000, nu 0.25/0.35, 6 loads, tol 1e-6"),
    "batch512_spheres": dict(dim=3, n=None, desc="512 cells, N in {32,48,64,96}, "
                             "RSA spheres vf 0.1-0.4, contrast 10-100, 6 loads"),
    "lognormal3d_128": dict(dim=3, n=128, desc="3D 128^3 log-normal E (ell 6, "
                            "seed 5), nu 0.3, J = C1111 + C2323, gradient wrt E"),
}
