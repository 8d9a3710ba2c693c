"""Operator and preconditioner parity on a seeded sample of grid shapes:
every axis length drawn from the supported sizes up to 48 (4, 6, 8, 12, 16,
24, 32, 48), 2D and 3D, unequal edge lengths, FP64 and FP32.  The tiled
kernels fall back to other tiles or to the runtime-tile kernel where a tile
does not divide the grid, and the FFT passes meet every codelet length
below 48; this sweep checks that every such combination matches the
oracle (tolerances as in tests/test_gpu_parity.py)."""
import numpy as np
import pytest

from oracle import fem, matfree

pytestmark = pytest.mark.gpu

SIZES = (4, 6, 8, 12, 16, 24, 32, 48)


def shapes(count=24, seed=11):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        d = 2 if i % 4 == 3 else 3
        out.append(tuple(int(v) for v in rng.choice(SIZES, size=d)))
    return out


def relerr(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


@pytest.mark.parametrize("shape", shapes())
def test_operator_and_preconditioner_on_sampled_shapes(lib, shape):
    rng = np.random.default_rng(sum(shape))
    nshape = tuple(reversed(shape))
    E = rng.uniform(1.0, 40.0, nshape)
    nu = rng.uniform(0.05, 0.45, nshape)
    lengths = [1.0 + 0.15 * a for a in range(len(shape))]
    grid = fem.Grid(shape, lengths=lengths)
    lam, mu = fem.lame(E, nu)
    u = rng.standard_normal((grid.d,) + grid.nshape)
    Ku = matfree.apply_K(grid, lam, mu, u).ravel()
    r = rng.standard_normal((grid.d,) + grid.nshape)
    r -= r.reshape(grid.d, -1).mean(axis=1).reshape((grid.d,) + (1,) * grid.d)
    for prec, tol_k, tol_m in ((0, 1e-12, 1e-10), (1, 2e-5, 1e-4)):
        with lib.Cell(shape, precision=prec, lengths=grid.L) as c:
            c.set_material(E.ravel(), nu.ravel())
            q = c.apply_operator(u.ravel(), precision=prec)
            zref = matfree.FourierPreconditioner(grid, *c.reference_medium())(r).ravel()
            z = c.apply_preconditioner(r.ravel(), precision=prec)
        assert relerr(q, Ku) < tol_k, (shape, prec, relerr(q, Ku))
        assert relerr(z, zref) < tol_m, (shape, prec, relerr(z, zref))
