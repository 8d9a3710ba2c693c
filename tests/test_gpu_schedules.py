"""Every compiled kernel variant a schedule can select, against the oracle,
and the autotuner that picks among them.

Schedules (six ints): stencil tile, stencil z extent, x-pass rows per
block, y-pass columns per block, last-pass columns per block, last-pass
radix order.  Tolerances as in the single-step parity tests: operator FP64
1e-12 / FP32 2e-5, preconditioner FP64 1e-10 / FP32 1e-4.
"""
import json

import numpy as np
import pytest

from oracle import fem, matfree
from paper_2004_05197_amd import microstructures as ms

pytestmark = pytest.mark.gpu


def relerr(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


def rand_material(shape, seed, Emin=1.0, Emax=10.0):
    rng = np.random.default_rng(seed)
    nshape = tuple(reversed(shape))
    return rng.uniform(Emin, Emax, nshape), rng.uniform(0.05, 0.45, nshape)


# (64, 32, 24): every compiled tile divides the grid (tile 5: the FP32
# row-wave kernel); (48, 48, 12): only the 16 x 16 tile does (the others,
# and the row-wave kernel, which needs nx in {64, 128, 256}, fall back to
# it); z extents 8..64 against nz = 24 and 12 give ragged last z tiles
STENCIL_CASES = [(shape, t, tz) for shape in [(64, 32, 24), (48, 48, 12)]
                 for t in range(6) for tz in (8, 16, 32, 64)]


@pytest.mark.parametrize("shape,tile,tz", STENCIL_CASES)
@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 2e-5)])
def test_operator_every_stencil_variant(lib, shape, tile, tz, prec, tol):
    E, nu = rand_material(shape, 1)
    grid = fem.Grid(shape, lengths=[1.0, 1.1, 0.9])
    lam, mu = fem.lame(E, nu)
    u = np.random.default_rng(2).standard_normal((3,) + grid.nshape)
    ref = matfree.apply_K(grid, lam, mu, u).ravel()
    with lib.Cell(shape, precision=prec, lengths=grid.L) as c:
        c.set_material(E.ravel(), nu.ravel())
        c.schedule = (tile, tz, 0, 0, 0, 0)
        assert c.schedule == (tile, tz, 0, 0, 0, 0)
        q = c.apply_operator(u.ravel(), precision=prec)
    assert relerr(q, ref) < tol


FFT_VARIANTS = [(x, y, z, rp) for x in (0, 1, 2, 3) for y in (0, 1, 2, 3) for z in (0, 1, 2, 3) for rp in (0, 1)]


@pytest.mark.parametrize("shape", [(64, 32, 24), (48, 96, 16), (32, 48), (96, 8)])
@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 1e-4)])
def test_preconditioner_every_fft_variant(lib, shape, prec, tol):
    E, nu = rand_material(shape, 3, 1.0, 50.0)
    grid = fem.Grid(shape)
    r = np.random.default_rng(4).standard_normal((grid.d,) + grid.nshape)
    r -= r.reshape(grid.d, -1).mean(axis=1).reshape((grid.d,) + (1,) * grid.d)
    with lib.Cell(shape, precision=prec) as c:
        c.set_material(E.ravel(), nu.ravel())
        zref = matfree.FourierPreconditioner(grid, *c.reference_medium())(r).ravel()
        for x, y, z, rp in FFT_VARIANTS:
            c.schedule = (0, 32, x, y, z, rp)
            zz = c.apply_preconditioner(r.ravel(), precision=prec)
            assert relerr(zz, zref) < tol, (x, y, z, rp)


def test_solve_under_other_schedules(lib):
    """Full FP64 solves under non-default schedules: C* of a 16^3 sphere cell
    within 1e-10 of the oracle's direct solve for each."""
    mask, _, _ = ms.rsa_spheres(16, 0.3, seed=2, rmin=1.0, rmax=2.0)
    E = np.where(mask, 20.0, 1.0)
    nu = np.full(E.shape, 0.3)
    grid = fem.Grid((16, 16, 16))
    Cref, _, _ = fem.effective_stiffness(grid, E, nu)
    for sched in [(1, 8, 1, 1, 1, 1), (2, 16, 0, 1, 0, 1), (0, 64, 1, 0, 1, 0)]:
        with lib.Cell((16, 16, 16), precision=lib.FP64, tol=1e-11) as c:
            c.set_material(E.ravel(), nu.ravel())
            c.schedule = sched
            C, info = c.effective_stiffness()
        assert info["status"] == "CELL_OK"
        assert relerr(C, Cref) < 1e-10, sched


def test_schedule_validation(lib):
    with lib.Cell((16, 16, 16)) as c:
        for bad in [(6, 32, 0, 0, 0, 0), (0, 12, 0, 0, 0, 0), (0, 32, 4, 0, 0, 0), (0, 32, 0, 4, 0, 0),
                    (0, 32, 0, 0, 4, 0), (0, 32, 0, 0, 0, -1), (0, 32, 0, 0, 0, 2)]:
            with pytest.raises(lib.CellError) as e:
                c.schedule = bad
            assert e.value.status == lib.CELL_E_ARG
        assert c.schedule == (0, 32, 0, 0, 0, 0)
        with pytest.raises(lib.CellError) as e:
            c.autotune()  # no material yet
        assert e.value.status == lib.CELL_E_STATE


def test_autotune_and_cache(lib, tmp_path, monkeypatch):
    """The autotuner picks a valid schedule, writes it to the cache, a new
    handle of the same key starts from it, and solves stay correct."""
    path = tmp_path / "tune.json"
    monkeypatch.setenv("CELLFFT_TUNE_CACHE", str(path))
    E, nu, _ = ms.spheres_cell(48, 0.2, seed=8, contrast=30.0, rmin=3.0, rmax=5.0)
    with lib.Cell((48, 48, 48), precision=lib.FP64, tol=1e-10) as c:
        c.set_material(E.ravel(), nu.ravel())
        Cref, _ = c.effective_stiffness()
    with lib.Cell((48, 48, 48), precision=lib.MIXED, tol=1e-7) as c:
        c.set_material(E.ravel(), nu.ravel())
        s1 = c.autotune()
        C1, info = c.effective_stiffness()
    assert s1[0] in range(6) and s1[1] in (8, 16, 32, 64)
    assert relerr(C1, Cref) < 1e-6
    cache = json.loads(path.read_text())
    assert list(cache.values()) == [list(s1)]
    key = next(iter(cache))
    assert "|3d|48x48x48|f32|6" in key
    with lib.Cell((48, 48, 48), precision=lib.MIXED, tol=1e-7) as c:
        assert c.schedule == s1  # from the cache at creation
        c.set_material(E.ravel(), nu.ravel())
        assert c.autotune() == s1  # cached: no re-timing
        C2, _ = c.effective_stiffness()
    assert np.array_equal(C1, C2)
    # batches tune every group
    cells = [c for c in ms.random_cells(3)]
    with lib.Batch([(c["n"],) * 3 for c in cells], precision=lib.MIXED, tol=1e-6) as b:
        for i, c in enumerate(cells):
            b.set_material(i, c["E"].ravel(), c["nu"].ravel())
        b.autotune()
        C, infos = b.effective_stiffness()
    assert all(i["status"] == "CELL_OK" for i in infos)
    assert len(json.loads(path.read_text())) == 1 + len({c["n"] for c in cells})
