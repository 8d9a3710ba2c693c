"""Batches of independent cells and the captured iteration chunks.

- A batch (cells of several grid sizes, each with its own material and
  reference medium) returns, cell by cell, the bits of the single-cell solve:
  the same kernels run on the same data, one slot per (cell, load).
- Replaying the captured HIP graph of a chunk of iterations returns the bits
  of launching the same kernels one by one, solve after solve; for a batch
  the graph holds the chunks of all unfinished groups and is captured again
  when a group finishes.
- The uneven workload (sphere cells of sizes 32..96, contrast 10-100):
  mixed precision within 1e-6 of FP64, bounds, symmetry, and the oracle's
  PCG on a 32^3 cell.
"""
import numpy as np
import pytest

from oracle import fem, matfree
from paper_2004_05197_amd import microstructures as ms

pytestmark = pytest.mark.gpu


def relerr(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


def small_cells():
    """Three 3D cells on two grids, different materials and reference media."""
    out = []
    m, _, _ = ms.rsa_spheres(16, 0.3, seed=4, rmin=1.5, rmax=3.0)
    out.append(((16, 16, 16), np.where(m, 10.0, 1.0), np.full(m.shape, 0.3)))
    rng = np.random.default_rng(11)
    out.append(((16, 16, 16), rng.uniform(1.0, 50.0, (16, 16, 16)), rng.uniform(0.1, 0.4, (16, 16, 16))))
    m, _, _ = ms.rsa_spheres(24, 0.2, seed=5, rmin=2.0, rmax=4.0)
    out.append(((24, 24, 24), np.where(m, 100.0, 1.0), np.full(m.shape, 0.25)))
    return out


@pytest.mark.parametrize("precision", ["FP64", "MIXED"])
def test_batch_equals_single_cells(lib, precision):
    prec = getattr(lib, precision)
    tol = 1e-10 if precision == "FP64" else 1e-6
    cells = small_cells()
    with lib.Batch([c[0] for c in cells], precision=prec, tol=tol) as b:
        assert b.groups == 2
        for i, (_, E, nu) in enumerate(cells):
            b.set_material(i, E.ravel(), nu.ravel())
        Cb, infos = b.effective_stiffness()
        # a second call on the same batch repeats the bits
        Cb2, _ = b.effective_stiffness()
    assert np.array_equal(Cb, Cb2)
    for i, (shape, E, nu) in enumerate(cells):
        with lib.Cell(shape, precision=prec, tol=tol) as c:
            c.set_material(E.ravel(), nu.ravel())
            Cs, info = c.effective_stiffness()
        assert np.array_equal(Cb[i], Cs), (i, relerr(Cb[i], Cs))
        assert infos[i]["iters"] == info["iters"]
        assert infos[i]["relres"] == info["relres"]
        assert infos[i]["status"] == "CELL_OK"
        assert infos[i]["sym_gap"] == info["sym_gap"]


def test_batch_solve_mean_stress_2d(lib):
    """2D cells on two grids (per-cell reference media in the last pass),
    two non-unit macro strains: mean stresses equal the single-cell bits."""
    E0, nu0 = ms.circle2d(32)
    rng = np.random.default_rng(2)
    cells = [((32, 32), E0, nu0),
             ((32, 32), rng.uniform(1.0, 20.0, (32, 32)), np.full((32, 32), 0.2)),
             ((16, 16), rng.uniform(0.5, 2.0, (16, 16)), rng.uniform(0.0, 0.45, (16, 16)))]
    eb = np.array([[1e-2, 0.0, 0.0], [0.3e-2, -0.1e-2, 0.5e-2]])
    with lib.Batch([c[0] for c in cells], precision=lib.FP64, tol=1e-11) as b:
        for i, (_, E, nu) in enumerate(cells):
            b.set_material(i, E.ravel(), nu.ravel())
        S, infos = b.solve(eb)
    for i, (shape, E, nu) in enumerate(cells):
        with lib.Cell(shape, precision=lib.FP64, tol=1e-11) as c:
            c.set_material(E.ravel(), nu.ravel())
            Ss, info = c.solve(eb)
        assert np.array_equal(S[i], Ss), i
        assert infos[i]["iters"] == info["iters"]
    # and the oracle's direct solve of the first cell
    grid = fem.Grid((32, 32))
    u = fem.solve_direct(grid, E0, nu0, eb)
    h = fem.homogenize(grid, E0, nu0, u, eb)
    assert relerr(S[0], h["mean_stress"]) < 1e-9


def test_graph_replay_equals_eager(lib, monkeypatch):
    """The chunk graph is captured at the first chunk of every solve and
    replayed until convergence; three solves in a row, with other device work
    between them, each give the bits of eager launches."""
    shape = (24, 24, 24)
    m, _, _ = ms.rsa_spheres(24, 0.25, seed=9, rmin=2.0, rmax=4.0)
    E = np.where(m, 50.0, 1.0).ravel()
    nu = np.full(E.shape, 0.3)
    res = {}
    for mode in ("0", "1"):
        monkeypatch.setenv("CELLFFT_GRAPHS", mode)
        for prec in (lib.FP64, lib.MIXED):
            with lib.Cell(shape, precision=prec, tol=1e-9 if prec == lib.FP64 else 1e-6) as c:
                c.set_material(E, nu)
                runs = []
                for k in range(3):
                    C, info = c.effective_stiffness()
                    u = c.displacement(k)  # eager work between the solves
                    runs.append((C, info["iters"], u))
                res[(mode, prec)] = runs
    for prec in (lib.FP64, lib.MIXED):
        eager, graph = res[("0", prec)], res[("1", prec)]
        for k in range(3):
            assert np.array_equal(graph[k][0], eager[0][0]), (prec, k)
            assert graph[k][1] == eager[0][1]
            assert np.array_equal(graph[k][2], eager[k][2])


def test_batch_graph_equals_eager(lib, monkeypatch):
    """One captured graph per chunk for the whole batch (every unfinished
    group's iterations, captured again whenever a group finishes: the groups
    here converge after different numbers of chunks) gives the bits of eager
    launches, twice in a row, with eager work between the solves."""
    cells = small_cells()
    m, _, _ = ms.rsa_spheres(12, 0.2, seed=6, rmin=1.5, rmax=2.5)
    cells.append(((12, 12, 12), np.where(m, 1000.0, 1.0), np.full(m.shape, 0.3)))
    res = {}
    for mode in ("0", "1"):
        monkeypatch.setenv("CELLFFT_GRAPHS", mode)
        for prec in (lib.FP64, lib.MIXED):
            with lib.Batch([c[0] for c in cells], precision=prec, tol=1e-9 if prec == lib.FP64 else 1e-6) as b:
                assert b.groups == 3
                for i, (_, E, nu) in enumerate(cells):
                    b.set_material(i, E.ravel(), nu.ravel())
                runs = []
                for _ in range(2):
                    C, infos = b.effective_stiffness()
                    runs.append((C, [inf["iters"] for inf in infos]))
                res[(mode, prec)] = runs
    for prec in (lib.FP64, lib.MIXED):
        eager, graph = res[("0", prec)], res[("1", prec)]
        chunks = {max(it) // 8 for it in eager[0][1]}
        assert len(chunks) > 1, eager[0][1]  # the groups finish in different chunks
        for k in range(2):
            assert np.array_equal(graph[k][0], eager[0][0]), (prec, k)
            assert graph[k][1] == eager[0][1]


def test_batch_rejects_mismatched_configs(lib):
    with pytest.raises(lib.CellError) as e:
        lib.Batch([(16, 16, 16), (16, 16)])
    assert e.value.status == lib.CELL_E_ARG
    with pytest.raises(lib.CellError) as e:
        lib.Batch([(16, 16, 16), (20, 16, 16)])
    assert e.value.status == lib.CELL_E_UNSUPPORTED
    with lib.Batch([(8, 8, 8), (12, 12, 12)]) as b:
        with pytest.raises(lib.CellError) as e:
            b.effective_stiffness()  # no material yet
        assert e.value.status == lib.CELL_E_STATE
        with pytest.raises(lib.CellError) as e:
            b.set_material(-1, np.ones(1728), np.full(1728, 0.3))  # cell index out of range
        assert e.value.status == lib.CELL_E_ARG


def voigt_reuss(E, nu, d):
    """Voigt (mean stiffness) and Reuss (inverse of the mean compliance)
    bounds over the voxels; D is linear in (lambda, mu), and the compliance
    mean runs over the distinct (lambda, mu) phases."""
    lam, mu = fem.lame(np.ravel(E), np.ravel(nu))
    V = fem.D_voigt(lam.mean(), mu.mean(), d)
    ph, cnt = np.unique(lam + 1j * mu, return_counts=True)
    S = sum(k * np.linalg.inv(fem.D_voigt(p.real, p.imag, d)) for p, k in zip(ph, cnt)) / cnt.sum()
    return V, np.linalg.inv(S)


def test_uneven_workload_mixed(lib):
    """Uneven sphere cells (seeds 1000..1011, sizes from {32,48,64,96}, vf
    0.1-0.4, contrast 10-100), 6 unit loads each, mixed precision tol 1e-6,
    batched: every C* within 1e-6 of the FP64 GPU solve, inside the
    Voigt/Reuss bounds, symmetric mean-stress form; a 32^3 cell against the
    oracle's matrix-free PCG."""
    cells = list(ms.random_cells(12))
    assert len({c["n"] for c in cells}) >= 3
    with lib.Batch([(c["n"],) * 3 for c in cells], precision=lib.MIXED, tol=1e-6) as b:
        for i, c in enumerate(cells):
            b.set_material(i, c["E"].ravel(), c["nu"].ravel())
        C, infos = b.effective_stiffness()
    for i, c in enumerate(cells):
        assert infos[i]["status"] == "CELL_OK"
        assert max(infos[i]["relres"]) <= 1e-6
        assert infos[i]["sym_gap"] < 1e-5
        with lib.Cell((c["n"],) * 3, precision=lib.FP64, tol=1e-10) as s:
            s.set_material(c["E"].ravel(), c["nu"].ravel())
            C64, _ = s.effective_stiffness()
        assert relerr(C[i], C64) < 1e-6, (i, c["n"], relerr(C[i], C64))
        V, R = voigt_reuss(c["E"], c["nu"], 3)
        sc = np.abs(C64).max()
        assert np.linalg.eigvalsh(V - C[i]).min() >= -1e-8 * sc
        assert np.linalg.eigvalsh(C[i] - R).min() >= -1e-8 * sc
    k = next(i for i, c in enumerate(cells) if c["n"] == 32)
    grid = fem.Grid((32, 32, 32))
    eb = np.stack([np.eye(6)[0], np.eye(6)[3]])
    U = []
    for J in range(2):
        u, it, rel = matfree.pcg(grid, cells[k]["E"], cells[k]["nu"], eb[J], tol=1e-10)
        U.append(u)
    h = matfree.homogenize(grid, cells[k]["E"], cells[k]["nu"], np.stack(U), eb)
    sub = C[k][np.ix_([0, 3], [0, 3])]
    assert relerr(sub, h["C_energy"]) < 1e-6


def test_profiled_solve_equals_graph_solve(lib):
    """Per-launch event timing launches the iteration kernels one by one
    (events inside a captured graph carry no timestamps): the profiled solve
    gives the bits of the graph-replayed one, and every chunk is counted."""
    E, nu, _ = ms.spheres_cell(32, 0.2, seed=3, contrast=20.0, rmin=2.0, rmax=4.0)
    with lib.Cell((32, 32, 32), precision=lib.MIXED, tol=1e-6) as c:
        c.set_material(E.ravel(), nu.ravel())
        Cg, ig = c.effective_stiffness()
        c.profile(True)
        Cp, ip = c.effective_stiffness()
        prof = c.profile_read()
        c.profile(False)
    assert np.array_equal(Cg, Cp)
    assert ig["iters"] == ip["iters"]
    n_apply = prof["k_apply"][1]
    assert n_apply % 8 == 0 and n_apply >= max(ip["iters"])
    for k in ("y_fwd", "last", "y_inv", "x_inv"):
        assert prof[k][1] == n_apply + 1, k  # plus the initial preconditioning
    assert prof["residual"][1] >= 2  # the load vectors, then at least one refresh
    # the x-transformed residual is rebuilt after every residual recomputation
    assert prof["x_fwd"][1] == n_apply + prof["residual"][1]
    assert all(v[0] > 0 for k, v in prof.items() if v[1] > 0)
