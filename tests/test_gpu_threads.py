"""Handles are independent (the header's threading rule): two handles
driven from two host threads at once (ctypes releases the interpreter lock
during each call, so the library calls overlap; each handle runs on its own
stream and captures its graphs in thread-local mode) give the same results,
bit for bit, as the same solves one after the other.  (The per-thread
last-error message is checked without a GPU in test_abi.py.)"""
import threading

import numpy as np
import pytest

from paper_2004_05197_amd import microstructures as ms

pytestmark = pytest.mark.gpu


def _cells(lib):
    m, _, _ = ms.rsa_spheres(32, 0.25, seed=7, rmin=2.0, rmax=4.0)
    E1 = np.where(m, 50.0, 1.0).ravel()
    rng = np.random.default_rng(8)
    E2 = np.exp(rng.normal(0.0, 1.0, 24 * 16 * 12))
    return [((32, 32, 32), lib.MIXED, 1e-6, E1), ((24, 16, 12), lib.FP64, 1e-10, E2)]


def _solve(lib, shape, prec, tol, E, reps, out, key):
    res = []
    with lib.Cell(shape, precision=prec, tol=tol) as c:
        c.set_material(E, np.full(E.size, 0.3))
        for _ in range(reps):
            C, info = c.effective_stiffness()
            res.append((C.copy(), list(info["iters"]), c.displacement(2).copy()))
    out[key] = res


def test_two_handles_from_two_threads(lib):
    cells = _cells(lib)
    seq = {}
    for k, (shape, prec, tol, E) in enumerate(cells):
        _solve(lib, shape, prec, tol, E, 1, seq, k)
    par = {}
    errors = []

    def run(k):
        try:
            shape, prec, tol, E = cells[k]
            _solve(lib, shape, prec, tol, E, 3, par, k)
        except Exception as e:  # reported below
            errors.append(e)

    ts = [threading.Thread(target=run, args=(k,)) for k in range(len(cells))]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert not errors, errors
    for k in range(len(cells)):
        C0, it0, u0 = seq[k][0]
        for C, it, u in par[k]:
            assert it == it0
            assert np.array_equal(C, C0)
            assert np.array_equal(u, u0)

