"""Cases run by tests/test_gpu_bounds_checked.py in a child process against
one build of the library (CELLFFT_LIBRARY selects it): solves and operator
applications through every kernel family, each followed by the bounds
counter of that build.  Prints one JSON object: per case its results and
the counter (-1 for the normal build, which checks nothing).

Not a test module itself (no test_ prefix); run as
`python tests/checked_cases.py`.
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2004_05197_amd import binding as B  # noqa: E402
from paper_2004_05197_amd import microstructures as ms  # noqa: E402


def field(shape, seed):
    rng = np.random.default_rng(seed)
    E = np.exp(rng.normal(0.0, 1.0, shape[::-1])).ravel()
    nu = rng.uniform(0.2, 0.35, E.size)
    return E, nu


def main():
    out = {}
    B.bounds_violations()  # clear

    def record(name, **res):
        res["viol"] = B.bounds_violations()
        out[name] = {k: (np.asarray(v).tolist() if not isinstance(v, (int, float, str)) else v)
                     for k, v in res.items()}
        print(f"[checked] {name}: {res['viol']}", file=sys.stderr, flush=True)

    # 3D effective stiffness, both precisions, ragged non-cubic grid
    shape = (24, 16, 12)
    E, nu = field(shape, 1)
    for prec in (B.FP64, B.MIXED):
        with B.Cell(shape, precision=prec, tol=1e-9 if prec == B.FP64 else 1e-6) as c:
            c.set_material(E, nu)
            C, info = c.effective_stiffness()
            g = c.adjoint(np.eye(6))
        record(f"stiffness3d_p{prec}", C=C, iters=info["iters"], grad=g[:64])
    # every FP32 stencil tile and x/y/z pass variant on a grid the row-wave tile takes
    shape = (64, 16, 16)
    E, nu = field(shape, 2)
    u = np.random.default_rng(3).normal(size=3 * 64 * 16 * 16)
    for tile in range(6):
        with B.Cell(shape, precision=B.MIXED, tol=1e-6) as c:
            c.set_material(E, nu)
            c.schedule = (tile, 8 if tile < 5 else 16, tile % 4, (tile + 1) % 4, tile % 4, tile % 2)
            q = c.apply_operator(u)
            z = c.apply_preconditioner(u)
            C, info = c.effective_stiffness()
        record(f"tile{tile}", q=q[:256], z=z[:256], C=C, iters=info["iters"])
    # FP64 tiles
    for tile in range(5):
        with B.Cell(shape, precision=B.FP64, tol=1e-9) as c:
            c.set_material(E, nu)
            c.schedule = (tile, 16, tile % 4, (tile + 3) % 4, tile % 4, (tile + 1) % 2)
            q = c.apply_operator(u)
        record(f"tile{tile}_fp64", q=q[:256])
    # 2D
    shape = (32, 48)
    E, nu = field(shape, 4)
    with B.Cell(shape, precision=B.MIXED, tol=1e-6) as c:
        c.set_material(E, nu)
        C, info = c.effective_stiffness()
    record("stiffness2d", C=C, iters=info["iters"])
    # batch of uneven cells
    shapes = [(16, 16, 16), (24, 24, 24), (16, 16, 16), (32, 32, 32)]
    with B.Batch(shapes, precision=B.MIXED, tol=1e-6) as b:
        for i, sh in enumerate(shapes):
            m, _, _ = ms.rsa_spheres(sh[0], 0.25, seed=10 + i, rmin=1.0, rmax=3.0)
            b.set_material(i, np.where(m, 30.0, 1.0).ravel(), np.full(m.size, 0.3))
        C, infos = b.effective_stiffness()
    record("batch", C=C)
    # neo-Hookean Newton-PCG
    shape = (12, 12, 12)
    E, nu = field(shape, 5)
    with B.Cell(shape, precision=B.FP64, tol=1e-9) as c:
        c.set_material(E, nu)
        F = np.eye(3) + 0.02 * np.array([[1.0, 0.3, 0.0], [0.0, -0.5, 0.2], [0.1, 0.0, 0.4]])
        P, info = c.solve_hyper(F[None])
    record("hyper", P=P)
    # surrogate operator (a smooth field: the surrogate interpolates the
    # stencil between sample nodes)
    shape = (16, 16, 16)
    g = ms.gaussian_random_field(shape, 4.0, 6)
    with B.Cell(shape, precision=B.MIXED, tol=1e-6) as c:
        c.set_material(np.exp(0.5 * g).ravel(), np.full(g.size, 0.3))
        c.set_surrogate(2, 3)
        C, info = c.effective_stiffness()
    record("surrogate", C=C)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
