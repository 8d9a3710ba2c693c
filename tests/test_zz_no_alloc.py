"""The allocation-free operator entry point against cell_apply_operator:
identical q (same kernel and schedule, bitwise) and u.Ku within 1e-14 of
the sum of the absolute terms from the exactly rounded sum of the products
u_i q_i (math.fsum: the fixed-order FP64 reduction's rounding only), on two
calls in a row through the C ABI, the second on a smaller grid; the
library's scratch keeps the first call's contents, which must not leak into
the second.  Also the size limit and the error paths."""
import math

import numpy as np
import pytest


def _dot_ok(e, u, q):
    t = u * q
    return abs(e - math.fsum(t)) <= 1e-14 * math.fsum(np.abs(t))

pytestmark = pytest.mark.gpu


def _case(lib, shape, seed):
    import torch
    rng = np.random.default_rng(seed)
    n = int(np.prod(shape))
    d = len(shape)
    E = rng.uniform(1.0, 10.0, n)
    nu = rng.uniform(0.1, 0.4, n)
    u = rng.standard_normal(d * n)
    c = lib.Cell(shape, precision=lib.FP64)
    c.set_material(E, nu)
    ref = c.apply_operator(u, precision=lib.FP64)
    ud = torch.tensor(u, dtype=torch.float64, device="cuda")
    qd = torch.full_like(ud, np.nan)
    e = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    return c, u, ref, ud, qd, e


def test_noalloc_matches_apply_operator_twice(lib):
    import torch
    cases = [_case(lib, (64, 32, 24), 1), _case(lib, (16, 12, 8), 2)]
    for c, u, ref, ud, qd, e in cases:  # second call: smaller grid
        c.apply_operator_noalloc(ud, qd, e)
        torch.cuda.synchronize()
        q = qd.cpu().numpy()
        assert np.array_equal(q, ref)
        assert _dot_ok(float(e.item()), u, ref)
    # 2D as well, then the first grid again (the scratch now holds the 2D call's partials)
    c2, u2, ref2, ud2, qd2, e2 = _case(lib, (48, 32), 3)
    c2.apply_operator_noalloc(ud2, qd2, e2)
    c, u, ref, ud, qd, e = cases[0]
    qd.fill_(np.nan)
    c.apply_operator_noalloc(ud, qd, None)
    torch.cuda.synchronize()
    assert np.array_equal(qd2.cpu().numpy(), ref2)
    assert _dot_ok(float(e2.item()), u2, ref2)
    assert np.array_equal(qd.cpu().numpy(), ref)
    for cc in cases + [(c2,)]:
        cc[0].close()


def test_noalloc_errors(lib):
    import torch
    with lib.Cell((16, 16, 16), precision=lib.FP64) as c:
        u = torch.zeros(3 * 4096, dtype=torch.float64, device="cuda")
        q = torch.zeros_like(u)
        with pytest.raises(lib.CellError) as e:
            c.apply_operator_noalloc(u, q)
        assert e.value.status == lib.CELL_E_STATE
        c.set_material(np.full(4096, 2.0), np.full(4096, 0.3))
        c.set_surrogate(2, 3)
        with pytest.raises(lib.CellError) as e:
            c.apply_operator_noalloc(u, q)
        assert e.value.status == lib.CELL_E_UNSUPPORTED
        c.set_surrogate(0)
        c.apply_operator_noalloc(u, q)
        torch.cuda.synchronize()
        assert float(q.abs().max()) == 0.0
