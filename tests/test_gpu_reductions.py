"""Fixed-order FP64 reductions of the solver against exact summation.

Every norm and dot product of the iteration is a per-block FP64 partial
summed in index order by a one-block finalize kernel (no atomics).  Such a
sum differs from the exactly rounded sum of the same terms (math.fsum on the
host) by at most a few units in the last place times the sum of the absolute
terms.  Checked here on the residual norms of a whole FP64 solve: the
reported ||f - K u|| / ||f|| is sqrt(rr / ff) with both sums reduced on the
device; on the host, rr is summed exactly from the returned residual and ff
from the oracle's load vectors (assembled independently)."""
import math

import numpy as np
import pytest

from oracle import fem

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape", [(16, 12, 8), (24, 16)])
def test_residual_norms_against_exact_sums(lib, shape):
    rng = np.random.default_rng(11)
    n = int(np.prod(shape))
    E = np.exp(rng.normal(0.0, 1.0, n))
    nu = rng.uniform(0.15, 0.4, n)
    d = len(shape)
    with lib.Cell(shape, precision=lib.FP64, tol=1e-7) as c:
        c.set_material(E, nu)
        _, info = c.effective_stiffness()
        res = [c.residual(l).ravel() for l in range(c.nv)]
    f = fem.assemble_rhs(fem.Grid(shape), E, nu, fem.unit_loads(d))
    for l in range(len(res)):
        rr = math.fsum(res[l] * res[l])
        ff = math.fsum(f[l] * f[l])
        rel2 = info["relres"][l] ** 2
        assert abs(rel2 - rr / ff) <= 1e-12 * (rr / ff), (l, rel2, rr / ff)
