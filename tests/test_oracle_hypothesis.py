"""Randomised sweeps of the CPU oracle's pins (hypothesis, derandomised so
every run draws the same cases): small periodic grids of any shape from 2 to
5 nodes per axis in 2D and 3D, log-uniform Young's moduli over up to four
decades and Poisson ratios from -0.4 to 0.45 per voxel.  For every draw:

  * C* lies between the Reuss and Voigt bounds (Loewner order) and is SPD;
  * the energy form and the mean-stress form agree and are symmetric
    (Hill-Mandel);
  * C* is invariant under a periodic roll of the material and scales with a
    common factor of E;
  * on the smallest grids, half of C*_JJ |Y| equals the total energy of the
    oracle's solution evaluated independently (least-squares simplex
    gradients and the tensor form of W, Sec. 2.2).
"""
import numpy as np
from hypothesis import given, settings, strategies as st

from oracle import fem
from test_oracle_pins import energy_bruteforce, voigt_to_tensor

SETTINGS = dict(max_examples=25, deadline=None, derandomize=True, database=None)


@st.composite
def cells(draw, max_n=5):
    d = draw(st.sampled_from([2, 3]))
    shape = tuple(draw(st.integers(2, max_n)) for _ in range(d))
    seed = draw(st.integers(0, 2**31 - 1))
    decades = draw(st.floats(0.0, 4.0))
    rng = np.random.default_rng(seed)
    grid = fem.Grid(shape)
    E = 10.0 ** rng.uniform(0.0, decades, grid.nshape)
    nu = rng.uniform(-0.4, 0.45, grid.nshape)
    return grid, E, nu


@settings(**SETTINGS)
@given(cells())
def test_bounds_forms_and_invariances(cell):
    grid, E, nu = cell
    C, Cs, u = fem.effective_stiffness(grid, E, nu)
    scale = np.abs(C).max()
    lam, mu = fem.lame(np.ravel(E), np.ravel(nu))
    Ds = [fem.D_voigt(l, m, grid.d) for l, m in zip(lam, mu)]
    voigt = np.mean(Ds, axis=0)
    reuss = np.linalg.inv(np.mean([np.linalg.inv(D) for D in Ds], axis=0))
    assert np.linalg.eigvalsh(voigt - C).min() >= -1e-9 * scale
    assert np.linalg.eigvalsh(C - reuss).min() >= -1e-9 * scale
    assert np.linalg.eigvalsh(C).min() > 0
    assert np.abs(C - C.T).max() <= 1e-12 * scale
    assert np.abs(C - Cs).max() <= 1e-9 * scale
    shift = tuple(1 + a for a in range(grid.d))
    axes = tuple(range(grid.d))
    Cr, _, _ = fem.effective_stiffness(grid, np.roll(E, shift, axes), np.roll(nu, shift, axes))
    assert np.abs(Cr - C).max() <= 1e-9 * scale
    C3, _, _ = fem.effective_stiffness(grid, 3.0 * E, nu)
    assert np.abs(C3 - 3.0 * C).max() <= 1e-9 * scale


@settings(max_examples=8, deadline=None, derandomize=True, database=None)
@given(cells(max_n=3))
def test_energy_against_independent_evaluation(cell):
    grid, E, nu = cell
    C, _, u = fem.effective_stiffness(grid, E, nu)
    loads = fem.unit_loads(grid.d)
    for J in range(grid.nv):
        W = energy_bruteforce(grid, E, nu, u[J], voigt_to_tensor(loads[J], grid.d))
        assert abs(W - 0.5 * C[J, J] * grid.volume) <= 1e-10 * abs(C[J, J])
