"""The oracle reproduces the stored values under tests/golden/ (written by
tests/golden/make_golden.py, which calls only the oracle): a change of the
oracle's arithmetic shows up here.  The stored values are the oracle's own,
not the paper's (it prints none for this problem); what pins them to the
mathematics is tests/test_oracle_pins.py."""
import json
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

import make_golden  # noqa: E402


def load(name):
    with open(os.path.join(HERE, "golden", name + ".json")) as fh:
        return json.load(fh)


@pytest.mark.parametrize("name", sorted(make_golden.CASES))
def test_oracle_reproduces_golden(name):
    stored = load(name)
    fresh = make_golden.CASES[name]()
    for key in ("C_energy", "mean_stress"):
        if key in stored:
            a, b = np.asarray(fresh[key]), np.asarray(stored[key])
            assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max(), (name, key)


def test_golden_structure():
    c = np.asarray(load("circle2d_32")["C_energy"])
    # symmetric, positive definite; the centred circle is symmetric under
    # x <-> y (C1111 = C2222)
    assert np.allclose(c, c.T, rtol=0, atol=1e-12 * np.abs(c).max())
    assert np.all(np.linalg.eigvalsh(0.5 * (c + c.T)) > 0)
    assert abs(c[0, 0] - c[1, 1]) < 1e-12 * c[0, 0]
    s = np.asarray(load("circle2d_32")["mean_stress"])
    assert np.allclose(s, 1e-2 * c[:, 0], rtol=1e-9)  # mean stress = C* eps at the discrete solution
