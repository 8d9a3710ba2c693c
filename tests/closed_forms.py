"""Closed-form effective stiffness of laminates (Backus averaging).

For layers of whole voxel slabs the exact continuum fluctuation is piecewise
affine along the layer normal with kinks on node planes, so it lies in the
P1 space and the discrete C* equals these averages exactly.
"""
import numpy as np

from oracle import fem


def backus(lam, mu, w, d, normal):
    """Exact effective Voigt stiffness of a laminate with layer weights w."""
    avg = lambda x: float(np.sum(w * x))
    M = lam + 2 * mu
    inv1M = 1.0 / avg(1.0 / M)
    lM = avg(lam / M)
    C = np.zeros((3, 3) if d == 2 else (6, 6))
    pairs = fem.voigt_pairs(d)
    idx = {p: k for k, p in enumerate(pairs)}
    idx.update({(b, a): k for (a, b), k in list(idx.items())})
    tang = [a for a in range(d) if a != normal]
    C[normal, normal] = inv1M
    for t in tang:
        C[t, normal] = C[normal, t] = lM * inv1M
        C[t, t] = avg(4 * mu * (lam + mu) / M) + lM ** 2 * inv1M
        C[idx[(t, normal)], idx[(t, normal)]] = 1.0 / avg(1.0 / mu)
    if d == 3:
        t1, t2 = tang
        C[t1, t2] = C[t2, t1] = avg(2 * mu * lam / M) + lM ** 2 * inv1M
        C[idx[(t1, t2)], idx[(t1, t2)]] = avg(mu)
    return C
