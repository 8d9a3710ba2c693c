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


def laminate_neohooke(phases, frac, Fbar):
    """Neo-Hookean laminate with layers normal to x, phases (lambda, mu) with
    volume fractions frac: the exact solution has F_k = F_bar + a_k (x) e_x
    with sum frac_k a_k = 0 (compatibility) and equal tractions P(F_k) e_x
    (equilibrium), a small nonlinear system solved here independently of any
    finite-element code.  Returns (mean first Piola stress, energy density)."""
    from scipy.optimize import fsolve
    from oracle import hyper
    d = Fbar.shape[0]
    K = len(phases)

    def Fk(a):
        out = []
        for k in range(K):
            F = Fbar.copy()
            F[:, 0] += a[k * d:(k + 1) * d]
            out.append(F)
        return out

    def eqs(a):
        Fs = Fk(a)
        t = [hyper.piola(F[None], np.array([l]), np.array([m]))[0][:, 0] for F, (l, m) in zip(Fs, phases)]
        res = [t[k] - t[-1] for k in range(K - 1)]
        res.append(sum(frac[k] * a[k * d:(k + 1) * d] for k in range(K)))
        return np.concatenate(res)

    a = fsolve(eqs, np.zeros(K * d), xtol=1e-14)
    assert np.abs(eqs(a)).max() < 1e-12
    Fs = Fk(a)
    P = sum(f * hyper.piola(F[None], np.array([l]), np.array([m]))[0] for f, F, (l, m) in zip(frac, Fs, phases))
    W = sum(f * hyper.energy_density(F[None], np.array([l]), np.array([m]))[0] for f, F, (l, m) in zip(frac, Fs, phases))
    return P, W
