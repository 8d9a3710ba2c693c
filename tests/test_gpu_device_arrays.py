"""The C ABI's device-array paths (on_device = 1) against its host-array
paths on the same cell: material set from device tensors, the displacement,
residual and gradient written to device memory, an initial guess read from
device memory, and a batch's material from device tensors.  Same kernels on
the same data, so the results are compared bit for bit."""
import ctypes as ct

import numpy as np
import pytest

from paper_2004_05197_amd import microstructures as ms

pytestmark = pytest.mark.gpu


def cell_material():
    mask, _, _ = ms.rsa_spheres(16, 0.25, seed=8, rmin=1.5, rmax=3.0)
    E = np.where(mask, 30.0, 1.0)
    nu = np.where(mask, 0.2, 0.35)
    return E.ravel(), nu.ravel()


@pytest.mark.parametrize("prec", ["FP64", "MIXED"])
def test_device_arrays_equal_host_arrays(lib, prec):
    import torch
    p = getattr(lib, prec)
    E, nu = cell_material()
    dJ = np.zeros((6, 6))
    dJ[0, 0] = dJ[3, 3] = 1.0
    res = {}
    for mode in ("host", "device"):
        with lib.Cell((16, 16, 16), precision=p, tol=1e-9 if prec == "FP64" else 1e-6) as c:
            if mode == "host":
                c.set_material(E, nu)
            else:
                c.set_material(torch.tensor(E, device="cuda"), torch.tensor(nu, device="cuda"))
            C, info = c.effective_stiffness()
            n3 = 3 * c.n
            if mode == "host":
                u = c.displacement(2)
                r = c.residual(2)
                g = c.adjoint(dJ)
            else:
                ud = torch.full((n3,), np.nan, dtype=torch.float64, device="cuda")
                rd = torch.full((n3,), np.nan, dtype=torch.float64, device="cuda")
                assert lib._lib.cell_get_displacement(c._h, 2, ct.c_void_p(ud.data_ptr()), 1) == 0
                assert lib._lib.cell_get_residual(c._h, 2, ct.c_void_p(rd.data_ptr()), 1) == 0
                gd = torch.full((c.n,), np.nan, dtype=torch.float64, device="cuda")
                c.adjoint(dJ, out=gd)
                torch.cuda.synchronize()
                u, r, g = ud.cpu().numpy(), rd.cpu().numpy(), gd.cpu().numpy()
            # a warm-started solve from the solution just found (device or host guess)
            u0 = c.displacement(0)
            c.set_initial_guess(0, torch.tensor(u0.ravel(), device="cuda") if mode == "device" else u0.ravel())
            S, info2 = c.solve(np.eye(6)[:1])
            res[mode] = (C, info["iters"], np.ravel(u), np.ravel(r), np.ravel(g), S, info2["iters"])
    h, d = res["host"], res["device"]
    for k in (0, 2, 3, 4, 5):
        assert np.array_equal(h[k], d[k]), k
    assert h[1] == d[1] and h[6] == d[6]
    assert h[6][0] <= 1  # the guess is the solution already


def test_batch_device_material(lib):
    import torch
    E, nu = cell_material()
    rng = np.random.default_rng(3)
    E2 = rng.uniform(1.0, 20.0, 12 ** 3)
    nu2 = rng.uniform(0.1, 0.4, 12 ** 3)
    res = {}
    for mode in ("host", "device"):
        with lib.Batch([(16, 16, 16), (12, 12, 12)], precision=lib.FP64, tol=1e-9) as b:
            for i, (e, v) in enumerate(((E, nu), (E2, nu2))):
                if mode == "host":
                    b.set_material(i, e, v)
                else:
                    b.set_material(i, torch.tensor(e, device="cuda"), torch.tensor(v, device="cuda"))
            res[mode] = b.effective_stiffness()[0]
    assert np.array_equal(res["host"], res["device"])


@pytest.mark.parametrize("device", [False, True])
def test_rejected_material_keeps_the_previous_one(lib, device):
    # the device-side check reports the first invalid voxel (E before nu at
    # one voxel) and writes nothing; the next solve uses the earlier material
    import torch
    E, nu = cell_material()
    wrap = (lambda a: torch.tensor(a, device="cuda")) if device else (lambda a: a)
    with lib.Cell((16, 16, 16), precision=lib.FP64, tol=1e-10) as c:
        c.set_material(wrap(E), wrap(nu))
        C0, _ = c.effective_stiffness()
        bad_E, bad_nu = E.copy(), nu.copy()
        bad_E[1234] = np.nan
        bad_nu[1234] = 0.7
        bad_nu[99] = -1.0
        with pytest.raises(lib.CellError) as ei:
            c.set_material(wrap(bad_E), wrap(nu))
        assert ei.value.status == lib.CELL_E_NONFINITE and "voxel 1234" in lib.last_error()
        with pytest.raises(lib.CellError) as ei:
            c.set_material(wrap(bad_E), wrap(bad_nu))
        assert ei.value.status == lib.CELL_E_ARG and "voxel 99" in lib.last_error()
        with pytest.raises(lib.CellError) as ei:
            c.set_material(wrap(E * 0.0), wrap(nu))
        assert ei.value.status == lib.CELL_E_NONFINITE and "voxel 0" in lib.last_error()
        C1, _ = c.effective_stiffness()
    assert np.array_equal(C0, C1)
