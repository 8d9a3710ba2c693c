"""ctypes binding of the HIP C-ABI library ``libcellfft.so``.

Argument marshalling only: every step of the solve runs in the library's
HIP kernels.  Arrays may be numpy arrays (host) or torch tensors; CUDA
(HIP) torch tensors are passed as device pointers (``on_device = 1``) and
the library runs on the stream given at construction (default: its own).

Importing this module loads the library and raises ``ImportError`` if it
has not been built (``python -m paper_2004_05197_amd.build``); there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# CELLFFT_LIBRARY selects another build of the same library (the host-
# sanitized one of the ABI tests, the bounds-checked one of the debug
# tests); the default is the in-tree build
LIB_PATH = os.environ.get("CELLFFT_LIBRARY") or os.path.join(_HERE, "libcellfft.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2004_05197_amd.build`")

# torch bundles its own HIP and HSA runtimes under the same sonames as the
# system ones this library links.  Loaded after torch, the library binds to
# torch's copies (one runtime in the process, so torch's device pointers and
# streams are the library's too); loaded first, it pulls in the system copies
# and torch, loading its own beside them, then finds no GPU.  So torch is
# imported before the library is loaded.
try:
    import torch as _torch  # noqa: F401
except ImportError:  # plain ctypes use without torch: one runtime only
    _torch = None

_lib = ct.CDLL(LIB_PATH)

CELL_OK = 0
CELL_NOT_CONVERGED = 1
CELL_E_ARG = -1
CELL_E_NOMEM = -2
CELL_E_DEVICE = -3
CELL_E_STATE = -4
CELL_E_NONFINITE = -5
CELL_E_BREAKDOWN = -6
CELL_E_UNSUPPORTED = -7
FP64 = 0
MIXED = 1

STATUS_NAMES = {0: "CELL_OK", 1: "CELL_NOT_CONVERGED", -1: "CELL_E_ARG", -2: "CELL_E_NOMEM",
                -3: "CELL_E_DEVICE", -4: "CELL_E_STATE", -5: "CELL_E_NONFINITE",
                -6: "CELL_E_BREAKDOWN", -7: "CELL_E_UNSUPPORTED"}


class CellConfig(ct.Structure):
    _fields_ = [("dim", ct.c_int), ("n", ct.c_int * 3), ("len", ct.c_double * 3),
                ("precision", ct.c_int), ("tol", ct.c_double), ("max_iter", ct.c_int),
                ("max_loads", ct.c_int), ("stream", ct.c_void_p), ("device", ct.c_int)]


class CellInfo(ct.Structure):
    _fields_ = [("nload", ct.c_int), ("iters", ct.c_int * 6), ("refinements", ct.c_int * 6),
                ("relres", ct.c_double * 6), ("hill_mandel_gap", ct.c_double),
                ("sym_gap", ct.c_double), ("seconds", ct.c_double)]

    def as_dict(self):
        k = self.nload
        return dict(nload=k, iters=list(self.iters[:k]), refinements=list(self.refinements[:k]),
                    relres=list(self.relres[:k]), hill_mandel_gap=self.hill_mandel_gap,
                    sym_gap=self.sym_gap, seconds=self.seconds)


class CellHyperInfo(ct.Structure):
    _fields_ = [("nload", ct.c_int), ("newton_iters", ct.c_int * 6), ("cg_iters", ct.c_int * 6),
                ("resnorm", ct.c_double * 6), ("energy", ct.c_double * 6), ("indefinite_steps", ct.c_int * 6),
                ("seconds", ct.c_double)]

    def as_dict(self):
        k = self.nload
        return dict(nload=k, newton_iters=list(self.newton_iters[:k]), cg_iters=list(self.cg_iters[:k]),
                    resnorm=list(self.resnorm[:k]), energy=list(self.energy[:k]),
                    indefinite_steps=list(self.indefinite_steps[:k]), seconds=self.seconds)


_P = ct.c_void_p
_D = ct.POINTER(ct.c_double)
_SIGS = {
    "cell_create": (ct.c_int, [ct.POINTER(CellConfig), ct.POINTER(_P)]),
    "cell_set_material": (ct.c_int, [_P, _P, _P, ct.c_int]),
    "cell_solve": (ct.c_int, [_P, ct.c_int, _P, _P, ct.POINTER(CellInfo)]),
    "cell_effective_stiffness": (ct.c_int, [_P, _P, ct.POINTER(CellInfo)]),
    "cell_adjoint": (ct.c_int, [_P, _P, _P, ct.c_int]),
    "cell_get_displacement": (ct.c_int, [_P, ct.c_int, _P, ct.c_int]),
    "cell_destroy": (None, [_P]),
    "cell_last_error": (ct.c_char_p, []),
    "cell_debug_bounds_violations": (ct.c_int, []),
    "cell_apply_operator": (ct.c_int, [_P, ct.c_int, _P, _P]),
    "cell_apply_preconditioner": (ct.c_int, [_P, ct.c_int, _P, _P]),
    "cell_reference_medium": (ct.c_int, [_P, _D, _D]),
    "cell_energy_matrix": (ct.c_int, [_P, _P]),
    "cell_get_residual": (ct.c_int, [_P, ct.c_int, _P, ct.c_int]),
    "cell_get_residual_history": (ct.c_int, [_P, ct.c_int, _P, ct.c_int, ct.POINTER(ct.c_int)]),
    "cell_profile": (ct.c_int, [_P, ct.c_int]),
    "cell_profile_read": (ct.c_int, [_P, _P, _P]),
    "cell_batch_create": (ct.c_int, [ct.POINTER(CellConfig), ct.c_int, ct.POINTER(_P)]),
    "cell_batch_set_material": (ct.c_int, [_P, ct.c_int, _P, _P, ct.c_int]),
    "cell_batch_solve": (ct.c_int, [_P, ct.c_int, _P, _P, _P]),
    "cell_batch_effective_stiffness": (ct.c_int, [_P, _P, _P]),
    "cell_batch_profile": (ct.c_int, [_P, ct.c_int]),
    "cell_batch_profile_read": (ct.c_int, [_P, _P, _P]),
    "cell_batch_groups": (ct.c_int, [_P]),
    "cell_batch_destroy": (None, [_P]),
    "cell_batch_autotune": (ct.c_int, [_P, ct.c_int]),
    "cell_batch_get_displacement": (ct.c_int, [_P, ct.c_int, ct.c_int, _P, ct.c_int]),
    "cell_batch_get_residual": (ct.c_int, [_P, ct.c_int, ct.c_int, _P, ct.c_int]),
    "cell_autotune": (ct.c_int, [_P, ct.c_int]),
    "cell_solve_hyper": (ct.c_int, [_P, ct.c_int, _P, ct.c_double, ct.c_int, _P, ct.POINTER(CellHyperInfo)]),
    "cell_apply_hyper_tangent": (ct.c_int, [_P, ct.c_int, _P, _P, _P, _P]),
    "cell_set_surrogate": (ct.c_int, [_P, ct.c_int, ct.c_int, _P]),
    "cell_get_surrogate_stencil": (ct.c_int, [_P, _P]),
    "cell_hyper_residual": (ct.c_int, [_P, _P, _P, _P, _P]),
    "cell_get_schedule": (ct.c_int, [_P, _P]),
    "cell_set_schedule": (ct.c_int, [_P, _P]),
    "cell_apply_operator_noalloc": (ct.c_int, [_P, _P, _P, _P]),
    "cell_set_initial_guess": (ct.c_int, [_P, ct.c_int, _P, ct.c_int]),
    "cell_solve_projection": (ct.c_int, [_P, ct.c_int, _P, _P, ct.POINTER(CellInfo)]),
}

KERNEL_KINDS = ["k_apply", "x_fwd", "y_fwd", "last", "y_inv", "x_inv", "residual", "merge", "homog"]
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class CellError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def last_error():
    return _lib.cell_last_error().decode()


def bounds_violations():
    """Out-of-range kernel accesses counted by the bounds-checked build since
    the last call (clears the counters); -1 for the normal build."""
    return int(_lib.cell_debug_bounds_violations())


def _check(status):
    if status < 0:
        raise CellError(status, last_error())
    return status


def _is_torch(x):
    try:
        import torch
        return isinstance(x, torch.Tensor)
    except ImportError:
        return False


def _in_ptr(x, count):
    """(pointer, on_device, keepalive) for a float64 input of `count` values."""
    if _is_torch(x):
        if x.dtype != __import__("torch").float64 or x.numel() != count:
            raise ValueError("expected a float64 tensor with %d values" % count)
        x = x.contiguous()
        if x.is_cuda:
            return ct.c_void_p(x.data_ptr()), 1, x
        a = x.numpy()
    else:
        a = np.ascontiguousarray(np.asarray(x, dtype=np.float64)).ravel()
        if a.size != count:
            raise ValueError("expected %d values, got %d" % (count, a.size))
    return a.ctypes.data_as(ct.c_void_p), 0, a


def _config(shape, precision, tol, max_iter, max_loads, lengths, stream, device):
    shape = tuple(int(s) for s in shape)
    dim = len(shape)
    cfg = CellConfig()
    cfg.dim = dim
    for a in range(3):
        cfg.n[a] = shape[a] if a < dim else 1
        cfg.len[a] = (lengths[a] if lengths is not None and a < dim else 0.0)
    cfg.precision = int(precision)
    cfg.tol = float(tol)
    cfg.max_iter = int(max_iter)
    cfg.max_loads = int(max_loads)
    cfg.stream = None if stream is None else ct.c_void_p(getattr(stream, "cuda_stream", stream))
    cfg.device = int(device)
    return cfg


class Cell:
    """One periodic cell grid on the GPU (wraps a ``cell_t`` handle)."""

    def __init__(self, shape, precision=FP64, tol=0.0, max_iter=0, max_loads=0,
                 lengths=None, stream=None, device=-1):
        shape = tuple(int(s) for s in shape)
        self.dim = len(shape)
        cfg = _config(shape, precision, tol, max_iter, max_loads, lengths, stream, device)
        h = ct.c_void_p()
        _check(_lib.cell_create(ct.byref(cfg), ct.byref(h)))
        self._h = h
        self.shape = shape
        self.n = int(np.prod(shape))
        self.nv = 3 if self.dim == 2 else 6
        self.precision = int(precision)
        self.solves = 0  # incremented by every solve (autograd consistency check)

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.cell_destroy(self._h)
        self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- solver calls ---------------------------------------------------------
    def set_material(self, E, nu):
        pe, de, ke = _in_ptr(E, self.n)
        pn, dn, kn = _in_ptr(nu, self.n)
        if de != dn:
            raise ValueError("E and nu must both be on the host or both on the device")
        _check(_lib.cell_set_material(self._h, pe, pn, de))

    def solve(self, macro_strains):
        eb = np.ascontiguousarray(np.atleast_2d(np.asarray(macro_strains, dtype=np.float64)))
        nl = eb.shape[0]
        out = np.zeros((nl, self.nv))
        info = CellInfo()
        st = _check(_lib.cell_solve(self._h, nl, eb.ctypes.data_as(ct.c_void_p),
                                    out.ctypes.data_as(ct.c_void_p), ct.byref(info)))
        self.solves += 1
        return out, dict(info.as_dict(), status=STATUS_NAMES[st])

    def solve_projection(self, macro_strains):
        """The strain-based projection variant (3D, FP64): mean stresses
        (nload, 6) and info (iterations, relative residuals)."""
        eb = np.ascontiguousarray(np.atleast_2d(np.asarray(macro_strains, dtype=np.float64)))
        nl = eb.shape[0]
        out = np.zeros((nl, self.nv))
        info = CellInfo()
        st = _check(_lib.cell_solve_projection(self._h, nl, eb.ctypes.data_as(ct.c_void_p),
                                               out.ctypes.data_as(ct.c_void_p), ct.byref(info)))
        return out, dict(info.as_dict(), status=STATUS_NAMES[st])

    def effective_stiffness(self):
        C = np.zeros((self.nv, self.nv))
        info = CellInfo()
        st = _check(_lib.cell_effective_stiffness(self._h, C.ctypes.data_as(ct.c_void_p), ct.byref(info)))
        self.solves += 1
        return C, dict(info.as_dict(), status=STATUS_NAMES[st])

    def adjoint(self, dJ_dC, out=None):
        a = np.ascontiguousarray(np.asarray(dJ_dC, dtype=np.float64).reshape(self.nv, self.nv))
        if out is not None and _is_torch(out) and out.is_cuda:
            _check(_lib.cell_adjoint(self._h, a.ctypes.data_as(ct.c_void_p), ct.c_void_p(out.data_ptr()), 1))
            return out
        g = np.zeros(self.n)
        _check(_lib.cell_adjoint(self._h, a.ctypes.data_as(ct.c_void_p), g.ctypes.data_as(ct.c_void_p), 0))
        return g

    def solve_hyper(self, F_bar, tol=0.0, max_newton=0):
        """Neo-Hookean cell problem for macroscopic deformation gradients
        F_bar (nload, d, d); returns (mean first Piola stress (nload, d, d), info)."""
        Fb = np.ascontiguousarray(np.asarray(F_bar, dtype=np.float64).reshape(-1, self.dim, self.dim))
        nl = Fb.shape[0]
        P = np.zeros((nl, self.dim, self.dim))
        info = CellHyperInfo()
        st = _check(_lib.cell_solve_hyper(self._h, nl, Fb.ctypes.data_as(ct.c_void_p), float(tol), int(max_newton),
                                          P.ctypes.data_as(ct.c_void_p), ct.byref(info)))
        self.solves += 1
        return P, dict(info.as_dict(), status=STATUS_NAMES[st])

    def hyper_tangent(self, F_bar, u, p, precision=None):
        Fb = np.ascontiguousarray(np.asarray(F_bar, dtype=np.float64).reshape(self.dim, self.dim))
        u = np.ascontiguousarray(np.asarray(u, dtype=np.float64)).ravel()
        p = np.ascontiguousarray(np.asarray(p, dtype=np.float64)).ravel()
        q = np.zeros_like(u)
        pr = self.precision if precision is None else precision
        _check(_lib.cell_apply_hyper_tangent(self._h, int(pr), Fb.ctypes.data_as(ct.c_void_p), u.ctypes.data_as(ct.c_void_p),
                                             p.ctypes.data_as(ct.c_void_p), q.ctypes.data_as(ct.c_void_p)))
        return q

    def set_surrogate(self, M, q=3):
        """Surrogate stencil operator for later solves (M = 0: off); returns
        the setup time in seconds."""
        t = ct.c_double(0.0)
        _check(_lib.cell_set_surrogate(self._h, int(M), int(q), ct.byref(t)))
        return t.value

    def surrogate_stencil(self):
        """The interpolated stencil blocks (7, 3, 3, n) (FP64)."""
        out = np.zeros((7, 3, 3, self.n))
        _check(_lib.cell_get_surrogate_stencil(self._h, out.ctypes.data_as(ct.c_void_p)))
        return out

    def hyper_residual(self, F_bar, u):
        Fb = np.ascontiguousarray(np.asarray(F_bar, dtype=np.float64).reshape(self.dim, self.dim))
        u = np.ascontiguousarray(np.asarray(u, dtype=np.float64)).ravel()
        f = np.zeros_like(u)
        sums = np.zeros(10)
        _check(_lib.cell_hyper_residual(self._h, Fb.ctypes.data_as(ct.c_void_p), u.ctypes.data_as(ct.c_void_p),
                                        f.ctypes.data_as(ct.c_void_p), sums.ctypes.data_as(ct.c_void_p)))
        return f, sums

    def set_initial_guess(self, load, u0=None):
        """Initial guess [d][n] (numpy, or a float64 torch tensor on the host
        or the device) of load case `load` for later linear solves; None
        clears it."""
        if u0 is None:
            _check(_lib.cell_set_initial_guess(self._h, int(load), None, 0))
            return
        p, dev, keep = _in_ptr(u0, self.dim * self.n)
        _check(_lib.cell_set_initial_guess(self._h, int(load), p, dev))

    def displacement(self, load=0):
        u = np.zeros((self.dim, self.n))
        _check(_lib.cell_get_displacement(self._h, int(load), u.ctypes.data_as(ct.c_void_p), 0))
        return u

    def energy_matrix(self, nload):
        C = np.zeros((nload, nload))
        _check(_lib.cell_energy_matrix(self._h, C.ctypes.data_as(ct.c_void_p)))
        return C

    def residual(self, load=0):
        r = np.zeros((self.dim, self.n))
        _check(_lib.cell_get_residual(self._h, int(load), r.ctypes.data_as(ct.c_void_p), 0))
        return r

    def residual_history(self, load=0):
        """||r_k|| / ||f|| after k = 0, 1, ... iterations of the last linear
        solve of load `load`."""
        cnt = ct.c_int(0)
        _check(_lib.cell_get_residual_history(self._h, int(load), None, 0, ct.byref(cnt)))
        h = np.zeros(cnt.value)
        _check(_lib.cell_get_residual_history(self._h, int(load), h.ctypes.data_as(ct.c_void_p), cnt.value,
                                               ct.byref(cnt)))
        return h

    def apply_operator(self, u, precision=None):
        u = np.ascontiguousarray(np.asarray(u, dtype=np.float64)).ravel()
        q = np.zeros_like(u)
        p = self.precision if precision is None else precision
        _check(_lib.cell_apply_operator(self._h, int(p), u.ctypes.data_as(ct.c_void_p),
                                        q.ctypes.data_as(ct.c_void_p)))
        return q

    def apply_operator_noalloc(self, u, q, uKu=None):
        """q = K u (FP64) on device tensors without any allocation by the
        library (float64 CUDA tensors of d n values; uKu: optional float64
        CUDA tensor of one value).  Asynchronous on the handle's stream."""
        import torch
        for t in (u, q) + (() if uKu is None else (uKu,)):
            if not (_is_torch(t) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
                raise ValueError("expected contiguous float64 CUDA tensors")
        if u.numel() != self.dim * self.n or q.numel() != self.dim * self.n or (uKu is not None and uKu.numel() != 1):
            raise ValueError("u and q need d n values, uKu one")
        _check(_lib.cell_apply_operator_noalloc(self._h, ct.c_void_p(u.data_ptr()), ct.c_void_p(q.data_ptr()),
                                                None if uKu is None else ct.c_void_p(uKu.data_ptr())))
        return q

    def apply_preconditioner(self, r, precision=None):
        r = np.ascontiguousarray(np.asarray(r, dtype=np.float64)).ravel()
        z = np.zeros_like(r)
        p = self.precision if precision is None else precision
        _check(_lib.cell_apply_preconditioner(self._h, int(p), r.ctypes.data_as(ct.c_void_p),
                                              z.ctypes.data_as(ct.c_void_p)))
        return z

    def profile(self, enable=True):
        _check(_lib.cell_profile(self._h, int(bool(enable))))

    def profile_read(self):
        ms = np.zeros(len(KERNEL_KINDS))
        cnt = np.zeros(len(KERNEL_KINDS), dtype=np.int64)
        _check(_lib.cell_profile_read(self._h, ms.ctypes.data_as(ct.c_void_p), cnt.ctypes.data_as(ct.c_void_p)))
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(KERNEL_KINDS)}

    def autotune(self, force=False):
        _check(_lib.cell_autotune(self._h, int(bool(force))))
        return self.schedule

    @property
    def schedule(self):
        v = (ct.c_int * 6)()
        _check(_lib.cell_get_schedule(self._h, v))
        return tuple(v)

    @schedule.setter
    def schedule(self, sched):
        v = (ct.c_int * 6)(*[int(x) for x in sched])
        _check(_lib.cell_set_schedule(self._h, v))

    def reference_medium(self):
        lam = ct.c_double()
        mu = ct.c_double()
        _check(_lib.cell_reference_medium(self._h, ct.byref(lam), ct.byref(mu)))
        return lam.value, mu.value


class Batch:
    """Independent cells, possibly of different grid sizes, solved together
    (wraps a ``cell_batch_t`` handle): cells of one grid share every kernel
    launch, and the grids advance in lockstep on one stream."""

    def __init__(self, shapes, precision=FP64, tol=0.0, max_iter=0, max_loads=0,
                 stream=None, device=-1):
        shapes = [tuple(int(s) for s in sh) for sh in shapes]
        if not shapes:
            raise ValueError("a batch needs at least one cell")
        self.dim = len(shapes[0])
        cfgs = (CellConfig * len(shapes))()
        for i, sh in enumerate(shapes):
            cfgs[i] = _config(sh, precision, tol, max_iter, max_loads, None, stream, device)
        h = ct.c_void_p()
        _check(_lib.cell_batch_create(cfgs, len(shapes), ct.byref(h)))
        self._h = h
        self.shapes = shapes
        self.ncell = len(shapes)
        self.nv = 3 if self.dim == 2 else 6

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.cell_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def groups(self):
        return _lib.cell_batch_groups(self._h)

    def autotune(self, force=False):
        _check(_lib.cell_batch_autotune(self._h, int(bool(force))))

    def set_material(self, i, E, nu):
        n = int(np.prod(self.shapes[i]))
        pe, de, ke = _in_ptr(E, n)
        pn, dn, kn = _in_ptr(nu, n)
        if de != dn:
            raise ValueError("E and nu must both be on the host or both on the device")
        _check(_lib.cell_batch_set_material(self._h, int(i), pe, pn, de))

    def solve(self, macro_strains):
        eb = np.ascontiguousarray(np.atleast_2d(np.asarray(macro_strains, dtype=np.float64)))
        nl = eb.shape[0]
        out = np.zeros((self.ncell, nl, self.nv))
        infos = (CellInfo * self.ncell)()
        st = _check(_lib.cell_batch_solve(self._h, nl, eb.ctypes.data_as(ct.c_void_p),
                                          out.ctypes.data_as(ct.c_void_p), infos))
        return out, [dict(i.as_dict(), status=STATUS_NAMES[st]) for i in infos]

    def effective_stiffness(self):
        C = np.zeros((self.ncell, self.nv, self.nv))
        infos = (CellInfo * self.ncell)()
        st = _check(_lib.cell_batch_effective_stiffness(self._h, C.ctypes.data_as(ct.c_void_p), infos))
        return C, [dict(i.as_dict(), status=STATUS_NAMES[st]) for i in infos]

    def displacement(self, i, load=0):
        u = np.zeros((self.dim, int(np.prod(self.shapes[i]))))
        _check(_lib.cell_batch_get_displacement(self._h, int(i), int(load), u.ctypes.data_as(ct.c_void_p), 0))
        return u

    def residual(self, i, load=0):
        r = np.zeros((self.dim, int(np.prod(self.shapes[i]))))
        _check(_lib.cell_batch_get_residual(self._h, int(i), int(load), r.ctypes.data_as(ct.c_void_p), 0))
        return r

    def profile(self, enable=True):
        _check(_lib.cell_batch_profile(self._h, int(bool(enable))))

    def profile_read(self):
        ms = np.zeros(len(KERNEL_KINDS))
        cnt = np.zeros(len(KERNEL_KINDS), dtype=np.int64)
        _check(_lib.cell_batch_profile_read(self._h, ms.ctypes.data_as(ct.c_void_p),
                                            cnt.ctypes.data_as(ct.c_void_p)))
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(KERNEL_KINDS)}


def exported_symbols():
    """Names of the C-ABI functions bound here."""
    return sorted(_SIGS)
