"""Thin ctypes binding of libyeepic.so (argument marshalling only).

Every computation happens in the HIP library; PyTorch supplies device memory
and the stream.  The library must be built in-tree first
(``python -m paper_2004_03754_amd.build``); importing this module never falls
back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libyeepic.so")
_lib = None

PIC_FP64, PIC_FP32_FIELDS = 0, 1
PIC_MAX_M = 16
PIC_PUSH_BORIS, PIC_PUSH_ANALYTIC, PIC_PUSH_HC = 0, 1, 2
PIC_TARGET_E, PIC_TARGET_B, PIC_TARGET_XU, PIC_TARGET_YEET_E, PIC_TARGET_YEET_B = 0, 1, 2, 3, 4
STATUS = {0: "PIC_OK", -1: "PIC_EINVAL", -2: "PIC_ECFL", -3: "PIC_EHIP", -4: "PIC_ESHAPE",
          -5: "PIC_ENOMEM", -6: "PIC_EUNSUPPORTED", -7: "PIC_ENONFINITE", -8: "PIC_ENOCONV"}
PUSHERS = {"boris": PIC_PUSH_BORIS, "analytic": PIC_PUSH_ANALYTIC, "hc": PIC_PUSH_HC}
PIC_DEPOSIT_ATOMIC, PIC_DEPOSIT_DETERMINISTIC = 0, 1


class YeePICError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class _GridDesc(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("n", ctypes.c_int64 * 3), ("dx", ctypes.c_double * 3),
                ("dt", ctypes.c_double), ("M", ctypes.c_int), ("CE", ctypes.POINTER(ctypes.c_double)),
                ("CB", ctypes.POINTER(ctypes.c_double)), ("prec", ctypes.c_int),
                ("E", ctypes.c_void_p * 3), ("B", ctypes.c_void_p * 3), ("J", ctypes.c_void_p * 3),
                ("stream", ctypes.c_void_p)]


class _Particles(ctypes.Structure):
    _fields_ = [("np", ctypes.c_int64), ("x", ctypes.c_void_p * 3), ("u", ctypes.c_void_p * 3),
                ("q", ctypes.c_double), ("m", ctypes.c_double), ("w", ctypes.c_double),
                ("id", ctypes.c_void_p)]


class _Adjoint(ctypes.Structure):
    _fields_ = [("lE", ctypes.c_void_p * 3), ("lB", ctypes.c_void_p * 3), ("gCE", ctypes.c_void_p),
                ("gCB", ctypes.c_void_p), ("En", ctypes.c_void_p * 3), ("Bn", ctypes.c_void_p * 3),
                ("Bh", ctypes.c_void_p * 3), ("lEo", ctypes.c_void_p * 3), ("lBo", ctypes.c_void_p * 3)]


EXPORTS = ["pic_design_coeffs", "pic_init_grid", "pic_set_fields", "pic_advance_B_half", "pic_advance_E",
           "pic_field_sweep", "pic_gather_push", "pic_deposit_J", "pic_step_n", "pic_sync", "pic_check",
           "pic_grid_widths", "pic_destroy", "pic_last_error", "pic_set_sort_interval", "pic_adjoint_step", "pic_step_to",
           "pic_current_correction", "pic_set_shape", "pic_move_window", "pic_window",
           "pic_adjoint_step_noalloc", "pic_set_deposit_mode", "pic_set_exact_iterations", "pic_set_absorber"]


def lib():
    """Load libyeepic.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is missing: build it with `python -m paper_2004_03754_amd.build`")
        L = ctypes.CDLL(_LIB_PATH)
        vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        L.pic_last_error.restype = ctypes.c_char_p
        L.pic_design_coeffs.argtypes = [i, d, i, i, i, d, d, ctypes.POINTER(d)]
        L.pic_init_grid.argtypes = [ctypes.POINTER(_GridDesc), ctypes.POINTER(vp)]
        L.pic_set_fields.argtypes = [vp, ctypes.c_void_p * 3, ctypes.c_void_p * 3, ctypes.c_void_p * 3]
        L.pic_advance_B_half.argtypes = [vp]
        L.pic_advance_E.argtypes = [vp, i]
        L.pic_field_sweep.argtypes = [vp, i]
        L.pic_current_correction.argtypes = [vp, vp]
        L.pic_gather_push.argtypes = [vp, ctypes.POINTER(_Particles), i, vp]
        L.pic_deposit_J.argtypes = [vp, ctypes.POINTER(_Particles), vp, i]
        L.pic_step_n.argtypes = [vp, ctypes.POINTER(ctypes.POINTER(_Particles)), i, i, i, i]
        L.pic_set_sort_interval.argtypes = [vp, i]
        L.pic_set_shape.argtypes = [vp, i]
        L.pic_set_deposit_mode.argtypes = [vp, i]
        L.pic_set_absorber.argtypes = [vp, i, d]
        L.pic_set_exact_iterations.argtypes = [vp, i]
        PP = ctypes.POINTER(ctypes.POINTER(_Particles))
        L.pic_move_window.argtypes = [vp, ctypes.c_int64, PP, i]
        L.pic_window.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        L.pic_adjoint_step.argtypes = [vp, ctypes.POINTER(_Adjoint), PP, PP, i, i]
        L.pic_adjoint_step_noalloc.argtypes = [vp, ctypes.POINTER(_Adjoint), PP, PP, i, i]
        L.pic_step_to.argtypes = [vp, PP, i, i, ctypes.c_void_p * 3, ctypes.c_void_p * 3, ctypes.c_void_p]
        L.pic_sync.argtypes = [vp]
        L.pic_check.argtypes = [vp, ctypes.POINTER(_Particles)]
        L.pic_grid_widths.argtypes = [vp, ctypes.POINTER(i), ctypes.POINTER(i)]
        L.pic_destroy.argtypes = [vp]
        L.pic_destroy.restype = None
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise YeePICError(rc, lib().pic_last_error().decode())


def design_coeffs(M, r, target="E", p=2, n=10, wk1=0.4, width_factor=2.0):
    """App. B customized coefficients computed by the library (host)."""
    t = {"E": PIC_TARGET_E, "B": PIC_TARGET_B, "xu": PIC_TARGET_XU, "yeet_E": PIC_TARGET_YEET_E,
         "yeet_B": PIC_TARGET_YEET_B}[target]
    out = (ctypes.c_double * M)()
    _check(lib().pic_design_coeffs(M, float(r), t, p, n, float(wk1), float(width_factor), out))
    return np.array(out[:], dtype=np.float64)


def _ptr3(ts):
    arr = (ctypes.c_void_p * 3)()
    for c in range(3):
        arr[c] = ts[c].data_ptr() if ts is not None and ts[c] is not None else None
    return arr


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Particles:
    """One species: x and u are float64 device tensors of shape (3, np)
    (rows contiguous); q, m, w are charge, mass and macro-weight."""

    def __init__(self, x, u, q=-1.0, m=1.0, w=1.0, id=None):
        import torch
        assert x.dtype == torch.float64 and u.dtype == torch.float64
        assert x.is_contiguous() and u.is_contiguous() and x.shape == u.shape and x.shape[0] == 3
        if id is not None:
            assert id.dtype == torch.int64 and id.is_contiguous() and id.shape == (x.shape[1],)
        self.x, self.u, self.id = x, u, id
        self.q, self.m, self.w = float(q), float(m), float(w)
        self._s = _Particles()
        npart = x.shape[1]
        self._s.np = npart
        for d in range(3):
            self._s.x[d] = x.data_ptr() + d * npart * 8 if npart else None
            self._s.u[d] = u.data_ptr() + d * npart * 8 if npart else None
        self._s.q, self._s.m, self._s.w = self.q, self.m, self.w
        self._s.id = id.data_ptr() if (id is not None and npart) else None

    @property
    def np(self):
        """Particles in the run: the leading np entries of each row of x, u
        (and of id); a window move that drops particles lowers it."""
        return int(self._s.np)

    def live(self):
        """Views (x, u, id) of the np particles in the run."""
        n = self.np
        return self.x[:, :n], self.u[:, :n], (self.id[:n] if self.id is not None else None)


class Grid:
    """A periodic Yee mesh with caller-owned field tensors (each [n3][n2][n1])."""

    def __init__(self, E, B, dx, dt, CE, CB, J=None, prec="fp64", ndim=3, stream=None):
        import torch
        dtype = torch.float64 if prec == "fp64" else torch.float32
        for t in list(E) + list(B) + (list(J) if J is not None else []):
            assert t.dtype == dtype and t.is_contiguous() and t.is_cuda
        n3, n2, n1 = E[0].shape
        CE = np.ascontiguousarray(CE, dtype=np.float64)
        CB = np.ascontiguousarray(CB, dtype=np.float64)
        assert CE.shape == CB.shape
        self.E, self.B, self.J = list(E), list(B), (list(J) if J is not None else None)
        self.stream = stream
        self._ce, self._cb = CE, CB
        d = _GridDesc()
        d.ndim = ndim
        d.n[:] = [n1, n2, n3]
        dxs = list(dx) + [1.0] * (3 - len(dx))
        d.dx[:] = [float(v) for v in dxs[:3]]
        d.dt = float(dt)
        d.M = CE.shape[0]
        d.CE = CE.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.CB = CB.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.prec = PIC_FP64 if prec == "fp64" else PIC_FP32_FIELDS
        d.E, d.B, d.J = _ptr3(E), _ptr3(B), _ptr3(J)
        d.stream = _stream_handle(stream)
        h = ctypes.c_void_p()
        _check(lib().pic_init_grid(ctypes.byref(d), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().pic_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_fields(self, E, B, J=None):
        """Point the grid at other field arrays of the same shape and precision."""
        self.E, self.B, self.J = list(E), list(B), (list(J) if J is not None else None)
        _check(lib().pic_set_fields(self._h, _ptr3(E), _ptr3(B), _ptr3(J)))

    def adjoint_step(self, lE, lB, gCE, gCB, species=(), lambdas=(), pusher="boris", next_E=None, next_B=None,
                     half_B=None, noalloc=False, out_E=None, out_B=None):
        """Reverse of one vacuum step from the grid's current state (see
        pic_adjoint_step): lE, lB (FP64, field layout) and the particle
        cotangents in ``lambdas`` are mapped from t^{n+1} to t^n (in place
        unless out_E, out_B are given);
        gCE, gCB (16 doubles on the device) are accumulated.  next_E, next_B:
        the forward state at t^{n+1}, if the caller has it; half_B (with
        them): the step's B^{n+1/2}, as step_to writes it.  noalloc: call
        pic_adjoint_step_noalloc (library-held scratch, no allocation).
        out_E, out_B: receive the field cotangents at t^n (out of place; lE
        and lB are then only read; with the forward state and half_B given,
        a 2D grid and C^B = c e1 this takes the fused reverse sweep)."""
        adj = _Adjoint()
        adj.lE, adj.lB = _ptr3(lE), _ptr3(lB)
        adj.gCE, adj.gCB = gCE.data_ptr(), gCB.data_ptr()
        adj.En, adj.Bn, adj.Bh = _ptr3(next_E), _ptr3(next_B), _ptr3(half_B)
        adj.lEo, adj.lBo = _ptr3(out_E), _ptr3(out_B)
        ns = len(species)
        assert len(lambdas) == ns
        a = (ctypes.POINTER(_Particles) * max(1, ns))()
        b = (ctypes.POINTER(_Particles) * max(1, ns))()
        for s_, (p, lam) in enumerate(zip(species, lambdas)):
            a[s_] = ctypes.pointer(p._s)
            b[s_] = ctypes.pointer(lam._s)
        fn = lib().pic_adjoint_step_noalloc if noalloc else lib().pic_adjoint_step
        _check(fn(self._h, ctypes.byref(adj), a, b, ns, PUSHERS[pusher]))

    def widths(self):
        a, b = ctypes.c_int(), ctypes.c_int()
        _check(lib().pic_grid_widths(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def advance_B_half(self):
        _check(lib().pic_advance_B_half(self._h))

    def advance_E(self, use_J=False):
        _check(lib().pic_advance_E(self._h, int(use_J)))

    def sweep(self, use_J=False):
        _check(lib().pic_field_sweep(self._h, int(use_J)))

    def current_correction(self, J1_out):
        """The x1 current Ampere's law uses (pic_current_correction) from the
        grid's J[0] into J1_out (one array of the field layout and precision)."""
        _check(lib().pic_current_correction(self._h, J1_out.data_ptr()))

    def gather_push(self, p: Particles, pusher="boris", x_old=None):
        xo = None
        if x_old is not None:
            arr = (ctypes.c_void_p * 3)()
            npart = x_old.shape[1]
            for dd in range(3):
                arr[dd] = x_old.data_ptr() + dd * npart * 8
            xo = ctypes.cast(arr, ctypes.c_void_p)
            self._xo_keep = arr
        _check(lib().pic_gather_push(self._h, ctypes.byref(p._s), PUSHERS[pusher], xo))

    def deposit_J(self, p: Particles, x_old, zero_first=True):
        arr = (ctypes.c_void_p * 3)()
        npart = x_old.shape[1]
        for dd in range(3):
            arr[dd] = x_old.data_ptr() + dd * npart * 8
        _check(lib().pic_deposit_J(self._h, ctypes.byref(p._s), ctypes.cast(arr, ctypes.c_void_p),
                                   int(zero_first)))

    def step_n(self, species, nsteps, pusher="boris", deposit=False):
        arr = (ctypes.POINTER(_Particles) * max(1, len(species)))()
        for s, p in enumerate(species):
            arr[s] = ctypes.pointer(p._s)
        _check(lib().pic_step_n(self._h, arr, len(species), int(nsteps), PUSHERS[pusher], int(deposit)))

    def step_to(self, species, E_out, B_out, pusher="boris", B_half=None):
        """One vacuum step from the grid's fields into E_out, B_out (see
        pic_step_to); particles advance in place.  B_half (optional, three
        arrays like B_out) receives the step's B^{n+1/2}."""
        arr = (ctypes.POINTER(_Particles) * max(1, len(species)))()
        for s_, p in enumerate(species):
            arr[s_] = ctypes.pointer(p._s)
        half = _ptr3(B_half) if B_half is not None else None
        _check(lib().pic_step_to(self._h, arr, len(species), PUSHERS[pusher], _ptr3(E_out), _ptr3(B_out),
                                 ctypes.cast(half, ctypes.c_void_p) if half is not None else None))

    def set_shape(self, order):
        """Particle shape of gather and deposit: 1 linear, 2 quadratic."""
        _check(lib().pic_set_shape(self._h, int(order)))

    def move_window(self, cells, species=()):
        """Move the x1 window forward by ``cells`` (pic_move_window): the
        field arrays stay a ring (see ``window``); particles of ``species`` in
        the columns left behind are dropped and each species' np updated."""
        arr = (ctypes.POINTER(_Particles) * max(1, len(species)))()
        for s_, p in enumerate(species):
            arr[s_] = ctypes.pointer(p._s)
        _check(lib().pic_move_window(self._h, int(cells), arr, len(species)))

    def window(self):
        """(origin, moved): array column of window cell 0, cells moved."""
        o, m = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().pic_window(self._h, ctypes.byref(o), ctypes.byref(m)))
        return o.value, m.value

    def set_absorber(self, width, sigma=1.0):
        """pic_set_absorber: graded damping layers of ``width`` cells at the
        two x1 ends of the window (0 turns them off)."""
        _check(lib().pic_set_absorber(self._h, int(width), float(sigma)))

    def set_deposit_mode(self, deterministic):
        """pic_set_deposit_mode: fixed-order (deterministic) or atomic tile flush."""
        _check(lib().pic_set_deposit_mode(self._h, PIC_DEPOSIT_DETERMINISTIC if deterministic else PIC_DEPOSIT_ATOMIC))

    def set_exact_iterations(self, max_iter):
        """pic_set_exact_iterations: the exact pusher's iteration cap."""
        _check(lib().pic_set_exact_iterations(self._h, int(max_iter)))

    def set_sort_interval(self, steps):
        _check(lib().pic_set_sort_interval(self._h, int(steps)))

    def sync(self):
        _check(lib().pic_sync(self._h))

    def check(self, p: Particles | None = None):
        _check(lib().pic_check(self._h, ctypes.byref(p._s) if p is not None else None))
