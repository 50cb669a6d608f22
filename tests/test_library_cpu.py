"""Host-side checks of the C ABI library (no GPU needed): it loads, exports
every symbol the header declares, fits coefficients like the oracle, and
validates descriptors before touching the device."""
import ctypes
import os
import re

import mpmath as mp
import numpy as np
import pytest

from oracle import stencil
from paper_2004_03754_amd import binding as b

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    with open(os.path.join(ROOT, "include", "yeepic.h")) as f:
        header = f.read()
    declared = set(re.findall(r"\b(pic_[a-z_A-Z0-9]+)\s*\(", header))
    assert declared, "no declarations found"
    L = b.lib()
    for name in sorted(declared):
        assert hasattr(L, name), f"{name} declared but not exported"
    assert declared == set(b.EXPORTS)


@pytest.mark.parametrize("M,r,target", [(16, 0.5, "E"), (16, 0.5, "B"), (8, 0.5, "E"), (8, 0.25, "E"),
                                        (8, 0.25, "B"), (4, 0.3, "xu"), (8, 0.25, "yeet_E"),
                                        (8, 0.25, "yeet_B")])
def test_design_coeffs_matches_oracle_fit(M, r, target):
    """App. B: the library's binary128 null-space QR fit agrees with the
    oracle's 60-digit KKT solve (both approximate the same integrals)."""
    got = b.design_coeffs(M, r, target)
    ref = np.array([float(c) for c in stencil.fit_coeffs(M, mp.mpf(r), target)])
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(got - ref)) <= 1e-14 * scale
    # the constraint sum (2j-1) C_j = 1 holds to double rounding
    assert abs(np.sum((2 * np.arange(M) + 1) * got) - 1) < 1e-13


def test_design_coeffs_textbook_and_yee_exactness():
    """M = p/2 gives the textbook coefficients; r = 1/2 gives C^B = e1 up to
    a tail far below double resolution (trimmed by the grid)."""
    c = b.design_coeffs(2, 0.5, "E", p=4)
    assert np.allclose(c, [9 / 8, -1 / 24], rtol=1e-15)
    cb = b.design_coeffs(16, 0.5, "B")
    assert cb[0] == 1.0 and np.sum(np.abs(cb[1:])) < 2.0 ** -70


@pytest.mark.parametrize("bad", [dict(M=0), dict(M=17), dict(p=3), dict(r=1.0), dict(r=0.0), dict(wk1=-1.0)])
def test_design_coeffs_rejects_bad_arguments(bad):
    args = dict(M=8, r=0.5, target="E", p=2, n=10, wk1=0.4)
    args.update(bad)
    with pytest.raises(b.YeePICError) as e:
        b.design_coeffs(**args)
    assert e.value.code == -1


def _desc(**kw):
    d = b._GridDesc()
    d.ndim = kw.get("ndim", 3)
    d.n[:] = kw.get("n", [128, 8, 8])
    d.dx[:] = kw.get("dx", [np.pi / 16, np.pi / 4, np.pi / 4])
    d.dt = kw.get("dt", np.pi / 32)
    ce = np.ascontiguousarray(kw.get("CE", [1.0]), dtype=np.float64)
    cb = np.ascontiguousarray(kw.get("CB", [1.0]), dtype=np.float64)
    d.M = kw.get("M", ce.shape[0])
    d.CE = ce.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.CB = cb.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.prec = kw.get("prec", 0)
    fake = kw.get("ptr", 4096)
    for c in range(3):
        d.E[c] = fake
        d.B[c] = fake
        d.J[c] = None
    d._keep = (ce, cb)
    return d


@pytest.mark.parametrize("kw,code", [
    (dict(ndim=4), -1),                     # PIC_EINVAL
    (dict(prec=7), -1),
    (dict(M=0), -1),
    (dict(n=[100, 8, 8]), -4),              # PIC_ESHAPE: n1 not a multiple of 64
    (dict(n=[1 << 20, 1 << 12, 1]), -4),    # more than 2^31 cells
    (dict(ptr=4100), -4),                   # misaligned fields
    (dict(ptr=0), -1),                      # NULL fields
    (dict(dt=0.5), -2),                     # PIC_ECFL (Sec. 3.2)
    (dict(dt=-0.1), -1),
])
def test_init_grid_validation_before_device(kw, code):
    """Descriptor errors are reported before any device call (Sec. 3.2 CFL
    included), so these run without a GPU."""
    d = _desc(**kw)
    h = ctypes.c_void_p()
    rc = b.lib().pic_init_grid(ctypes.byref(d), ctypes.byref(h))
    assert rc == code, b.lib().pic_last_error()
    assert not h.value


def test_cfl_bound_is_the_papers(coeffs16):
    """The init check uses the Sec. 3.2 sufficient bound: just below it is
    accepted by validation (fails later only for lack of device memory),
    just above it is PIC_ECFL."""
    CE, CB = coeffs16
    dx = [np.pi / 16, np.pi / 4, np.pi / 4]
    dtmax = stencil.cfl_sufficient_dt(CE, CB, dx)
    h = ctypes.c_void_p()
    d = _desc(CE=CE, CB=CB, dt=dtmax * 1.0001)
    assert b.lib().pic_init_grid(ctypes.byref(d), ctypes.byref(h)) == -2
    d = _desc(CE=CE, CB=CB, dt=dtmax * 0.9999)
    assert b.lib().pic_init_grid(ctypes.byref(d), ctypes.byref(h)) != -2
    if h.value:  # a GPU was present: the grid was created on fake field pointers
        b.lib().pic_destroy(h)


def test_null_handles_are_rejected_without_a_device():
    """Entry points given a NULL grid return PIC_EINVAL before any device
    call (window, shape, sort interval, correction, step loop)."""
    L = b.lib()
    o, m = ctypes.c_int64(), ctypes.c_int64()
    assert L.pic_move_window(None, 1, None, 0) == -1
    assert L.pic_window(None, ctypes.byref(o), ctypes.byref(m)) == -1
    assert L.pic_set_shape(None, 1) == -1
    assert L.pic_set_sort_interval(None, 3) == -1
    assert L.pic_current_correction(None, None) == -1
    assert L.pic_step_n(None, None, 0, 1, 0, 0) == -1
