"""Pins of the seeded input generators (CPU only): the Gaussian laser beam's
longitudinal fields.

E2 = B3 = f(x1) g(x2, x3) alone has a divergence of the size of the
transverse field's x2 (x3) derivative; the first-order longitudinal terms
E1 = a(x_head - x1) (2 x2/w0^2) g and B1 = a(x_head - x1) (2 x3/w0^2) g make
both fields divergence-free in the continuum, so on the staggered mesh only
the discretisation error of the Yee differences remains (second order in the
cell size).  The mesh keeps the Gaussian's tail negligible at its periodic
edges (half-width 4 w0)."""
import numpy as np
import pytest

from oracle import fdtd
from paper_2004_03754_amd import workloads as wl

DX = (wl.DX1, wl.DX2, wl.DX3)
L0 = wl.LAMBDA0
YEE = np.array([1.0])


def _divs(E, B):
    return (float(np.max(np.abs(fdtd.div_ampere(E, YEE, DX)))),
            float(np.max(np.abs(fdtd.div_faraday(B, YEE, DX)))))


@pytest.mark.parametrize("w0,n", [(1.0, (256, 64, 64)), (2.0, (256, 128, 128))])
def test_gaussian_beam_is_divergence_free_to_second_order(w0, n):
    pulse = wl.Sin2Pulse(a0=1.0, Lp=4 * L0)
    E, B = wl.laser_fields(n, DX, pulse, x_head=6 * L0, w0=w0 * L0)
    dE, dB = _divs(E, B)
    # the transverse fields alone
    dE0, dB0 = _divs([np.zeros_like(E[0]), E[1], E[2]], [np.zeros_like(B[0]), B[1], B[2]])
    assert dE0 > 1e-2 and dB0 > 1e-2
    assert dE <= 5e-3 * dE0, (dE, dE0)
    assert dB <= 5e-3 * dB0, (dB, dB0)
    # each longitudinal component is odd in its own transverse coordinate
    # about the axis and vanishes without a transverse profile
    assert np.max(np.abs(E[0])) > 0 and np.max(np.abs(B[0])) > 0
    assert wl.laser_longitudinal(n, DX, pulse, x_head=6 * L0) is None


def test_longitudinal_factors_match_the_fields():
    """laser_fields' E1, B1 are the outer products of laser_longitudinal's
    factors (the form the benchmark builds on the device)."""
    n = (128, 32, 16)
    pulse = wl.Sin2Pulse(a0=3.0, Lp=4 * L0)
    E, B = wl.laser_fields(n, DX, pulse, x_head=3 * L0, w0=L0)
    e1, p1, b1, q1 = wl.laser_longitudinal(n, DX, pulse, x_head=3 * L0, w0=L0)
    assert np.array_equal(E[0], p1[:, :, None] * e1[None, None, :])
    assert np.array_equal(B[0], q1[:, :, None] * b1[None, None, :])
    # E1 at x2 = j dx2 (on the axis row it vanishes), B1 at x3 = (k + 1/2) dx3
    assert np.all(p1[:, n[1] // 2] == 0.0)
    assert np.all(np.sign(q1[: n[2] // 2]) <= 0) and np.all(np.sign(q1[n[2] // 2:]) >= 0)
