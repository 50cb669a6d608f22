"""Pins of the oracle's quadratic shape (the Sec. 4.2 run's particle shape):
the quadratic B-spline gather against its definition and its moments, and
the Esirkepov deposit on 4-node stencils against continuity and Gauss's law
(CPU only)."""
import numpy as np
import pytest

from oracle import fdtd, particles as pt, pic
from paper_2004_03754_amd import workloads as wl

DX = (wl.DX1, wl.DX2, wl.DX3)


def _b2(t):
    """The quadratic B-spline written piecewise."""
    t = abs(t)
    if t <= 0.5:
        return 0.75 - t * t
    if t <= 1.5:
        return 0.5 * (1.5 - t) ** 2
    return 0.0


def _brute_gather_q(f, off, x, dx, ndim):
    """App. A with the quadratic shape: sum over every grid point (periodic
    images) of f times the product of 1D B-splines."""
    n3, n2, n1 = f.shape
    ns = (n1, n2, n3)
    L = [ns[d] * dx[d] for d in range(3)]
    out = np.zeros(x.shape[1])
    for p in range(x.shape[1]):
        tot = 0.0
        for k in range(n3 if ndim == 3 else 1):
            for j in range(n2):
                for i in range(n1):
                    w = 1.0
                    for d, idx in enumerate((i, j, k)[:ndim]):
                        dist = abs(x[d, p] - (idx + off[d]) * dx[d])
                        dist = min(dist, L[d] - dist)
                        w *= _b2(dist / dx[d])
                    tot += f[k, j, i] * w
        out[p] = tot
    return out


@pytest.mark.parametrize("ndim", [2, 3])
def test_quadratic_gather_matches_definition(ndim):
    n = (7, 5, 4 if ndim == 3 else 1)
    E, B = wl.random_fields(n, seed=31)
    L = [n[d] * DX[d] for d in range(3)]
    x, _ = wl.uniform_particles(6, [0, 0, 0], L, seed=32)
    x[0, 0] = 0.0
    x[1, 1] = L[1] - 1e-13
    x[0, 2] = 2.5 * DX[0]  # half-way between nodes: the nearest-node choice flips
    Ep, Bp = pt.gather(E, B, x, DX, ndim, order=2)
    for c in range(3):
        assert np.allclose(Ep[c], _brute_gather_q(E[c], pt.E_OFF[c], x, DX, ndim), rtol=1e-13, atol=1e-13)
        assert np.allclose(Bp[c], _brute_gather_q(B[c], pt.B_OFF[c], x, DX, ndim), rtol=1e-13, atol=1e-13)


def test_quadratic_gather_moments():
    """The B-spline keeps constants and affine fields, and gathers x1^2 as
    x1^2 + dx1^2/4 (its second central moment), away from the seam."""
    n = (16, 8, 8)
    shape = (n[2], n[1], n[0])
    x, _ = wl.uniform_particles(50, [3 * DX[0], 2 * DX[1], 2 * DX[2]], [12 * DX[0], 6 * DX[1], 6 * DX[2]],
                                seed=33)
    c = np.full(shape, 2.5)
    Ep, Bp = pt.gather((c, c, c), (c, c, c), x, DX, order=2)
    assert np.allclose(Ep, 2.5, rtol=1e-15) and np.allclose(Bp, 2.5, rtol=1e-15)
    i = np.arange(n[0])
    for off in (0.0, 0.5):
        X = (i + off) * DX[0]
        lin = np.broadcast_to(0.3 + 1.7 * X, shape).copy()
        sq = np.broadcast_to(X * X, shape).copy()
        g_lin = pt.gather_component(lin, x, DX, (off, 0.0, 0.0), 3, order=2)
        g_sq = pt.gather_component(sq, x, DX, (off, 0.0, 0.0), 3, order=2)
        assert np.allclose(g_lin, 0.3 + 1.7 * x[0], rtol=1e-14)
        assert np.allclose(g_sq, x[0] ** 2 + DX[0] ** 2 / 4, rtol=1e-13)


@pytest.mark.parametrize("ndim", [2, 3])
def test_quadratic_deposit_continuity(ndim):
    """Sec. 3.3 with the quadratic shape: (rho^{n+1} - rho^n)/dt +
    d_Yee . J = 0 to roundoff, including moves that change the nearest node
    and cross the periodic seam; the total current is q w disp/dt."""
    n = (6, 5, 4 if ndim == 3 else 1)
    shape = (n[2], n[1], n[0])
    L = [n[d] * DX[d] for d in range(3)]
    x0, u = wl.uniform_particles(200, [0, 0, 0], L, seed=34, u_th=0.5)
    x0[0, :5] = 0.02 * DX[0]
    x1, _ = wl.small_moves(x0, DX, L, seed=35)
    q, w, dt = -1.0, 0.37, wl.DT
    J = pt.deposit(x0, x1, q, w, DX, dt, shape, ndim, u=u, order=2)
    rho0 = pt.charge_density(x0, q, w, DX, shape, ndim, order=2)
    rho1 = pt.charge_density(x1, q, w, DX, shape, ndim, order=2)
    res = (rho1 - rho0) / dt + fdtd.div_ampere(J, [1.0], DX)
    assert np.max(np.abs(res)) < 1e-12 * np.max(np.abs(rho1 - rho0) / dt)
    disp = pt.min_image(x1[:ndim], x0[:ndim], L[:ndim])
    for c in range(ndim):
        assert np.isclose(J[c].sum(), q * w * disp[c].sum() / dt, rtol=1e-11)


@pytest.mark.parametrize("r", [0.5, 0.25])
def test_gauss_law_with_quadratic_shape(r, coeffs16, coeffs16_quarter):
    """Gauss's law over 6 plasma steps with quadratic gather and deposit, at
    dt = dx1/2 and (with the x1 current correction) at dt = dx1/4."""
    CE, CB = coeffs16 if r == 0.5 else coeffs16_quarter
    dt = r * DX[0]
    n = (32, 6, 5)
    shape = (n[2], n[1], n[0])
    L = [n[d] * DX[d] for d in range(3)]
    E, B = wl.random_fields(n, seed=36, scale=0.05)
    x, u = wl.uniform_particles(300, [0, 0, 0], L, seed=37, u_th=0.3)
    sp = {"x": x, "u": u, "q": -1.0, "m": 1.0, "w": 0.01}
    g0 = fdtd.div_ampere(E, CB, DX) - pt.charge_density(sp["x"], -1.0, 0.01, DX, shape, order=2)
    for _ in range(6):
        E, B = pic.step(E, B, [sp], CE, CB, DX, dt, deposit=True, order=2)
    g = fdtd.div_ampere(E, CB, DX) - pt.charge_density(sp["x"], -1.0, 0.01, DX, shape, order=2)
    assert np.max(np.abs(g - g0)) < 1e-12 * np.max(np.abs(fdtd.div_ampere(E, CB, DX)))
