"""Pins of the oracle's field step (CPU only)."""
import numpy as np
import pytest

from oracle import fdtd, stencil as st
from paper_2004_03754_amd import workloads as wl


def _measured_omegas(G, dt):
    """Non-static eigenvalues of a sweep's amplification matrix -> omega."""
    lam = np.linalg.eigvals(G)
    moving = lam[np.abs(lam - 1) > 1e-9]
    assert np.allclose(np.abs(moving), 1, atol=1e-12)
    return np.sort(np.abs(np.angle(moving))) / dt


@pytest.mark.parametrize("solver", ["yee", "custom"])
@pytest.mark.parametrize("kvec", [(3, 0, 0), (11, 0, 0), (5, 1, 0), (2, 1, 1)])
def test_single_mode_dispersion(solver, kvec, coeffs16):
    """Eq. (dispersion) generalised to 3D: a single Fourier mode of the
    discrete sweep rotates by omega with sin(omega dt/2) = (dt/2)
    sqrt(sum_d [k]_Ed [k]_Bd), the x2/x3 operators being Yee.  For M = 1 along
    x1 this is the Yee relation sin(omega dt/2)/dt = sin(k dx/2)/dx."""
    dx = (wl.DX1, wl.DX2, wl.DX3)
    dt = wl.DT
    n = (64, 4, 4)
    if solver == "yee":
        CE = CB = np.array([1.0])
    else:
        CE, CB = coeffs16
    k = [2 * np.pi * kvec[d] / (n[d] * dx[d]) for d in range(3)]
    G = fdtd.amplification_matrix(k, CE, CB, dx, dt, n)
    s = st.symbol(CE, k[0], dx[0]) * st.symbol(CB, k[0], dx[0])
    s += st.yee_symbol(k[1], dx[1]) ** 2 + st.yee_symbol(k[2], dx[2]) ** 2
    w_formula = st.omega_from_symbols(s, dt)
    w_meas = _measured_omegas(G, dt)
    assert np.allclose(w_meas, w_formula, rtol=1e-11, atol=0)
    if solver == "yee" and kvec[1] == kvec[2] == 0:
        assert np.allclose(np.sin(w_meas * dt / 2) / dt, np.sin(k[0] * dx[0] / 2) / dx[0], rtol=1e-12)


def test_custom_solver_phase_velocity_of_laser_mode(coeffs16):
    """The k0 = 1 mode (32 cells per wavelength) of the M = 16 proposed
    solver moves at c: measured from the stepped mode, not the symbol."""
    CE, CB = coeffs16
    dx = (wl.DX1, wl.DX2, wl.DX3)
    n = (64, 1, 1)  # two wavelengths along x1
    G = fdtd.amplification_matrix([1.0, 0.0, 0.0], CE, CB, dx, wl.DT, n)
    w = _measured_omegas(G, wl.DT)
    assert np.allclose(w, 1.0, rtol=0, atol=1e-12)


def test_unstable_dt_grows(coeffs16):
    """Sec. 3.2: beyond the CFL bound some mode grows (|eigenvalue| > 1)."""
    CE, CB = coeffs16
    dx = (wl.DX1, wl.DX2, wl.DX3)
    dtmax = st.cfl_sufficient_dt(CE, CB, dx)
    dt = 1.6 * dtmax
    n = (32, 2, 2)
    grow = 0.0
    for k1 in range(0, 17):
        k = [2 * np.pi * k1 / (n[0] * dx[0]), np.pi / dx[1], np.pi / dx[2]]
        lam = np.linalg.eigvals(fdtd.amplification_matrix(k, CE, CB, dx, dt, n))
        grow = max(grow, np.max(np.abs(lam)))
    assert grow > 1 + 1e-6


@pytest.mark.parametrize("ndim", [2, 3])
def test_divergences_preserved(ndim, coeffs16):
    """Faraday's divergence (C^E in x1) of B and, without current, Gauss's
    divergence (C^B in x1) of E are constant to roundoff over 20 sweeps."""
    CE, CB = coeffs16
    CB = CB + np.r_[0.0, 0.01 * np.ones(15)]  # a non-trivial Ampere stencil too
    n = (48, 8, 6 if ndim == 3 else 1)
    dx = (wl.DX1, wl.DX2, wl.DX3)
    E, B = wl.random_fields(n, seed=1)
    d0B = fdtd.div_faraday(B, CE, dx)
    d0E = fdtd.div_ampere(E, CB, dx)
    for _ in range(20):
        E, B = fdtd.sweep(E, B, None, CE, CB, dx, wl.DT)
    scaleB = np.max(np.abs(d0B))
    scaleE = np.max(np.abs(d0E))
    assert np.max(np.abs(fdtd.div_faraday(B, CE, dx) - d0B)) < 1e-12 * scaleB
    assert np.max(np.abs(fdtd.div_ampere(E, CB, dx) - d0E)) < 1e-12 * scaleE


def test_sweep_is_half_steps(coeffs16):
    """The fused sweep equals B half step, E step, B half step applied one by
    one, and the J term enters E only (Eq. maxwell)."""
    CE, CB = coeffs16
    n = (32, 4, 3)
    dx = (wl.DX1, wl.DX2, wl.DX3)
    E, B = wl.random_fields(n, seed=2)
    J, _ = wl.random_fields(n, seed=3)
    En, Bn = fdtd.sweep(E, B, J, CE, CB, dx, wl.DT)
    Bh = fdtd.advance_B(E, B, CE, dx, wl.DT / 2)
    E2 = fdtd.advance_E(E, Bh, J, CB, dx, wl.DT)
    B2 = fdtd.advance_B(E2, Bh, CE, dx, wl.DT / 2)
    for a, b in zip(En + Bn, E2 + B2):
        assert np.array_equal(a, b)
    # J only enters through Ampere: E(J) - E(0) = -dt J in the E step
    E0, _ = fdtd.sweep(E, B, None, CE, CB, dx, wl.DT)
    Bh0 = fdtd.advance_B(E, B, CE, dx, wl.DT / 2)
    for c in range(3):
        e_j = fdtd.advance_E(E, Bh0, J, CB, dx, wl.DT)[c]
        e_0 = fdtd.advance_E(E, Bh0, None, CB, dx, wl.DT)[c]
        assert np.allclose(e_j - e_0, -wl.DT * J[c], rtol=0, atol=1e-14)
    assert not np.allclose(E0[0], En[0])


def test_stencil_taps_brute_force():
    """App. B operators written as explicit sums over grid indices on a small
    1D row, against the roll-based implementation."""
    g = np.random.default_rng(5)
    f = g.standard_normal((1, 1, 23))
    C = g.standard_normal(4)
    n = 23
    dE = np.zeros(n)
    dB = np.zeros(n)
    for i in range(n):
        for j in range(1, 5):
            dE[i] += C[j - 1] * (f[0, 0, (i + j) % n] - f[0, 0, (i - j + 1) % n])
            dB[i] += C[j - 1] * (f[0, 0, (i + j - 1) % n] - f[0, 0, (i - j) % n])
    assert np.allclose(fdtd.d1_faraday(f, C, 0.5)[0, 0], dE / 0.5, rtol=1e-14, atol=1e-14)
    assert np.allclose(fdtd.d1_ampere(f, C, 0.5)[0, 0], dB / 0.5, rtol=1e-14, atol=1e-14)
