"""Pins of the oracle's coefficient fit and k-space analysis (CPU only)."""
import json
import os
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest
import scipy.integrate

from oracle import stencil as st

HERE = os.path.dirname(__file__)


@pytest.fixture(scope="module")
def fits():
    """Proposed-solver coefficients at r = 1/2 for M = 8 and 16 (App. B,
    printed weight, n = 10, w_k1 = 0.4)."""
    out = {}
    for M in (8, 16):
        out[M] = (st.fit_coeffs(M, mp.mpf(1) / 2, "E"), st.fit_coeffs(M, mp.mpf(1) / 2, "B"))
    return out


def test_textbook_coefficients_from_constraint():
    """App. B with M = p/2: the constraint alone gives the textbook staggered
    coefficients (pins the constraint matrix)."""
    with open(os.path.join(HERE, "golden", "textbook_staggered.json")) as f:
        ref = json.load(f)
    for p in (2, 4, 6, 8):
        got = st.standard_coeffs(p)
        want = [Fraction(s) for s in ref[f"p{p}"]]
        assert got == want


def test_paper_printed_dispersion_numbers(golden):
    """Sec. 2.1: Yee beta_phi = 0.99875 (gamma_phi = 20) and 8th order
    beta_phi = 1.00042 for dx1 = 0.2, dt = 0.1, k = k0 = 1; one-wavelength
    slips after ~5e4 and ~1.5e5 steps."""
    dx, dt = golden["fig2_dx1"], golden["fig2_dx1"] * golden["fig2_dt_over_dx1"]
    yee = [1.0]
    c8 = [float(c) for c in st.standard_coeffs(8)]
    b = float(st.phase_velocity(yee, yee, 1.0, dx, dt))
    b8 = float(st.phase_velocity(c8, c8, 1.0, dx, dt))
    assert round(b, 5) == golden["yee_beta_phi"]["value"]
    assert round(b8, 5) == golden["eighth_beta_phi"]["value"]
    assert abs(1 / np.sqrt(1 - b * b) - golden["yee_gamma_phi"]["value"]) < 0.01
    slip = 2 * np.pi / ((1 - b) * dt)
    slip8 = 2 * np.pi / ((b8 - 1) * dt)
    assert abs(slip / golden["yee_slip_steps"]["value"] - 1) < 0.02
    assert abs(slip8 / golden["eighth_slip_steps"]["value"] - 1) < 0.02


def test_fit_B_is_yee_at_half(fits):
    """At dt = dx1/2 the target [k]_B1 of Eq. (new_op) is exactly the Yee
    symbol (the j = 1 basis function), so the unique minimiser is e1."""
    for M in (8, 16):
        cb = fits[M][1]
        with mp.workdps(60):
            assert abs(cb[0] - 1) < mp.mpf(10) ** -35
            assert max(abs(c) for c in cb[1:]) < mp.mpf(10) ** -35


def test_fit_satisfies_constraint_and_is_optimal(fits):
    """App. B: M C = e1 holds, and moving along the constraint's null space
    only increases the weighted error F (checked with scipy's adaptive
    quadrature in FP64, independent of the oracle's Gauss-Legendre sums)."""
    ce = np.array([float(c) for c in fits[8][0]])
    M = len(ce)
    odd = np.arange(1, 2 * M, 2, dtype=np.float64)
    with mp.workdps(60):
        assert abs(sum((2 * j + 1) * c for j, c in enumerate(fits[8][0])) - 1) < mp.mpf(10) ** -40
    r = 0.5

    def F(C):
        def integrand(k):
            w = np.exp(-np.log(2) * (2 * k / 0.4) ** 10)
            approx = np.sum(C * np.sin(odd * np.pi * k)) / np.pi
            return w * (approx - np.tan(np.pi * k * r) / (np.pi * r)) ** 2
        return scipy.integrate.quad(integrand, 0, 0.5, limit=400, epsabs=1e-30, epsrel=1e-12)[0]

    f0 = F(ce)
    g = np.random.default_rng(0)
    for _ in range(4):
        v = g.standard_normal(M)
        v -= odd * (odd @ v) / (odd @ odd)  # null space of the constraint row
        v *= 1e-3 / np.linalg.norm(v)
        assert F(ce + v) > f0


def test_fit_with_M_equal_half_p_is_textbook():
    """App. B with M = p/2 leaves nothing to fit: any target gives the
    textbook coefficients."""
    c = st.fit_coeffs(2, 0.5, "E", p=4, panels=8, G=16, dps=40)
    with mp.workdps(40):
        assert abs(c[0] - mp.mpf(9) / 8) < mp.mpf(10) ** -35
        assert abs(c[1] + mp.mpf(1) / 24) < mp.mpf(10) ** -35


def test_paper_phase_error_magnitudes(fits, golden):
    """Sec. 3.1 (Fig. 2b): ~1e-5 phase-velocity error for k1 < 0.3 k_g1 with
    8 coefficients; 16 coefficients nearly two orders of magnitude better."""
    dx, dt = 0.2, 0.1
    k = np.linspace(1e-4, 0.3, 3001) * 2 * np.pi / dx
    err = {}
    for M in (8, 16):
        ce = [float(c) for c in fits[M][0]]
        cb = [float(c) for c in fits[M][1]]
        err[M] = float(np.max(np.abs(st.phase_velocity(ce, cb, k, dx, dt) - 1)))
    target = golden["m8_phase_error_order"]["value"]
    assert target / 10 < err[8] < target * 10
    assert np.log10(err[8] / err[16]) >= 1.5


def test_phase_velocity_is_c_at_laser_wavelength(fits):
    """Eq. (new_op) fitted with M = 16: at the configs' resolution
    (dx1 = lambda0/32, dt = dx1/2) the k0 mode moves at c and F = 1."""
    dx1 = 2 * np.pi / 32
    ce = [float(c) for c in fits[16][0]]
    cb = [float(c) for c in fits[16][1]]
    assert abs(float(st.phase_velocity(ce, cb, 1.0, dx1, dx1 / 2)) - 1) < 1e-12
    assert abs(float(st.f_factor(ce, cb, 1.0, dx1, dx1 / 2)) - 1) < 1e-12


def test_F_factor_proposed_vs_yee_and_xu(fits):
    """Sec. 3.1 (Fig. 2c): F ~ 1 over a wide k range for the proposed solver;
    Yee and the Xu solver ([k]_E = [k]_B = [k]_{1,t}) deviate."""
    dx, dt = 0.2, 0.1
    k = np.linspace(0.01, 0.25, 200) * 2 * np.pi / dx
    ce = [float(c) for c in fits[16][0]]
    cb = [float(c) for c in fits[16][1]]
    Fp = st.f_factor(ce, cb, k, dx, dt)
    assert np.max(np.abs(Fp - 1)) < 1e-6
    Fy = st.f_factor([1.0], [1.0], k, dx, dt)
    assert np.max(np.abs(Fy - 1)) > 1e-3
    # Xu solver: exact [k]_{1,t} for both operators, so F = cos(omega dt/2)
    kt = np.sin(k * dt / 2) / (dt / 2)
    w = st.omega_from_symbols(kt * kt, dt)
    Fx = np.cos(w * dt / 2)
    assert np.allclose(w, k, rtol=1e-12)
    assert np.max(np.abs(Fx - 1)) > 1e-2


@pytest.mark.parametrize("r", [0.5, 0.25])
def test_xu_fitted_pair_keeps_c_and_gives_F_cos(r):
    """Sec. 4 (Xu solver): [k]_E1 = [k]_B1 = [k]_{1,t}.  With both operators
    equal to the fitted Xu stencil, Eq. (dispersion) gives sin(omega dt/2) =
    sin(k1 dt/2), so v_phi = 1, and the factor of Eq. (f2_q) reduces to
    F = cos(k1 dt/2).  Both hold over kappa <= 0.3 to the fit residual
    (measured 2.3e-8 in v_phi, 5e-9 in F), and F departs from 1 there."""
    cx = np.array([float(c) for c in st.fit_coeffs(16, mp.mpf(r), "xu")])
    dx = 0.2
    dt = r * dx
    k = np.linspace(1e-4, 0.3, 3001) * 2 * np.pi / dx
    vp = st.phase_velocity(cx, cx, k, dx, dt)
    F = st.f_factor(cx, cx, k, dx, dt)
    assert np.max(np.abs(vp - 1)) < 1e-7
    assert np.max(np.abs(F - np.cos(k * dt / 2))) < 1e-7
    assert np.max(np.abs(F - 1)) > 1e-3


def test_cfl_exact_yee_closed_form_and_discrete_growth():
    """Sec. 3.2 exact condition.  For Yee (C = 1) the x1 product peaks at the
    Nyquist mode, [k]^2 = 4/dx1^2, so the bound is
    (dt/2) sqrt(4/dx1^2 + 4/dx2^2 [+ 4/dx3^2]) = dt sqrt(sum 1/dx_d^2) (the
    magic step is where it equals 1).  The discrete sweep's one-step
    amplification of the Nyquist mode has spectral radius 1 just below the
    limit and grows just above it.  For the fitted M = 16 pair the 3D value
    exceeds the 2D one by the x3 term alone; its C^E alternates in sign, so
    at the Nyquist mode [k]_E1 = (2/dx1) sum|C^E| and the sufficient bound is
    attained (exact value 1 there)."""
    dx1, dx2, dx3 = 2 * np.pi / 32, 2 * np.pi / 8, 2 * np.pi / 6
    for dx in ([dx1, dx2], [dx1, dx2, dx3]):
        dtm = 1.0 / np.sqrt(sum(1.0 / d ** 2 for d in dx))
        for f in (0.7, 1.0, 1.3):
            assert abs(st.cfl_exact_max([1.0], [1.0], dx, f * dtm) - f) < 1e-14
        assert st.cfl_exact_max([1.0], [1.0], dx, dtm * (1 - 1e-3)) < 1
        assert st.cfl_exact_max([1.0], [1.0], dx, dtm * (1 + 1e-3)) > 1
    from oracle import fdtd
    dx = [dx1, dx2, dx3]
    dtm = 1.0 / np.sqrt(sum(1.0 / d ** 2 for d in dx))
    k = (np.pi / dx1, np.pi / dx2, np.pi / dx3)
    rad = {}
    for f in (0.99, 1.01):
        G = fdtd.amplification_matrix(k, [1.0], [1.0], dx, f * dtm, n=(2, 2, 2))
        rad[f] = float(np.max(np.abs(np.linalg.eigvals(G))))
    assert abs(rad[0.99] - 1) < 1e-9
    assert rad[1.01] > 1 + 1e-2
    ce, cb = st.fit_pair(16, 0.5)
    dt = dx1 / 2
    v2 = st.cfl_exact_max(ce, cb, [dx1, dx2], dt)
    v3 = st.cfl_exact_max(ce, cb, [dx1, dx2, dx3], dt)
    assert abs((v3 ** 2 - v2 ** 2) - (dt / 2) ** 2 * 4 / dx3 ** 2) < 1e-14
    assert np.all(ce[:-1] * ce[1:] < 0)
    assert abs(st.cfl_exact_max(ce, cb, [dx1, dx2, dx3], st.cfl_sufficient_dt(ce, cb, [dx1, dx2, dx3])) - 1) < 1e-14


def test_oblique_waves(fits):
    """Sec. 3.1.1: leading term of Eq. (vphi_ob) is exactly 1 for the proposed
    solver (eta = 1) and below 1 for Yee; the symbol-based v_phi matches the
    unified formula; Yee at the 2D magic time step has v_phi(pi/4) = 1;
    kappa(0) = 1 for the proposed solver."""
    dx1 = dx2 = 0.2
    for dt in (0.1, 0.2 / np.sqrt(2) * 0.999):
        assert abs(st.oblique_leading_term(1.0, dt, 1.0) - 1) < 1e-15
        assert st.oblique_leading_term(1.0, dt, dx1 / dt) < 1
        th = np.linspace(0, np.pi / 2, 31)
        vy, _ = st.oblique([1.0], [1.0], 1.0, th, dx1, dx2, dt)
        assert np.allclose(vy, st.oblique_vphi_formula(1.0, th, dx1, dx2, dt, dx1 / dt), rtol=1e-13)
    dt = 0.1
    ce16 = [float(c) for c in st.fit_coeffs(16, mp.mpf(dt) / dx1, "E")]
    cb16 = [float(c) for c in st.fit_coeffs(16, mp.mpf(dt) / dx1, "B")]
    th = np.linspace(0, np.pi / 2, 31)
    vp, kap = st.oblique(ce16, cb16, 1.0, th, dx1, dx2, dt)
    assert np.allclose(vp, st.oblique_vphi_formula(1.0, th, dx1, dx2, dt, 1.0), rtol=1e-7)
    assert abs(kap[0] - 1) < 1e-7
    vy, ky = st.oblique([1.0], [1.0], 1.0, th, dx1, dx2, dt)
    assert np.all(np.abs(vp[:-1] - 1) <= np.abs(vy[:-1] - 1))
    assert np.all(np.abs(kap - 1) <= np.abs(ky - 1) + 1e-12)
    # Yee, square cells, dt -> dx/sqrt(2): v_phi = 1 at 45 degrees
    dtm = dx1 / np.sqrt(2)
    v45, _ = st.oblique([1.0], [1.0], 1.0, np.pi / 4, dx1, dx2, dtm)
    assert abs(float(v45) - 1) < 1e-12


def test_cfl_at_configs(fits):
    """Sec. 3.2: dt = dx1/2 is within the sufficient bound for the M = 16
    proposed solver on the configs' meshes (2D and 3D); the Yee 2D bound
    equals 1/sqrt(1/dx1^2 + 1/dx2^2)."""
    dx1, dx2 = 2 * np.pi / 32, 2 * np.pi / 8
    dt = dx1 / 2
    ce = [float(c) for c in fits[16][0]]
    cb = [float(c) for c in fits[16][1]]
    r3 = dt / st.cfl_sufficient_dt(ce, cb, [dx1, dx2, dx2])
    r2 = dt / st.cfl_sufficient_dt(ce, cb, [dx1, dx2])
    assert 0.6 < r2 < r3 < 0.7
    assert st.cfl_exact_max(ce, cb, [dx1, dx2, dx2], dt) <= 1
    assert abs(st.cfl_sufficient_dt([1.0], [1.0], [dx1, dx2]) - 1 / np.sqrt(1 / dx1**2 + 1 / dx2**2)) < 1e-15
