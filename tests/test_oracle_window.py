"""Pins of the oracle's moving window and of the single-particle runs of
Sec. 4.1 (a drifting electron in a flat-top plane wave, window moving at c).

The window's shift is checked against its definition from both sides
(composition, which particles leave, what enters at the front); the run as a
whole is pinned by the closed-form trajectory (itself checked against a
direct integration of the Lorentz force) and by the plane wave keeping its
shape in the co-moving window with the proposed solver but not with Yee's.
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import pic, trajectory, window
from paper_2004_03754_amd import workloads as wl

# Sec. 4.1 grid: dt = 0.05, dx1 = 0.2 (r = 1/4), dx2 = 20
DX1, DX2, DT = 0.2, 20.0, 0.05
N1, N2 = 1024, 4
GAMMA0 = 20.0
X_HEAD = 180.0


def _random_species(n1, n2, n3, seed, npart=400):
    g = wl.rng(seed)
    L = np.array([n1 * DX1, n2 * DX2, n3 * DX2])
    # keep positions away from cell faces so that "x1 < s dx1" has one answer
    cell = g.integers(0, n1, npart)
    frac = 0.05 + 0.9 * g.random(npart)
    x = np.stack([(cell + frac) * DX1, L[1] * g.random(npart), L[2] * g.random(npart)])
    u = g.standard_normal((3, npart))
    return dict(x=x, u=u, id=np.arange(npart, dtype=np.int64), q=-1.0, m=1.0, w=1.0)


def test_shift_matches_definition():
    n1, n2, n3 = 128, 3, 2
    E, B = wl.random_fields((n1, n2, n3), seed=71)
    sp = _random_species(n1, n2, n3, 72)
    x0 = sp["x"].copy()
    s = 37
    E1, B1 = window.move(E, B, [sp], s, DX1)
    for f, f1 in zip(E + B, E1 + B1):
        # window cell i now holds old cell i + s; the s front cells are vacuum
        for i in (0, 1, 50, n1 - s - 1):
            np.testing.assert_array_equal(f1[..., i], f[..., i + s])
        assert not np.any(f1[..., n1 - s:])
        # the field energy kept is exactly that of the columns still inside
        assert np.sum(f1 ** 2) == pytest.approx(np.sum(f[..., s:] ** 2), rel=1e-15)
    left = x0[0] < s * DX1
    assert left.sum() > 0 and (~left).sum() > 0
    np.testing.assert_array_equal(sp["id"], np.flatnonzero(~left))
    np.testing.assert_allclose(sp["x"][0], x0[0, ~left] - s * DX1, rtol=0, atol=1e-13)
    np.testing.assert_array_equal(sp["x"][1:], x0[1:, ~left])
    assert np.all(sp["x"][0] >= 0)


def test_shift_composes_and_zero_is_identity():
    n1, n2, n3 = 192, 2, 1
    E, B = wl.random_fields((n1, n2, n3), seed=73)
    a = _random_species(n1, n2, n3, 74)
    b = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in a.items()}
    Ea, Ba = window.move(E, B, [a], 0, DX1)
    for f, g in zip(E + B, Ea + Ba):
        np.testing.assert_array_equal(f, g)
    Ea, Ba = window.move(*window.move(E, B, [a], 11, DX1), [a], 29, DX1)
    Eb, Bb = window.move(E, B, [b], 40, DX1)
    for f, g in zip(Ea + Ba, Eb + Bb):
        np.testing.assert_array_equal(f, g)
    np.testing.assert_array_equal(a["id"], b["id"])
    np.testing.assert_allclose(a["x"], b["x"], rtol=0, atol=1e-13)
    with pytest.raises(ValueError):
        window.shift_field(E[0], n1)


def test_cells_due_moves_at_c():
    assert [window.cells_due(n, DT, DX1) for n in range(9)] == [0, 0, 0, 0, 1, 1, 1, 1, 2]
    assert window.cells_due(2000, DT, DX1) == 500


def _lorentz(pulse, qm):
    def f(t, y):
        x1, u = y[0], y[3:]
        g = np.sqrt(1.0 + u @ u)
        fld = -pulse.da(X_HEAD - x1 + t)
        v = u / g
        return np.concatenate([v, qm * np.array([v[1] * fld, fld - v[0] * fld, 0.0])])
    return f


@pytest.mark.parametrize("a0", [0.5, 3.0])
def test_drifting_closed_form_matches_lorentz_force(a0):
    """The closed form with h = gamma0 - u1_0 against DOP853 on the equations
    of motion in the analytic wave E2 = B3 = -a'(x_head - x1 + t)."""
    pulse = wl.FlatTopPulse(a0)
    xp = X_HEAD - (pulse.R + 16 * np.pi)
    u10 = np.sqrt(GAMMA0 ** 2 - 1)
    T = 300.0
    sol = solve_ivp(_lorentz(pulse, -1.0), (0, T), [xp, 0, 0, u10, 0, 0], method="DOP853",
                    rtol=1e-12, atol=1e-12, dense_output=True)
    for t in (37.0, 150.0, T):
        y = sol.sol(t)
        x, u, g = trajectory.state_at(lambda s: pulse.a(X_HEAD + s), -1.0, 0.0,
                                      np.array([[xp], [0.0], [0.0]]), t, gamma0=GAMMA0)
        assert abs(x[0, 0] - y[0]) <= 1e-9 * abs(y[0])
        assert abs(x[1, 0] - y[1]) <= 1e-9 * max(1.0, abs(y[1]))
        assert abs(u[1, 0] - y[4]) <= 1e-9 * a0
        assert abs(u[0, 0] - y[3]) <= 1e-9 * y[3]
        assert abs(g[0] - np.sqrt(1 + y[3:] @ y[3:])) <= 1e-9 * g[0]


def _suite_run(E, B, CE, CB, xp, nsteps):
    sp = dict(x=np.array([[xp], [0.5 * DX2], [0.0]]),
              u=np.array([[np.sqrt(GAMMA0 ** 2 - 1)], [0.0], [0.0]]), q=-1.0, m=1.0, w=1.0)
    moved = 0
    for n in range(nsteps):
        E, B = pic.step(E, B, [sp], CE, CB, (DX1, DX2, DX2), DT, pusher="hc", ndim=2)
        due = window.cells_due(n + 1, DT, DX1)
        if due > moved:
            E, B = window.move(E, B, [sp], due - moved, DX1)
            moved = due
    return E, B, sp, moved


def test_single_particle_run_proposed_vs_yee(coeffs16_quarter):
    """Sec. 4.1, first case: gamma0 = 20 drift at a0 = 0.5, starting where
    the vector potential vanishes in the flat top, Higuera-Cary pusher,
    window moving at c.  With the proposed solver the run follows the
    closed form and the plane wave keeps its shape in the window; with the
    Yee solver the laser lags and the transverse momentum departs from the
    theory (the paper's point about the Yee-type solvers)."""
    pulse = wl.FlatTopPulse(0.5)
    E, B = wl.laser_fields((N1, N2, 1), (DX1, DX2, DX2), pulse, x_head=X_HEAD)
    xp = X_HEAD - (pulse.R + 16 * np.pi)
    nsteps = 1000
    T = nsteps * DT
    x_th, _, _ = trajectory.state_at(lambda s: pulse.a(X_HEAD + s), -1.0, 0.0,
                                     np.array([[xp], [0.0], [0.0]]), T, gamma0=GAMMA0)
    _, u_th, _ = trajectory.state_at(lambda s: pulse.a(X_HEAD + s), -1.0, 0.0,
                                     np.array([[xp], [0.0], [0.0]]), T - DT / 2, gamma0=GAMMA0)
    CE, CB = coeffs16_quarter
    Ep, _, sp, moved = _suite_run(E, B, CE, CB, xp, nsteps)
    assert moved == 250
    assert abs(sp["x"][0, 0] + moved * DX1 - x_th[0, 0]) <= 1e-8 * x_th[0, 0]
    assert abs(sp["u"][1, 0] - u_th[1, 0]) <= 5e-4 * 0.5
    assert abs(sp["u"][0, 0] - u_th[0, 0]) <= 1e-5 * u_th[0, 0]
    # T is a whole number of cells: the wave in the window equals the start
    assert np.abs(Ep[1] - E[1]).max() <= 1e-6 * np.abs(E[1]).max()

    yee = np.zeros(16)
    yee[0] = 1.0
    Ey, _, spy, _ = _suite_run(E, B, yee, yee.copy(), xp, nsteps)
    assert abs(spy["u"][1, 0] - u_th[1, 0]) >= 10 * 5e-4 * 0.5
    assert np.abs(Ey[1] - E[1]).max() >= 1e-2 * np.abs(E[1]).max()
