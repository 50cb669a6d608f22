"""Pins of the oracle's gather, pushers and deposit (CPU only)."""
import numpy as np
import pytest
import scipy.integrate

from oracle import fdtd, particles as pt
from paper_2004_03754_amd import workloads as wl

DX = (wl.DX1, wl.DX2, wl.DX3)


def _brute_gather(f, off, x, dx, ndim):
    """App. A written out: sum over every grid point (with periodic images)
    of f times the product of 1D linear hats."""
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
                        X = (idx + off[d]) * dx[d]
                        dist = abs(x[d, p] - X)
                        dist = min(dist, L[d] - dist)
                        w *= max(0.0, 1.0 - dist / dx[d])
                    tot += f[k, j, i] * w
        out[p] = tot
    return out


@pytest.mark.parametrize("ndim", [2, 3])
def test_gather_matches_definition(ndim):
    """App. A: each component from its own staggered points, linear shape."""
    n = (7, 5, 4 if ndim == 3 else 1)
    E, B = wl.random_fields(n, seed=11)
    L = [n[d] * DX[d] for d in range(3)]
    x, _ = wl.uniform_particles(6, [0, 0, 0], L, seed=12)
    x[0, 0] = 0.0                      # on a node, at the wrap
    x[1, 1] = L[1] - 1e-13             # just below the box end
    Ep, Bp = pt.gather(E, B, x, DX, ndim)
    for c in range(3):
        assert np.allclose(Ep[c], _brute_gather(E[c], pt.E_OFF[c], x, DX, ndim), rtol=1e-13, atol=1e-13)
        assert np.allclose(Bp[c], _brute_gather(B[c], pt.B_OFF[c], x, DX, ndim), rtol=1e-13, atol=1e-13)


def test_gather_exact_for_affine_and_constant():
    """Linear interpolation reproduces constants everywhere and affine fields
    inside the grid (away from the periodic seam)."""
    n = (16, 8, 8)
    shape = (n[2], n[1], n[0])
    c = np.full(shape, 2.5)
    x, _ = wl.uniform_particles(50, [3 * DX[0], 2 * DX[1], 2 * DX[2]],
                                [12 * DX[0], 6 * DX[1], 6 * DX[2]], seed=13)
    Ep, Bp = pt.gather((c, c, c), (c, c, c), x, DX)
    assert np.allclose(Ep, 2.5, rtol=1e-15) and np.allclose(Bp, 2.5, rtol=1e-15)
    k, j, i = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    for comp in range(3):
        off = pt.E_OFF[comp]
        f = 0.3 * (i + off[0]) * DX[0] - 0.7 * (j + off[1]) * DX[1] + 1.1 * (k + off[2]) * DX[2]
        got = pt.gather_component(f, x, DX, off, 3)
        assert np.allclose(got, 0.3 * x[0] - 0.7 * x[1] + 1.1 * x[2], rtol=1e-13)


def _rand_fields(np_, seed, scale=1.0):
    g = np.random.default_rng(seed)
    return scale * g.standard_normal((3, np_)), scale * g.standard_normal((3, np_))


@pytest.mark.parametrize("push", [pt.boris, pt.analytic, pt.higuera_cary])
def test_pure_electric_field(push):
    """Every pusher: with B = 0 the lab-time momentum change is q E dt."""
    g = np.random.default_rng(1)
    u = g.standard_normal((3, 20)) * 3
    E = g.standard_normal((3, 20)) * 5
    B = np.zeros_like(E)
    qm, dt = -1.0, 0.1
    assert np.allclose(push(u, E, B, qm, dt), u + qm * E * dt, rtol=1e-12, atol=1e-12)


def test_exact_pusher_strong_fields():
    """The exact pusher's lab-time root t(tau) = dt in the strong-field
    regime, where t(tau) grows like exp(kappa tau) with kappa dt up to 1e4
    (the first guess tau = dt/gamma overflows): from rest a pure E field gives
    u = q E dt exactly, and near-null crossed fields of 1e4 (E along x2, B
    along x3 slightly weaker) keep the semigroup and time-reversal
    properties of an exact map."""
    E0 = np.array([1e2, 1e3, 1e4, 1e5])
    E = np.zeros((3, 4))
    E[0] = E0
    u = np.zeros((3, 4))
    qm, dt = -1.0, 0.1
    assert np.allclose(pt.analytic(u, E, np.zeros_like(E), qm, dt), qm * E * dt, rtol=1e-12, atol=0)
    delta = np.array([1e-4, 1e-3, 1e-2, 0.1, 0.5])
    E = np.zeros((3, 5))
    B = np.zeros((3, 5))
    E[1] = 1e4
    B[2] = 1e4 * (1 - delta)
    u = np.zeros((3, 5))
    dt = np.pi / 32
    one = pt.analytic(u, E, B, qm, dt)
    two = pt.analytic(pt.analytic(u, E, B, qm, dt / 2), E, B, qm, dt / 2)
    assert np.allclose(one, two, rtol=1e-9, atol=0)
    back = pt.analytic(one, E, B, qm, -dt)
    assert np.max(np.abs(back - u)) <= 1e-9 * np.max(np.abs(one))


def test_pure_magnetic_field_rotation():
    """|u| is conserved; the rotation angle is q B dt/gamma for the exact
    pusher and 2 arctan(q B dt/(2 gamma)) for Boris."""
    g = np.random.default_rng(2)
    npart = 16
    B = np.zeros((3, npart))
    B[2] = g.uniform(1, 50, npart)
    u = np.zeros((3, npart))
    u[0] = g.uniform(0.1, 30, npart)
    E = np.zeros_like(B)
    qm, dt = -1.0, 0.1
    gam = np.sqrt(1 + u[0] ** 2)
    for push, angle in ((pt.analytic, qm * B[2] * dt / gam),
                        (pt.boris, 2 * np.arctan(qm * B[2] * dt / (2 * gam)))):
        un = push(u, E, B, qm, dt)
        assert np.allclose(np.linalg.norm(un, axis=0), u[0], rtol=1e-13)
        got = np.arctan2(un[1], un[0])
        # u x B with B along z rotates u clockwise for positive qm B
        assert np.allclose(got, -angle, rtol=1e-11, atol=1e-13)


def test_higuera_cary_magnetic_rotation_keeps_speed():
    """Higuera-Cary in a pure B field (any orientation of u and B): a
    rotation, so |u| is kept to roundoff."""
    g = np.random.default_rng(3)
    u = g.standard_normal((3, 32)) * g.uniform(0.1, 30, 32)
    B = g.standard_normal((3, 32)) * g.uniform(1, 50, 32)
    un = pt.higuera_cary(u, np.zeros_like(B), B, -1.0, 0.1)
    assert np.allclose(np.linalg.norm(un, axis=0), np.linalg.norm(u, axis=0), rtol=1e-13)


@pytest.mark.parametrize("vd", [0.5, 0.9, 0.99])
def test_higuera_cary_keeps_relativistic_exb_drift(vd):
    """The property the paper cites the Higuera-Cary pusher for (Sec. 4.1:
    right for relativistically drifting particles): in crossed fields with
    |E| < |B| a particle moving at the E x B drift v_d = E x B / B^2 has
    constant u = gamma_d v_d, and the push keeps it over 50 steps to
    roundoff for any orientation; Boris does not."""
    g = np.random.default_rng(4)
    Bv = g.standard_normal(3)
    Bv *= 3.0 / np.linalg.norm(Bv)
    e = np.cross(Bv, g.standard_normal(3))
    Ev = e / np.linalg.norm(e) * vd * 3.0  # E perpendicular to B, |E| = v_d |B|
    v = np.cross(Ev, Bv) / (Bv @ Bv)
    u0 = (v / np.sqrt(1 - v @ v))[:, None]
    E, B = Ev[:, None], Bv[:, None]
    u = u0.copy()
    ub = u0.copy()
    for _ in range(50):
        u = pt.higuera_cary(u, E, B, -1.0, 0.2)
        ub = pt.boris(ub, E, B, -1.0, 0.2)
    assert np.max(np.abs(u - u0)) <= 1e-12 * np.max(np.abs(u0))
    assert np.max(np.abs(ub - u0)) > 1e-5 * np.max(np.abs(u0))


def test_null_field_from_rest():
    """E along x2, B = |E| along x3 (a plane-wave-like null field, F^3 = 0):
    from rest the exact solution has u2 + u2^3/6 = q E t, u1 = u2^2/2."""
    E0 = np.array([1.0, 10.0, 300.0, 1e4])
    npart = E0.size
    E = np.zeros((3, npart)); E[1] = E0
    B = np.zeros((3, npart)); B[2] = E0
    u = np.zeros((3, npart))
    qm, dt = -1.0, 0.05
    un = pt.analytic(u, E, B, qm, dt)
    s = un[1]
    assert np.allclose(s + s ** 3 / 6, qm * E0 * dt, rtol=1e-12)
    assert np.allclose(un[0], s * s / 2, rtol=1e-12)


def test_analytic_semigroup_and_reversal():
    """Exact map properties: two dt/2 pushes equal one dt push, and a -dt
    push undoes a dt push."""
    g = np.random.default_rng(3)
    npart = 24
    E, B = _rand_fields(npart, 4, scale=20.0)
    u = g.standard_normal((3, npart)) * 5
    qm, dt = -1.0, 0.1
    one = pt.analytic(u, E, B, qm, dt)
    two = pt.analytic(pt.analytic(u, E, B, qm, dt / 2), E, B, qm, dt / 2)
    assert np.allclose(one, two, rtol=1e-11, atol=1e-11)
    back = pt.analytic(one, E, B, qm, -dt)
    assert np.allclose(back, u, rtol=1e-10, atol=1e-10)


def test_analytic_matches_ode_integration():
    """The exact constant-field push against a tight adaptive integration of
    du/dt = q/m (E + u x B/gamma) in lab time (scipy DOP853)."""
    g = np.random.default_rng(5)
    npart = 8
    E, B = _rand_fields(npart, 6, scale=10.0)
    u = g.standard_normal((3, npart)) * 2
    qm, dt = -1.0, 0.1
    got = pt.analytic(u, E, B, qm, dt)
    for p in range(npart):
        def rhs(t, y):
            gam = np.sqrt(1 + y @ y)
            return qm * (E[:, p] + np.cross(y, B[:, p]) / gam)
        sol = scipy.integrate.solve_ivp(rhs, (0, dt), u[:, p], method="DOP853", rtol=1e-13, atol=1e-13)
        assert np.allclose(got[:, p], sol.y[:, -1], rtol=1e-10, atol=1e-10)


def test_position_update_and_wrap():
    """Sec. 4.1 position update x + dt u/gamma with the periodic wrap."""
    L = [4.0, 3.0, 2.0]
    x = np.array([[0.01, 3.99, 2.0], [0.5, 1.0, 2.999], [1.0, 0.0, 1.999]])
    u = np.array([[-1.0, 1.0, 0.0], [0.0, 0.0, 2.0], [0.0, -3.0, 1.0]])
    xn, disp = pt.advance_position(x, u, 0.1, L)
    g = np.sqrt(1 + np.sum(u * u, axis=0))
    raw = x + 0.1 * u / g
    assert np.allclose(disp, 0.1 * u / g)
    for d in range(3):
        assert np.all((xn[d] >= 0) & (xn[d] < L[d]))
        assert np.allclose(np.mod(raw[d], L[d]), xn[d])


@pytest.mark.parametrize("ndim", [2, 3])
def test_deposit_continuity(ndim):
    """Sec. 3.3: (rho^{n+1} - rho^n)/dt + d_Yee . J^{n+1/2} = 0 to roundoff
    for random sub-cell moves, including moves across the periodic seam."""
    n = (6, 5, 4 if ndim == 3 else 1)
    shape = (n[2], n[1], n[0])
    L = [n[d] * DX[d] for d in range(3)]
    x0, u = wl.uniform_particles(200, [0, 0, 0], L, seed=21, u_th=0.5)
    x0[0, :5] = 0.02 * DX[0]
    x1, _ = wl.small_moves(x0, DX, L, seed=22)
    q, w, dt = -1.0, 0.37, wl.DT
    J = pt.deposit(x0, x1, q, w, DX, dt, shape, ndim, u=u)
    rho0 = pt.charge_density(x0, q, w, DX, shape, ndim)
    rho1 = pt.charge_density(x1, q, w, DX, shape, ndim)
    div = fdtd.div_ampere(J, [1.0], DX)
    res = (rho1 - rho0) / dt + div
    assert np.max(np.abs(res)) < 1e-12 * np.max(np.abs(rho1 - rho0) / dt)


def _hat_path_average(X0, dX, Y0, dY, a, b):
    """int_0^1 S(X0 + s dX - a) S(Y0 + s dY - b) ds for the linear hat
    S(t) = max(0, 1 - |t|), by three-point Gauss-Legendre on [0, 1] (exact:
    for a path that stays inside one cell the integrand is a quadratic)."""
    xg, wg = np.polynomial.legendre.leggauss(3)
    s = (xg + 1) / 2
    S = lambda t: np.maximum(0.0, 1.0 - np.abs(t))
    return float(np.sum(wg * S(X0 + s * dX - a) * S(Y0 + s * dY - b)) / 2)


def test_deposit_2d_out_of_plane_current():
    """Sec. 3.3 in 2D3V: the out-of-plane current of a particle is q w v3,
    v3 = u3/gamma^{n+1/2} (u3 alone would be wrong wherever gamma > 1), spread
    over the nodes by a weight that moves with the particle:
      * its sum is 1 (sum J3 = q w v3);
      * by the linear shape's reproduction of linear functions, its first
        moments are the midpoint of the path, X0 + dX/2 and Y0 + dY/2, and its
        mixed moment sum a b W is the path average of X Y,
        X0 Y0 + (X0 dY + Y0 dX)/2 + dX dY/3;
      * for a move inside one cell it equals the time average of the shape
        product along the straight path (checked per node by quadrature).
    Moves cross faces and the periodic seam; gamma is far from 1."""
    n = (8, 6, 1)
    shape = (1, n[1], n[0])
    L = [n[d] * DX[d] for d in range(2)]
    g = np.random.default_rng(5)
    q, w, dt = -1.0, 0.37, wl.DT
    inside = 0
    for trial in range(24):
        x0 = np.array([[g.random() * L[0]], [g.random() * L[1]], [0.0]])
        d = (2 * g.random(2) - 1) * (0.9 if trial % 2 else 0.2) * np.array(DX[:2])
        if trial == 0:
            x0[0, 0], d[0] = 0.02 * DX[0], -0.5 * DX[0]   # backwards across the seam
        x1 = x0.copy()
        x1[:2, 0] = np.mod(x0[:2, 0] + d, L)
        u = np.array([[4.0 * g.standard_normal()], [g.standard_normal()], [3.0 * g.standard_normal()]])
        J = pt.deposit(x0, x1, q, w, DX, dt, shape, 2, u=u)
        v3 = u[2, 0] / np.sqrt(1 + float(u[:, 0] @ u[:, 0]))
        qv = q * w * v3
        X0, Y0 = x0[0, 0] / DX[0], x0[1, 0] / DX[1]
        dX, dY = d[0] / DX[0], d[1] / DX[1]
        # node coordinates as the periodic image nearest to the path start
        ia, jb = np.arange(n[0]), np.arange(n[1])
        a = ia + n[0] * np.round((X0 - ia) / n[0])
        b = jb + n[1] * np.round((Y0 - jb) / n[1])
        W = J[2][0] / qv  # [jb, ia]
        assert abs(W.sum() - 1) < 1e-14
        assert abs(np.sum(W * a[None, :]) - (X0 + dX / 2)) < 1e-13
        assert abs(np.sum(W * b[:, None]) - (Y0 + dY / 2)) < 1e-13
        mixed = X0 * Y0 + (X0 * dY + Y0 * dX) / 2 + dX * dY / 3
        assert abs(np.sum(W * b[:, None] * a[None, :]) - mixed) < 1e-12
        if np.floor(X0) == np.floor(X0 + dX) and np.floor(Y0) == np.floor(Y0 + dY):
            inside += 1
            for j_ in range(n[1]):
                for i_ in range(n[0]):
                    ref = _hat_path_average(X0, dX, Y0, dY, a[i_], b[j_])
                    assert abs(W[j_, i_] - ref) < 1e-14, (trial, i_, j_)
    assert inside >= 3


def test_deposit_total_current_and_rest():
    """Sum of J_d over the grid is q w (displacement_d)/dt per particle; a
    particle that does not move deposits exactly zero."""
    n = (6, 5, 4)
    shape = (n[2], n[1], n[0])
    L = [n[d] * DX[d] for d in range(3)]
    x0, _ = wl.uniform_particles(1, [0, 0, 0], L, seed=23)
    x1, d = wl.small_moves(x0, DX, L, seed=24)
    q, w, dt = -1.0, 0.5, wl.DT
    J = pt.deposit(x0, x1, q, w, DX, dt, shape, 3)
    disp = pt.min_image(x1, x0, L)
    for c in range(3):
        assert np.isclose(J[c].sum(), q * w * disp[c, 0] / dt, rtol=1e-12)
    J0 = pt.deposit(x0, x0.copy(), q, w, DX, dt, shape, 3)
    assert all(np.all(j == 0) for j in J0)
