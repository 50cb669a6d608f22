"""GPU parity of the moving window along x1 (Sec. 4.1 single-particle runs):
pic_move_window against the oracle's physically shifted window (fields
bit-exact after undoing the ring origin, the same particles leaving, in the
same order), runs with steps and moves against the oracle, and the gamma0 = 20
drift of Sec. 4.1 over a long run against the closed-form trajectory."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import pic, trajectory, window  # noqa: E402
from paper_2004_03754_amd import binding as b, workloads as wl  # noqa: E402

torch = pytest.importorskip("torch")
from gpu_util import dev, host  # noqa: E402

# Sec. 4.1 grid: dt = 0.05, dx1 = 0.2 (r = 1/4), dx2 = 20
DX1, DX2, DT = 0.2, 20.0, 0.05
DX = (DX1, DX2, DX2)
GAMMA0 = 20.0
X_HEAD = 180.0


def _species(n, seed, npart):
    g = wl.rng(seed)
    n1, n2, n3 = n
    cell = g.integers(0, n1, npart)
    frac = 0.05 + 0.9 * g.random(npart)  # away from cell faces
    x = np.stack([(cell + frac) * DX1, n2 * DX2 * g.random(npart), n3 * DX2 * g.random(npart)])
    u = g.standard_normal((3, npart))
    return x, u


def _ring_to_window(f, origin):
    return np.roll(f, -origin, axis=-1)


def _window_x1(x1, origin, L1):
    return np.mod(x1 - origin * DX1, L1)


@pytest.mark.parametrize("n,ndim", [((192, 5, 1), 2), ((128, 6, 3), 3)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_moves_match_oracle(n, ndim, prec):
    """A sequence of moves (37, 1, 0, 90, n1 - 1 cells) with J attached: the
    fields seen through the ring origin equal the oracle's shifted fields
    exactly, and the same particles are left, in the same order."""
    n1, n2, n3 = n
    dt_ = torch.float64 if prec == "fp64" else torch.float32
    E, B = wl.random_fields(n, seed=81)
    J = list(wl.random_fields(n, seed=82)[0])
    Ed, Bd, Jd = [dev(e, dt_) for e in E], [dev(x, dt_) for x in B], [dev(j, dt_) for j in J]
    # the oracle starts from exactly the values the GPU holds
    E, B, J = [host(e) for e in Ed], [host(x) for x in Bd], [host(j) for j in Jd]
    x, u = _species(n, 83, 2500)
    ids = np.arange(x.shape[1], dtype=np.int64)
    xd, ud, idd = dev(x), dev(u), dev(ids, torch.int64)
    if ndim == 2:
        xd[2].zero_()
        x[2] = 0.0
    c = np.zeros(1)
    c[0] = 1.0
    grid = b.Grid(Ed, Bd, DX, DT, c, c.copy(), J=Jd, prec=prec, ndim=ndim)
    p = b.Particles(xd, ud, id=idd)
    sp = dict(x=x.copy(), u=u.copy(), id=ids.copy(), q=-1.0, m=1.0, w=1.0)
    L1 = n1 * DX1
    for s in (37, 1, 0, 90, n1 - 1):
        print(f"window move {prec} {n} by {s}", flush=True)
        grid.move_window(s, [p])
        grid.sync()
        E, B, J = window.move(E, B, [sp], s, DX1, J=J)
        origin, moved = grid.window()
        assert origin == (moved % n1)
        for got, ref in zip(Ed + Bd + Jd, E + B + J):
            np.testing.assert_array_equal(_ring_to_window(host(got), origin), ref)
        assert p.np == sp["id"].size
        xg, ug, ig = (host(t) if t.dtype != torch.int64 else t.cpu().numpy() for t in p.live())
        np.testing.assert_array_equal(ig, sp["id"])
        np.testing.assert_allclose(_window_x1(xg[0], origin, L1), sp["x"][0], rtol=0, atol=1e-12 * L1)
        np.testing.assert_array_equal(xg[1:], sp["x"][1:])
        np.testing.assert_array_equal(ug, sp["u"])
    assert p.np < 2500
    grid.close()


def test_move_edge_cases():
    n = (128, 2, 1)
    E, B = wl.random_fields(n, seed=84)
    Ed, Bd = [dev(e) for e in E], [dev(x) for x in B]
    c = np.zeros(1)
    c[0] = 1.0
    grid = b.Grid(Ed, Bd, DX, DT, c, c.copy(), ndim=2)
    x = np.zeros((3, 300))
    x[0] = (np.arange(300) % 10 + 0.5) * DX1  # every particle in columns 0..9
    p = b.Particles(dev(x), dev(np.ones((3, 300))), id=dev(np.arange(300), torch.int64))
    for bad in (-1, 128, 1000):
        with pytest.raises(b.YeePICError):
            grid.move_window(bad, [p])
    print("window edge cases", flush=True)
    grid.move_window(0, [p])
    assert grid.window() == (0, 0) and p.np == 300
    grid.move_window(5, [])  # fields only: particles untouched
    assert grid.window() == (5, 5) and p.np == 300
    grid.move_window(5, [p])  # columns 5..9: half of them leave
    assert p.np == 150
    np.testing.assert_array_equal(p.live()[2].cpu().numpy(), np.flatnonzero(np.arange(300) % 10 < 5))
    grid.move_window(123, [p])  # columns 10..132 mod 128 = 0..4 as well: all leave
    assert p.np == 0 and grid.window() == (5, 133)
    grid.move_window(3, [p])  # an empty species is fine
    assert p.np == 0
    grid.sync()
    # the vacated columns are zero, the rest untouched
    o, _ = grid.window()
    got = _ring_to_window(host(Ed[1]), o)
    ref = window.shift_field(window.shift_field(window.shift_field(E[1], 10), 123), 3)
    np.testing.assert_array_equal(got, ref)
    grid.close()


def test_compaction_many_blocks_bit_exact():
    """1,000,003 particles (977 blocks, ragged tail): the survivors and their
    order equal the column rule evaluated on the host in the same precision."""
    n1 = 256
    n = (n1, 8, 1)
    E, B = wl.random_fields(n, seed=85)
    c = np.zeros(1)
    c[0] = 1.0
    grid = b.Grid([dev(e) for e in E], [dev(x) for x in B], DX, DT, c, c.copy(), ndim=2)
    g = wl.rng(86)
    npart = 1_000_003
    x = np.zeros((3, npart))
    x[0] = g.random(npart) * n1 * DX1
    x[1] = g.random(npart) * 8 * DX2
    ids = np.arange(npart, dtype=np.int64)
    p = b.Particles(dev(x), dev(g.standard_normal((3, npart))), id=dev(ids, torch.int64))
    origin = 0
    keep = np.ones(npart, dtype=bool)
    for s in (1, 7, 200):
        print(f"window compaction {npart} by {s}", flush=True)
        grid.move_window(s, [p])
        col = np.clip(np.floor(x[0] * (1.0 / DX1)), 0, n1 - 1).astype(np.int64)
        keep &= np.mod(col - origin, n1) >= s
        origin = (origin + s) % n1
        assert p.np == int(keep.sum())
        np.testing.assert_array_equal(p.live()[2].cpu().numpy(), ids[keep])
        np.testing.assert_array_equal(host(p.live()[0]), x[:, keep])
    grid.close()


def _suite_fields(n1, n2, pulse):
    return wl.laser_fields((n1, n2, 1), DX, pulse, x_head=X_HEAD)


def test_window_run_matches_oracle(coeffs16_quarter):
    """400 steps of the Sec. 4.1 configuration (proposed solver at r = 1/4,
    Higuera-Cary pusher, window moving at c: one cell every 4 steps) with the
    gamma0 = 20 electron and a few electrons at rest near the back edge, which
    leave the window: fields through the ring origin and the particles still
    inside agree with the oracle to 1e-12."""
    CE, CB = coeffs16_quarter
    n1, n2 = 1024, 4
    pulse = wl.FlatTopPulse(0.5)
    E, B = _suite_fields(n1, n2, pulse)
    xp = X_HEAD - (pulse.R + 16 * np.pi)
    x = np.zeros((3, 9))
    x[0] = [xp, 0.13, 0.31, 0.52, 0.77, 1.11, 1.9, 4.3, 9.0]
    x[1] = 0.5 * DX2
    u = np.zeros((3, 9))
    u[0, 0] = np.sqrt(GAMMA0 ** 2 - 1)
    ids = np.arange(9, dtype=np.int64)
    Ed, Bd = [dev(e) for e in E], [dev(v) for v in B]
    grid = b.Grid(Ed, Bd, DX, DT, CE, CB, ndim=2)
    p = b.Particles(dev(x), dev(u), id=dev(ids, torch.int64))
    sp = dict(x=x.copy(), u=u.copy(), id=ids.copy(), q=-1.0, m=1.0, w=1.0)
    moved = 0
    nsteps = 400
    print("window run 400 steps", flush=True)
    for n in range(nsteps):
        E, B = pic.step(E, B, [sp], CE, CB, DX, DT, pusher="hc", ndim=2)
        due = window.cells_due(n + 1, DT, DX1)
        if due > moved:
            E, B = window.move(E, B, [sp], due - moved, DX1)
            moved = due
    for k in range(nsteps // 4):
        grid.step_n([p], 4, pusher="hc")
        grid.move_window(1, [p])
    grid.sync()
    origin, gmoved = grid.window()
    assert gmoved == moved == 100
    for got, ref in zip(Ed + Bd, E + B):
        g_ = _ring_to_window(host(got), origin)
        assert np.max(np.abs(g_ - ref)) <= 1e-12 * max(np.max(np.abs(r)) for r in E + B)
    assert p.np == sp["id"].size and p.np < 9
    xg, ug, ig = p.live()
    np.testing.assert_array_equal(ig.cpu().numpy(), sp["id"])
    L1 = n1 * DX1
    np.testing.assert_allclose(_window_x1(host(xg)[0], origin, L1), sp["x"][0], rtol=0, atol=1e-12 * L1)
    np.testing.assert_allclose(host(ug), sp["u"], rtol=0, atol=1e-12 * GAMMA0)
    grid.close()


def _suite_gpu(CE, CB, a0, nsteps, prec="fp64"):
    n1, n2 = 1024, 4
    pulse = wl.FlatTopPulse(a0)
    E, B = _suite_fields(n1, n2, pulse)
    dt_ = torch.float64 if prec == "fp64" else torch.float32
    Ed, Bd = [dev(e, dt_) for e in E], [dev(v, dt_) for v in B]
    grid = b.Grid(Ed, Bd, DX, DT, CE, CB, prec=prec, ndim=2)
    xp = X_HEAD - (pulse.R + 16 * np.pi)
    x = np.array([[xp], [0.5 * DX2], [0.0]])
    u = np.array([[np.sqrt(GAMMA0 ** 2 - 1)], [0.0], [0.0]])
    p = b.Particles(dev(x), dev(u))
    for _ in range(nsteps // 4):
        grid.step_n([p], 4, pusher="hc")
        grid.move_window(1, [p])
    grid.sync()
    origin, moved = grid.window()
    E2 = _ring_to_window(host(Ed[1]), origin)
    x1 = host(p.x)[0, 0] - origin * DX1
    x1 = x1 + n1 * DX1 if x1 < 0 else x1
    out = dict(x1=moved * DX1 + x1, u=host(p.u)[:, 0], E2=E2, E2_0=E[1], xp=xp, pulse=pulse)
    grid.close()
    return out


@pytest.mark.parametrize("a0", [0.5, 3.0])
def test_single_particle_suite_long_run(a0, coeffs16_quarter):
    """20,000 steps (t = 1000, 5,000 window moves) of the gamma0 = 20 drift:
    the proposed solver follows the closed-form trajectory, the plane wave
    keeps its shape in the window, and the Yee solver departs from both."""
    CE, CB = coeffs16_quarter
    nsteps = 20000
    T = nsteps * DT
    print(f"single-particle suite a0={a0}", flush=True)
    r = _suite_gpu(CE, CB, a0, nsteps)
    pulse = r["pulse"]
    x0 = np.array([[r["xp"]], [0.0], [0.0]])
    a = lambda s: pulse.a(X_HEAD + s)  # noqa: E731
    x_th, _, _ = trajectory.state_at(a, -1.0, 0.0, x0, T, gamma0=GAMMA0)
    _, u_th, _ = trajectory.state_at(a, -1.0, 0.0, x0, T - DT / 2, gamma0=GAMMA0)
    err_u2 = abs(r["u"][1] - u_th[1, 0])
    err_x1 = abs(r["x1"] - x_th[0, 0])
    err_f = np.max(np.abs(r["E2"] - r["E2_0"])) / np.max(np.abs(r["E2_0"]))
    print(f"proposed: u2 {r['u'][1]:.6f} theory {u_th[1, 0]:.6f} x1 err {err_x1:.2e} field err {err_f:.2e}")
    assert err_u2 <= 5e-3 * a0
    assert err_x1 <= 3e-6 * x_th[0, 0]
    assert err_f <= 1e-5
    yee = np.zeros(16)
    yee[0] = 1.0
    ry = _suite_gpu(yee, yee.copy(), a0, nsteps)
    err_u2y = abs(ry["u"][1] - u_th[1, 0])
    err_fy = np.max(np.abs(ry["E2"] - ry["E2_0"])) / np.max(np.abs(ry["E2_0"]))
    print(f"yee: u2 {ry['u'][1]:.6f} field err {err_fy:.2e}")
    assert err_u2y >= 10 * err_u2
    assert err_fy >= 1e-1


def _trace_run(CE, CB, a0, nsteps):
    """The single-particle run, sampling u2, gamma and the phase xi = x1 - t
    (lab frame) after every window move."""
    n1 = 1024
    pulse = wl.FlatTopPulse(a0)
    E, B = _suite_fields(n1, 4, pulse)
    grid = b.Grid([dev(e) for e in E], [dev(v) for v in B], DX, DT, CE, CB, ndim=2)
    xp = X_HEAD - (pulse.R + 16 * np.pi)
    p = b.Particles(dev(np.array([[xp], [0.5 * DX2], [0.0]])),
                    dev(np.array([[np.sqrt(GAMMA0 ** 2 - 1)], [0.0], [0.0]])))
    u2, gam, xi = [], [], []
    for k in range(nsteps // 4):
        grid.step_n([p], 4, pusher="hc")
        grid.move_window(1, [p])
        u = host(p.u)[:, 0]
        origin, moved = grid.window()
        xw = float(host(p.x)[0, 0]) - origin * DX1
        xw = xw + n1 * DX1 if xw < 0 else xw
        u2.append(u[1])
        gam.append(np.sqrt(1.0 + u @ u))
        xi.append(moved * DX1 + xw - (k + 1) * 4 * DT)
    grid.close()
    t = (np.arange(len(u2)) + 1) * 4 * DT
    return t, np.array(u2), np.array(gam), np.array(xi), xp


def test_four_solver_comparison():
    """Sec. 4.1, first case (gamma0 = 20, a0 = 0.5, r = 1/4, Higuera-Cary,
    window at c) with the four solvers of the comparison over t = 6000, about
    one full oscillation of p2.  The closed form gives p2 = a_L between -a0 and
    a0, gamma_max = (1 + a0^2 + h^2)/2h and the first p2 maximum at
    t = (pi/2)(1 + h^2 + a0^2/2)/(2 h^2).  What the paper reports, checked:
    only the proposed solver keeps p2 within +-a0 and the energy gain at the
    theory (the others overestimate it); Xu's period agrees with the theory
    but its amplitude is larger than the proposed solver's (the time-stagger
    error); the Yee-type solvers dephase less at first and have much longer
    p2 periods."""
    r = DT / DX1
    a0 = 0.5
    nsteps = 120000
    h = GAMMA0 - np.sqrt(GAMMA0 ** 2 - 1)
    g_max = (1 + a0 ** 2 + h ** 2) / (2 * h)
    t_first_max = (np.pi / 2) * (1 + h ** 2 + a0 ** 2 / 2) / (2 * h ** 2)
    one = np.ones(1)
    solvers = {"yee": (one, one.copy()),
               "xu": (b.design_coeffs(16, r, "xu"), b.design_coeffs(16, r, "xu")),
               "yee_t": (b.design_coeffs(16, r, "yeet_E"), b.design_coeffs(16, r, "yeet_B")),
               "proposed": (b.design_coeffs(16, r, "E"), b.design_coeffs(16, r, "B"))}
    res = {}
    for name, (CE, CB) in solvers.items():
        print(f"four-solver run: {name}", flush=True)
        t, u2, gam, xi, xp = _trace_run(CE, CB, a0, nsteps)
        i_mid = np.searchsorted(t, 3000.0)
        imax = int(np.argmax(u2))
        down = np.flatnonzero((u2[imax:-1] > 0) & (u2[imax + 1:] <= 0))
        res[name] = dict(u2max=u2.max(), u2min=u2.min(), gmax=gam.max(), t_max=t[imax],
                         t_down=t[imax + down[0]] if down.size else np.inf, deph_mid=xp - xi[i_mid])
        print(name, {k: round(float(v), 5) for k, v in res[name].items()}, flush=True)
    p, xu, yee, yt = res["proposed"], res["xu"], res["yee"], res["yee_t"]
    # proposed: the closed form's amplitude, energy and period
    assert abs(p["u2max"] - a0) <= 1e-2 * a0 and abs(p["u2min"] + a0) <= 1e-2 * a0
    assert abs(p["gmax"] - g_max) <= 5e-3 * g_max
    assert abs(p["t_max"] - t_first_max) <= 5e-3 * t_first_max
    # every other solver overestimates the energy gain
    for other in (xu, yee, yt):
        assert other["gmax"] >= g_max * 1.02
    # Xu: the period of the corrected dispersion, the amplitude of the time-stagger error
    assert abs(xu["t_max"] - t_first_max) <= 3e-2 * t_first_max
    assert abs(xu["t_down"] - p["t_down"]) <= 3e-2 * p["t_down"]
    assert xu["u2max"] >= 1.1 * a0
    # Yee-type: smaller dephasing at first, much longer p2 period
    for yy in (yee, yt):
        assert yy["deph_mid"] <= 0.9 * min(p["deph_mid"], xu["deph_mid"])
        assert yy["t_max"] >= 2.5 * t_first_max


def _claims_run(CE, CB, pusher, a0, gamma0, T, samples):
    """The single-particle run from rest (gamma0 None) or with a drift;
    returns (xi, gamma) at the sample step counts (multiples of 4)."""
    n1 = 1024
    pulse = wl.FlatTopPulse(a0)
    E, B = _suite_fields(n1, 4, pulse)
    grid = b.Grid([dev(e) for e in E], [dev(v) for v in B], DX, DT, CE, CB, ndim=2)
    xp = X_HEAD - (pulse.R + 16 * np.pi)
    a = lambda s: pulse.a(X_HEAD + s)  # noqa: E731
    if gamma0 is None:
        # at rest at t = -dt/2 (u^{-1/2} = 0): x^0 from the closed form
        x0, _, _ = trajectory.state_at(a, -1.0, -DT / 2, np.array([[xp], [0.5 * DX2], [0.0]]), 0.0)
        u0 = np.zeros((3, 1))
    else:
        x0 = np.array([[xp], [0.5 * DX2], [0.0]])
        u0 = np.array([[np.sqrt(gamma0 ** 2 - 1)], [0.0], [0.0]])
    p = b.Particles(dev(x0), dev(u0))
    out = []
    want = set(int(s) for s in samples)
    for k in range(1, max(want) // 4 + 1):
        grid.step_n([p], 4, pusher=pusher)
        grid.move_window(1, [p])
        if 4 * k in want:
            u = host(p.u)[:, 0]
            origin, moved = grid.window()
            xw = float(host(p.x)[0, 0]) - origin * DX1
            xw = xw + n1 * DX1 if xw < 0 else xw
            out.append((moved * DX1 + xw - 4 * k * DT, np.sqrt(1.0 + u @ u)))
    grid.close()
    return np.array(out), x0


def _claims_theory(a0, gamma0, x0, samples):
    pulse = wl.FlatTopPulse(a0)
    a = lambda s: pulse.a(X_HEAD + s)  # noqa: E731
    t0 = -DT / 2 if gamma0 is None else 0.0
    xs = x0 if gamma0 is not None else np.array([[X_HEAD - (pulse.R + 16 * np.pi)], [0.0], [0.0]])
    th = []
    for n in samples:
        t = n * DT
        x, _, _ = trajectory.state_at(a, -1.0, t0, xs, t, gamma0=gamma0)
        _, _, g = trajectory.state_at(a, -1.0, t0, xs, t - DT / 2, gamma0=gamma0)
        th.append((x[0, 0] - t, g[0]))
    return np.array(th)


def test_sec41_solver_and_pusher_comparisons():
    """The rest of the Sec. 4.1 single-particle runs, window at c, r = 1/4,
    errors of xi = x1 - t and gamma against the closed form at 8 times.  What
    the paper reports and these runs reproduce: from rest at a0 = 10 (HC) the
    Yee-type solvers deviate, Xu does better and the proposed solver best; at
    a0 = 100, 1000 and 10^4 only the analytic pusher (with the proposed
    solver) gives the closed-form energy, Boris and HC do not; with a
    gamma0 = 20 drift at a0 = 100 the proposed solver is exact to plotting
    accuracy with HC and with the analytic pusher, while Yee is far off even
    with the analytic pusher, and at a0 = 10^4 HC and analytic err alike and
    Yee much more."""
    r = DT / DX1
    one = np.ones(1)
    solvers = {"yee": (one, one.copy()),
               "xu": (b.design_coeffs(16, r, "xu"), b.design_coeffs(16, r, "xu")),
               "yee_t": (b.design_coeffs(16, r, "yeet_E"), b.design_coeffs(16, r, "yeet_B")),
               "proposed": (b.design_coeffs(16, r, "E"), b.design_coeffs(16, r, "B"))}

    def errs(solver, pusher, a0, gamma0, T):
        nsteps = int(round(T / DT))
        samples = (np.linspace(nsteps // 8, nsteps, 8) // 4 * 4).astype(int)
        print(f"sec 4.1 run: {solver} {pusher} a0={a0} gamma0={gamma0}", flush=True)
        got, x0 = _claims_run(*solvers[solver], pusher, a0, gamma0, T, samples)
        th = _claims_theory(a0, gamma0, x0, samples)
        e = (float(np.max(np.abs(got[:, 0] - th[:, 0]))), float(np.max(np.abs(got[:, 1] - th[:, 1]) / th[:, 1])),
             float(abs(got[-1, 1] - th[-1, 1]) / th[-1, 1]))
        print(f"  xi err {e[0]:.4f} gamma rel err {e[1]:.4f} final gamma rel err {e[2]:.4f}", flush=True)
        return e

    # from rest, a0 = 10, Higuera-Cary: the solver ranking of the xi error
    e10 = {s: errs(s, "hc", 10.0, None, 400.0)[0] for s in solvers}
    assert e10["proposed"] < e10["xu"] < min(e10["yee"], e10["yee_t"])
    assert e10["proposed"] <= 0.6 and min(e10["yee"], e10["yee_t"]) >= 1.0
    # from rest, a0 = 100 .. 10^4, proposed solver: only the analytic pusher
    for a0, T in ((100.0, 400.0), (1000.0, 200.0), (10000.0, 200.0)):
        # gamma ~ 1 + (a0 (psi - psi0))^2/2 with psi - psi0 of order
        # (6 t/a0^2)^(1/3) (0.02 at a0 = 10^4, t = 200), so its relative error
        # is twice that of the phase: a phase error of 3e-4 is already 3 % in
        # gamma.  The phase error bounds the analytic pusher, the energy at
        # the end of the run separates the pushers.
        e = {pu: errs("proposed", pu, a0, None, T) for pu in ("boris", "hc", "analytic")}
        assert e["analytic"][0] <= 1e-2
        assert min(e["boris"][0], e["hc"][0]) >= 3 * e["analytic"][0]
        assert e["analytic"][2] <= 0.2 * min(e["boris"][2], e["hc"][2])
    # gamma0 = 20 drift
    d_hc = errs("proposed", "hc", 100.0, 20.0, 400.0)
    d_an = errs("proposed", "analytic", 100.0, 20.0, 400.0)
    d_yee = errs("yee", "analytic", 100.0, 20.0, 400.0)
    assert max(d_hc[1], d_an[1]) <= 1e-2 and max(d_hc[0], d_an[0]) <= 1e-2
    assert d_yee[1] >= 0.5
    h_hc = errs("proposed", "hc", 10000.0, 20.0, 400.0)
    h_an = errs("proposed", "analytic", 10000.0, 20.0, 400.0)
    h_yee = errs("yee", "analytic", 10000.0, 20.0, 400.0)
    assert 0.5 <= h_hc[1] / h_an[1] <= 2.0
    assert h_yee[1] >= 5 * max(h_hc[1], h_an[1])


def test_window_with_plasma_steps_matches_oracle(coeffs16):
    """Moves between plasma steps (3D, deposit on, particles sorted by tile
    and their current accumulated on chip): fields through the ring origin
    and the surviving particles (by id) agree with the oracle's shifted
    window to 1e-12 after 12 steps and 3 moves of 2 cells."""
    CE, CB = coeffs16
    n = (128, 8, 8)
    dx = (wl.DX1, wl.DX2, wl.DX3)
    E, B = wl.random_fields(n, seed=91, scale=0.05)
    L = [n[0] * dx[0], n[1] * dx[1], n[2] * dx[2]]
    x, u = wl.uniform_particles(3000, [0, 0, 0], L, seed=92, u_th=0.2)
    ids = np.arange(x.shape[1], dtype=np.int64)
    Ed, Bd = [dev(e) for e in E], [dev(v) for v in B]
    Jd = [dev(np.zeros_like(E[0])) for _ in range(3)]
    grid = b.Grid(Ed, Bd, dx, wl.DT, CE, CB, J=Jd)
    p = b.Particles(dev(x), dev(u), q=-1.0, m=1.0, w=1e-3, id=dev(ids, torch.int64))
    sp = dict(x=x.copy(), u=u.copy(), id=ids.copy(), q=-1.0, m=1.0, w=1e-3)
    print("window with plasma steps", flush=True)
    for _ in range(3):
        for _ in range(4):
            E, B = pic.step(E, B, [sp], CE, CB, dx, wl.DT, pusher="boris", deposit=True, ndim=3)
        E, B = window.move(E, B, [sp], 2, wl.DX1)
        grid.step_n([p], 4, pusher="boris", deposit=True)
        grid.move_window(2, [p])
    grid.sync()
    origin, moved = grid.window()
    assert moved == 6
    scale = max(np.max(np.abs(f)) for f in E + B)
    for got, ref in zip(Ed + Bd, E + B):
        assert np.max(np.abs(_ring_to_window(host(got), origin) - ref)) <= 1e-12 * scale
    xg, ug, ig = p.live()
    ig = ig.cpu().numpy()
    assert p.np == sp["id"].size < 3000
    order = np.argsort(ig)
    np.testing.assert_array_equal(ig[order], np.sort(sp["id"]))
    ref_order = np.argsort(sp["id"])
    xw = host(xg)[:, order]
    xw[0] = np.mod(xw[0] - origin * wl.DX1, L[0])
    np.testing.assert_allclose(xw, sp["x"][:, ref_order], rtol=0, atol=1e-12 * max(L))
    np.testing.assert_allclose(host(ug)[:, order], sp["u"][:, ref_order], rtol=0, atol=1e-12)
    grid.close()
