"""GPU parity of the hand-written adjoint (pic_adjoint_step and the
checkpointed autograd Function) against the oracle's autograd gradients,
plus dot-product, recomputation and finite-difference checks."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import adjoint as ad, pic  # noqa: E402
from paper_2004_03754_amd import binding as b, workloads as wl  # noqa: E402

torch = pytest.importorskip("torch")
from gpu_util import check, dev, host  # noqa: E402

DX = (wl.DX1, wl.DX2, wl.DX3)
QM = -1.0


def _t(a):
    return torch.tensor(np.asarray(a), dtype=torch.float64)


def _case(n, seed, npart, ndim, scale=0.3, u_th=0.3):
    E, B = wl.random_fields(n, seed=seed, scale=scale)
    L = [n[d] * DX[d] for d in range(3)]
    x, u = wl.uniform_particles(npart, [0, 0, 0], L, seed=seed + 1, u_th=u_th)
    if ndim == 2:
        x[2] = 0.5
    return E, B, x, u


def _cotangents(n, npart, seed):
    g = np.random.default_rng(seed)
    shape = (n[2], n[1], n[0])
    lE = [g.standard_normal(shape) for _ in range(3)]
    lB = [g.standard_normal(shape) for _ in range(3)]
    return lE, lB, g.standard_normal((3, npart)), g.standard_normal((3, npart))


def _oracle_vjp(E, B, x, u, CE, CB, lE, lB, lx, lu, ndim, nsteps=1, pusher="boris"):
    """Autograd of <lambda, state after nsteps> with respect to the initial
    state and the coefficients (oracle, CPU FP64)."""
    n3, n2, n1 = E[0].shape
    leaves = [_t(a).requires_grad_() for a in list(E) + list(B)] + [_t(x).requires_grad_(),
                                                                    _t(u).requires_grad_(),
                                                                    _t(CE).requires_grad_(),
                                                                    _t(CB).requires_grad_()]
    Ef, Bf, xf, uf = ad.run(leaves[:3], leaves[3:6], leaves[6], leaves[7], leaves[8], leaves[9], DX, wl.DT, QM,
                            nsteps, ndim, pusher)
    L = sum(torch.sum(a * _t(l)) for a, l in zip(list(Ef) + list(Bf), list(lE) + list(lB)))
    L = L + torch.sum(xf * _t(lx)) + torch.sum(uf * _t(lu))
    g = torch.autograd.grad(L, leaves)
    return [a.numpy() for a in g]


def _rel(got, ref):
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))


@pytest.mark.parametrize("ndim,n,npart,pusher,scale", [(3, (64, 6, 5), 200, "boris", 0.3),
                                                        (2, (128, 9, 1), 150, "boris", 0.3),
                                                        (3, (64, 6, 5), 200, "analytic", 0.3),
                                                        (2, (128, 9, 1), 150, "analytic", 0.3),
                                                        (3, (64, 6, 5), 200, "analytic", 40.0)])
def test_adjoint_step_matches_oracle(ndim, n, npart, pusher, scale, coeffs16):
    """One reverse step: field, position, momentum and coefficient
    cotangents equal the oracle's autograd VJP to 1e-12 (norm-wise).  The
    exact pusher is taken in weak fields (its series branch) and in fields
    of 40 (the hyperbolic and trigonometric branch)."""
    CE, CB = coeffs16
    E, B, x, u = _case(n, 11, npart, ndim, scale=scale)
    lE, lB, lx, lu = _cotangents(n, npart, 12)
    ref = _oracle_vjp(E, B, x, u, CE, CB, lE, lB, lx, lu, ndim, pusher=pusher)
    grid = b.Grid([dev(e) for e in E], [dev(v) for v in B], DX, wl.DT, CE, CB, ndim=ndim)
    p = b.Particles(dev(x), dev(u), q=QM, m=1.0)
    lEd, lBd = [dev(a) for a in lE], [dev(a) for a in lB]
    lxd, lud = dev(lx), dev(lu)
    lam = b.Particles(lxd, lud, q=QM, m=1.0)
    gCE = torch.zeros(16, dtype=torch.float64, device="cuda:0")
    gCB = torch.zeros(16, dtype=torch.float64, device="cuda:0")
    grid.adjoint_step(lEd, lBd, gCE, gCB, [p], [lam], pusher=pusher)
    grid.sync()
    got = [host(a) for a in lEd + lBd] + [host(lxd), host(lud), host(gCE), host(gCB)]
    names = ["E1", "E2", "E3", "B1", "B2", "B3", "x", "u", "CE", "CB"]
    errs = {}
    for name, g_, r in zip(names, got, ref):
        if name == "x" and ndim == 2:
            g_, r = g_[:2], r[:2]
        errs[name] = _rel(g_, r)
    print(f"adjoint step {pusher} ndim={ndim} field scale {scale}: " +
          " ".join(f"{k} {v:.1e}" for k, v in errs.items()), flush=True)
    for name, e in errs.items():
        assert e <= 1e-12, (name, e)
    # the forward state is left untouched
    assert np.array_equal(host(grid.E[1]), E[1]) and np.array_equal(host(p.u), u)
    grid.close()


def test_field_adjoint_dot_product(coeffs16):
    """<S v, w> = <v, S^T w> for the fused field sweep S and the adjoint
    field step (no particles), 3D, to 1e-13 relative."""
    CE, CB = coeffs16
    n = (64, 7, 6)
    vE, vB = wl.random_fields(n, seed=21)
    wE, wB = wl.random_fields(n, seed=22)
    Ed, Bd = [dev(a) for a in vE], [dev(a) for a in vB]
    grid = b.Grid(Ed, Bd, DX, wl.DT, CE, CB)
    grid.sweep()
    Sv = [host(a) for a in Ed + Bd]
    grid.set_fields([dev(a) for a in vE], [dev(a) for a in vB])
    lE, lB = [dev(a) for a in wE], [dev(a) for a in wB]
    gC = torch.zeros(16, dtype=torch.float64, device="cuda:0")
    grid.adjoint_step(lE, lB, gC, gC.clone())
    grid.sync()
    STw = [host(a) for a in lE + lB]
    lhs = sum(float(np.vdot(a, c)) for a, c in zip(Sv, list(wE) + list(wB)))
    rhs = sum(float(np.vdot(a, c)) for a, c in zip(list(vE) + list(vB), STw))
    scale = sum(float(np.vdot(a, a)) for a in Sv) ** 0.5 * sum(float(np.vdot(a, a)) for a in wE + wB) ** 0.5
    assert abs(lhs - rhs) <= 1e-13 * scale
    grid.close()


def test_stacked_2d_planes_match_single_plane_oracle(coeffs16):
    """A 2D grid with n3 = 3 is three independent meshes: the forward step
    loop and one adjoint step on the stack equal the oracle run on each plane
    with that plane's particles."""
    CE, CB = coeffs16
    n1, n2, nb, npb = 128, 8, 3, 40
    planes = [_case((n1, n2, 1), 40 + k, npb, 2) for k in range(nb)]
    cots = [_cotangents((n1, n2, 1), npb, 60 + k) for k in range(nb)]
    E = [np.concatenate([pl[0][c] for pl in planes], 0) for c in range(3)]
    B = [np.concatenate([pl[1][c] for pl in planes], 0) for c in range(3)]
    x = np.concatenate([pl[2] for pl in planes], 1)
    x[2] = np.repeat(np.arange(nb) + 0.5, npb)
    u = np.concatenate([pl[3] for pl in planes], 1)
    # forward, 3 steps
    grid = b.Grid([dev(e) for e in E], [dev(v) for v in B], DX, wl.DT, CE, CB, ndim=2)
    xd, ud = dev(x), dev(u)
    grid.step_n([b.Particles(xd, ud, q=QM, m=1.0)], 3, pusher="boris")
    grid.sync()
    for k, (Ek, Bk, xk, uk) in enumerate(planes):
        sp = {"x": xk.copy(), "u": uk.copy(), "q": QM, "m": 1.0, "w": 1.0}
        Er, Br = pic.run(Ek, Bk, [sp], CE, CB, DX, wl.DT, 3, pusher="boris", ndim=2)
        for g_, r in zip(grid.E + grid.B, list(Er) + list(Br)):
            assert _rel(host(g_)[k:k + 1], r) <= 1e-12
        sl = slice(k * npb, (k + 1) * npb)
        assert np.max(np.abs(host(ud)[:, sl] - sp["u"])) <= 1e-12
        assert np.max(np.abs(host(xd)[:2, sl] - sp["x"][:2])) <= 1e-12
    # adjoint, one step from the initial state
    grid.set_fields([dev(e) for e in E], [dev(v) for v in B])
    p = b.Particles(dev(x), dev(u), q=QM, m=1.0)
    lE = [dev(np.concatenate([c[0][q] for c in cots], 0)) for q in range(3)]
    lB = [dev(np.concatenate([c[1][q] for c in cots], 0)) for q in range(3)]
    lxd = dev(np.concatenate([c[2] for c in cots], 1))
    lud = dev(np.concatenate([c[3] for c in cots], 1))
    gCE = torch.zeros(16, dtype=torch.float64, device="cuda:0")
    gCB = torch.zeros(16, dtype=torch.float64, device="cuda:0")
    grid.adjoint_step(lE, lB, gCE, gCB, [p], [b.Particles(lxd, lud, q=QM, m=1.0)])
    grid.sync()
    sumCE, sumCB = 0, 0
    for k, ((Ek, Bk, xk, uk), (lEk, lBk, lxk, luk)) in enumerate(zip(planes, cots)):
        ref = _oracle_vjp(Ek, Bk, xk, uk, CE, CB, lEk, lBk, lxk, luk, 2)
        for g_, r in zip(lE + lB, ref[:6]):
            assert _rel(host(g_)[k:k + 1], r) <= 1e-12
        sl = slice(k * npb, (k + 1) * npb)
        assert _rel(host(lxd)[:2, sl], ref[6][:2]) <= 1e-12
        assert _rel(host(lud)[:, sl], ref[7]) <= 1e-12
        sumCE, sumCB = sumCE + ref[8], sumCB + ref[9]
    assert _rel(host(gCE), sumCE) <= 1e-12 and _rel(host(gCB), sumCB) <= 1e-12
    grid.close()


def test_checkpoint_recompute_is_bit_exact(coeffs16):
    """Resuming from a checkpoint reproduces the uninterrupted run bit for
    bit: 7 steps in one call equal 7 calls of one step (vacuum, FP64)."""
    CE, CB = coeffs16
    n = (128, 8, 1)
    E, B, x, u = _case(n, 31, 100, 2, u_th=0.5)
    runs = []
    for chunks in ([7], [1] * 7):
        Ed, Bd = [dev(e) for e in E], [dev(v) for v in B]
        grid = b.Grid(Ed, Bd, DX, wl.DT, CE, CB, ndim=2)
        xd, ud = dev(x), dev(u)
        p = b.Particles(xd, ud, q=QM, m=1.0)
        for c in chunks:
            grid.step_n([p], c, pusher="boris")
        grid.sync()
        runs.append([host(a) for a in Ed + Bd + [xd, ud]])
        grid.close()
    for a, c in zip(*runs):
        assert np.array_equal(a, c)


def test_step_to_and_given_next_state(coeffs16):
    """pic_step_to writes exactly what pic_step_n computes (bit for bit), and
    an adjoint step given the t^{n+1} state equals one that recomputes it."""
    CE, CB = coeffs16
    n = (128, 8, 2)
    E, B, x, u = _case(n, 51, 60, 2, u_th=0.5)
    x[2] = np.repeat([0.5, 1.5], 30)
    Ed, Bd = [dev(e) for e in E], [dev(v) for v in B]
    grid = b.Grid(Ed, Bd, DX, wl.DT, CE, CB, ndim=2)
    xa, ua = dev(x), dev(u)
    Eo, Bo = [torch.empty_like(e) for e in Ed], [torch.empty_like(v) for v in Bd]
    grid.step_to([b.Particles(xa, ua, q=QM, m=1.0)], Eo, Bo)
    grid.sync()
    assert all(np.array_equal(host(a), c) for a, c in zip(Ed + Bd, list(E) + list(B)))  # inputs untouched
    Ec, Bc = [dev(e) for e in E], [dev(v) for v in B]
    g2 = b.Grid(Ec, Bc, DX, wl.DT, CE, CB, ndim=2)
    xb, ub = dev(x), dev(u)
    g2.step_n([b.Particles(xb, ub, q=QM, m=1.0)], 1)
    g2.sync()
    for a, c in zip(Eo + Bo + [xa, ua], Ec + Bc + [xb, ub]):
        assert torch.equal(a, c)
    lE, lB, lx, lu = _cotangents(n, 60, 52)
    outs = []
    for nxt in (None, (Eo, Bo)):
        grid.set_fields([dev(e) for e in E], [dev(v) for v in B])
        lEd, lBd, lxd, lud = [dev(a) for a in lE], [dev(a) for a in lB], dev(lx), dev(lu)
        gC = [torch.zeros(16, dtype=torch.float64, device="cuda:0") for _ in range(2)]
        kw = {} if nxt is None else {"next_E": nxt[0], "next_B": nxt[1]}
        grid.adjoint_step(lEd, lBd, gC[0], gC[1], [b.Particles(dev(x), dev(u), q=QM, m=1.0)],
                          [b.Particles(lxd, lud, q=QM, m=1.0)], **kw)
        grid.sync()
        outs.append([host(a) for a in lEd + lBd + [lxd, lud] + gC])
    for a, c in zip(*outs):
        assert _rel(a, c) <= 1e-13
    grid.close()
    g2.close()


@pytest.mark.parametrize("ampere", ["yee", "wide"])
def test_step_to_half_field_output(ampere, coeffs16):
    """pic_step_to's optional B^{n+1/2} equals the separate Faraday half step
    (pic_advance_B_half) from the same E^n, B^n; an adjoint step handed it
    equals one that rebuilds it.  "yee": the width-1 Ampere stencil (fused
    Yee sweep writes it from its first stage); "wide": a width-3 Ampere
    stencil (the general sweep, B^{n+1/2} from its own half step)."""
    CE, CB = coeffs16
    if ampere == "wide":
        CB = np.zeros(16)
        CB[:3] = [1.2, -0.1, 0.02]
    n = (256, 12, 3)
    E, B, x, u = _case(n, 61, 80, 3, u_th=0.5)
    grid = b.Grid([dev(e) for e in E], [dev(v) for v in B], DX, wl.DT, CE, CB)
    Eo, Bo = [torch.empty_like(grid.E[0]) for _ in range(3)], [torch.empty_like(grid.B[0]) for _ in range(3)]
    Bh = [torch.full_like(grid.B[0], np.nan) for _ in range(3)]
    print(f"step_to B_half: {ampere} Ampere stencil, {n}", flush=True)
    grid.step_to([b.Particles(dev(x), dev(u), q=QM, m=1.0)], Eo, Bo, B_half=Bh)
    grid.sync()
    ref = b.Grid([dev(e) for e in E], [dev(v) for v in B], DX, wl.DT, CE, CB)
    ref.advance_B_half()
    ref.sync()
    for a, c in zip(Bh, ref.B):
        assert _rel(host(a), host(c)) <= 1e-14
    lE, lB, lx, lu = _cotangents(n, 80, 62)
    outs = []
    for half in (None, Bh):
        grid.set_fields([dev(e) for e in E], [dev(v) for v in B])
        lEd, lBd, lxd, lud = [dev(a) for a in lE], [dev(a) for a in lB], dev(lx), dev(lu)
        gC = [torch.zeros(16, dtype=torch.float64, device="cuda:0") for _ in range(2)]
        grid.adjoint_step(lEd, lBd, gC[0], gC[1], [b.Particles(dev(x), dev(u), q=QM, m=1.0)],
                          [b.Particles(lxd, lud, q=QM, m=1.0)], next_E=Eo, next_B=Bo, half_B=half)
        grid.sync()
        outs.append([host(a) for a in lEd + lBd + [lxd, lud] + gC])
    for a, c in zip(*outs):
        assert _rel(a, c) <= 1e-13
    grid.close()
    ref.close()


def _run_autograd(CE, CB, E, B, x, u, cfg, w):
    from paper_2004_03754_amd import autograd as pa
    Ef, Bf, xf, uf = pa.run(CE, CB, E, B, x, u, cfg)
    g = torch.sqrt(1.0 + torch.sum(uf * uf, 0))
    return (torch.mean(g) + torch.sum((Ef[1] - w[0]) ** 2) / torch.sum(w[0] ** 2) + torch.sum(w[1] * Bf[2])
            + 0.1 * torch.sum(torch.sin(xf[0])))


@pytest.mark.parametrize("nsteps,K,pusher", [(10, 4, "boris"), (6, 64, "boris"), (10, 4, "analytic")])
def test_autograd_run_matches_oracle(nsteps, K, pusher, coeffs16):
    """The checkpointed Function (segments of K steps, recomputed and then
    reversed) gives the oracle's gradients of a scalar loss with respect to
    C^E, C^B, the initial fields and the particles (stacked 2D, 2 planes)."""
    from paper_2004_03754_amd import autograd as pa
    CE, CB = coeffs16
    n1, n2, nb, npb = 128, 8, 2, 30
    planes = [_case((n1, n2, 1), 70 + k, npb, 2, u_th=0.5) for k in range(nb)]
    g = np.random.default_rng(9)
    w = [g.standard_normal((nb, n2, n1)), g.standard_normal((nb, n2, n1))]
    E = [np.concatenate([pl[0][c] for pl in planes], 0) for c in range(3)]
    B = [np.concatenate([pl[1][c] for pl in planes], 0) for c in range(3)]
    x = np.concatenate([pl[2] for pl in planes], 1)
    x[2] = np.repeat(np.arange(nb) + 0.5, npb)
    u = np.concatenate([pl[3] for pl in planes], 1)
    leaves = [_t(CE).requires_grad_(), _t(CB).requires_grad_()] + \
             [dev(a).requires_grad_() for a in E + B] + [dev(x).requires_grad_(), dev(u).requires_grad_()]
    cfg = pa.RunConfig(DX, wl.DT, nsteps, K=K, ndim=2, q=QM, pusher=pusher)
    L = _run_autograd(leaves[0], leaves[1], leaves[2:5], leaves[5:8], leaves[8], leaves[9], cfg,
                      [dev(a) for a in w])
    L.backward()
    # oracle: the same loss, plane by plane (the gamma mean is over all electrons)
    gsum = {"CE": 0, "CB": 0}
    for k, (Ek, Bk, xk, uk) in enumerate(planes):
        ol = [_t(CE).requires_grad_(), _t(CB).requires_grad_()] + \
             [_t(a).requires_grad_() for a in list(Ek) + list(Bk)] + [_t(xk).requires_grad_(),
                                                                       _t(uk).requires_grad_()]
        Ef, Bf, xf, uf = ad.run(ol[2:5], ol[5:8], ol[8], ol[9], ol[0], ol[1], DX, wl.DT, QM, nsteps, 2, pusher)
        gam = torch.sqrt(1.0 + torch.sum(uf * uf, 0))
        wk0, wk1 = _t(w[0][k:k + 1]), _t(w[1][k:k + 1])
        Lk = (torch.sum(gam) / (nb * npb) + torch.sum((Ef[1] - wk0) ** 2) / torch.sum(_t(w[0]) ** 2)
              + torch.sum(wk1 * Bf[2]) + 0.1 * torch.sum(torch.sin(xf[0])))
        gr = torch.autograd.grad(Lk, ol)
        gsum["CE"] = gsum["CE"] + gr[0].numpy()
        gsum["CB"] = gsum["CB"] + gr[1].numpy()
        for i in range(6):
            assert _rel(host(leaves[2 + i].grad)[k:k + 1], gr[2 + i].numpy()) <= 1e-11, ("field", i, k)
        sl = slice(k * npb, (k + 1) * npb)
        assert _rel(host(leaves[8].grad)[:2, sl], gr[8].numpy()[:2]) <= 1e-11
        assert _rel(host(leaves[9].grad)[:, sl], gr[9].numpy()) <= 1e-11
    assert _rel(leaves[0].grad.numpy(), gsum["CE"]) <= 1e-11
    assert _rel(leaves[1].grad.numpy(), gsum["CB"]) <= 1e-11


@pytest.mark.parametrize("a0s", [(1.0, 30.0), (100.0, 1000.0)])
def test_envelope_gradients_match_central_differences(a0s, coeffs16):
    """Config-4 shape at a small size: gradients of mean final gamma plus the
    vacuum phase error with respect to three coefficients and each plane's
    a0 (1 and 30, and 100 and 1000: the top of the workload's a0 range),
    through the envelope -> fields map and the checkpointed run, against
    central differences of the GPU forward (h = 1e-6 relative)."""
    from paper_2004_03754_amd import autograd as pa
    CE, CB = coeffs16
    n1, n2, nb, npb, nsteps = 256, 8, 2, 8, 40
    L0 = wl.LAMBDA0
    Lp = torch.full((nb,), 2 * L0, dtype=torch.float64)
    xh = torch.full((nb,), 3 * L0, dtype=torch.float64)
    x = np.zeros((3, nb * npb))
    x[0] = np.tile(3.2 * L0 + np.linspace(0, L0, npb), nb)
    x[1] = 0.5 * n2 * DX[1]
    x[2] = np.repeat(np.arange(nb) + 0.5, npb)
    u = np.zeros_like(x)
    cfg = pa.RunConfig(DX, wl.DT, nsteps, K=16, ndim=2, q=QM)
    # reference field: the initial pulse moved on by the elapsed time
    Eref, _ = pa.sin2_pulse_fields(n1, n2, nb, DX, torch.tensor(list(a0s)), Lp, xh + nsteps * wl.DT)

    def loss(ce, cb, a0):
        E0, B0 = pa.sin2_pulse_fields(n1, n2, nb, DX, a0, Lp, xh)
        Ef, Bf, xf, uf = pa.run(ce, cb, E0, B0, dev(x), dev(u), cfg)
        gam = torch.sqrt(1.0 + torch.sum(uf * uf, 0))
        return torch.mean(gam) + torch.sum((Ef[1] - Eref[1]) ** 2) / torch.sum(Eref[1] ** 2)

    ce, cb = _t(CE).requires_grad_(), _t(CB).requires_grad_()
    a0 = torch.tensor(list(a0s), dtype=torch.float64, requires_grad=True)
    Lv = loss(ce, cb, a0)
    Lv.backward()
    checks = [("CE", 0), ("CE", 5), ("CB", 1), ("a0", 0), ("a0", 1)]
    for name, j in checks:
        base = {"CE": _t(CE), "CB": _t(CB), "a0": torch.tensor(list(a0s), dtype=torch.float64)}
        h = 1e-6 * max(abs(float(base[name][j])), 1.0)
        vals = []
        for sgn in (1, -1):
            args = {k: v.clone() for k, v in base.items()}
            args[name][j] += sgn * h
            with torch.no_grad():
                vals.append(float(loss(args["CE"], args["CB"], args["a0"])))
        fd = (vals[0] - vals[1]) / (2 * h)
        gr = {"CE": ce.grad, "CB": cb.grad, "a0": a0.grad}[name][j].item()
        assert abs(fd - gr) <= 1e-5 * abs(fd) + 1e-8 * max(1.0, abs(float(Lv))), (name, j, fd, gr)


def test_config4_full_size_gradients():
    """The differentiated workload at its full size and length, as the bench
    runs it: 16 stacked 2048 x 256 planes, 2048 steps, one sin^2 envelope per
    plane (a0 = 10^U(0,3), seed 4, L_p = 10 lambda0, head at 12 lambda0), 64
    electrons per plane at rest ahead of it, Boris, the library's
    proposed-solver fit; loss = mean final gamma + the vacuum phase error of
    E2.  The oracle cannot run this size; two properties that hold at any
    size are checked instead.
    (1) The gradients with respect to C^E, C^B and every plane's (a0, L_p,
    head) do not depend on the checkpoint interval: K = 64 (the bench's, 32
    segments) and K = 128 give the same values to 1e-14 (each reverse step
    sees the same recomputed states).
    (2) Central differences of the GPU forward, h = 1e-9 relative, for the
    three largest a0 (where the electrons reach gamma ~ 1e5), one plane's
    L_p and head, the largest a0's L_p, C^E_1 and C^B_2, agree to 1e-3.  The
    bound is loose for a reason: the linear-shape gather makes the loss only
    piecewise smooth (its slope jumps whenever an electron crosses a cell
    face), and over 2048 steps of 1024 electrons the difference quotient
    moves by 1e-7 .. 3e-4 between steps of 1e-8, 1e-9 and 1e-10 (and by 2e-3
    at 1e-6), while the adjoint, the exact derivative of the discrete map
    (pinned to the oracle's autograd at 1e-12 at smaller sizes), does not."""
    from paper_2004_03754_amd import autograd as pa
    CE = b.design_coeffs(16, 0.5, "E")
    CB = b.design_coeffs(16, 0.5, "B")
    n1, n2, nb, npb, steps = 2048, 256, 16, 64, 2048
    L0 = wl.LAMBDA0
    a0v = torch.tensor(10.0 ** (3.0 * wl.rng(4).random(nb)), dtype=torch.float64)
    Lpv = torch.full((nb,), 10 * L0, dtype=torch.float64)
    hv = torch.full((nb,), 12 * L0, dtype=torch.float64)
    x = torch.zeros((3, nb * npb), dtype=torch.float64)
    x[0] = (12.5 * L0 + torch.arange(npb, dtype=torch.float64) * (2 * L0 / npb)).repeat(nb)
    x[1] = 0.5 * n2 * DX[1]
    x[2] = torch.arange(nb, dtype=torch.float64).repeat_interleave(npb) + 0.5
    xd = x.to("cuda:0").contiguous()
    ud = torch.zeros_like(xd)
    with torch.no_grad():
        Eref, _ = pa.sin2_pulse_fields(n1, n2, nb, DX, a0v, Lpv, hv + steps * wl.DT)
    den = torch.sum(Eref[1] ** 2)

    def loss(a, K=64):
        E0, B0 = pa.sin2_pulse_fields(n1, n2, nb, DX, a["a0"], a["Lp"], a["head"])
        cfg = pa.RunConfig(DX, wl.DT, steps, K=K, ndim=2)
        Ef, Bf, xf, uf = pa.run(a["CE"], a["CB"], E0, B0, xd, ud, cfg)
        return torch.mean(torch.sqrt(1.0 + torch.sum(uf * uf, 0))) + torch.sum((Ef[1] - Eref[1]) ** 2) / den

    base = {"CE": _t(CE), "CB": _t(CB), "a0": a0v, "Lp": Lpv, "head": hv}
    grads = {}
    for K in (64, 128):
        print(f"config-4 full size: 16 x 2048x256, 2048 steps, K = {K}", flush=True)
        lv = {k: v.clone().requires_grad_() for k, v in base.items()}
        Lv = loss(lv, K)
        Lv.backward()
        grads[K] = {k: v.grad.numpy().copy() for k, v in lv.items()}
    for k in base:
        check(_rel(grads[128][k], grads[64][k]), 1e-14, f"config-4 full size grad {k}: K = 128 vs K = 64")
    g64 = grads[64]
    order = np.argsort(a0v.numpy())
    checks = [("a0", int(order[-1])), ("a0", int(order[-2])), ("a0", int(order[-3])), ("Lp", int(order[nb // 2])),
              ("head", int(order[-1])), ("Lp", int(order[-1])), ("CE", 0), ("CB", 1)]
    for name, j in checks:
        h = 1e-9 * max(abs(float(base[name][j])), 1.0)
        vals = []
        for sgn in (1, -1):
            a = {k: v.clone() for k, v in base.items()}
            a[name][j] += sgn * h
            with torch.no_grad():
                vals.append(float(loss(a)))
        fd = (vals[0] - vals[1]) / (2 * h)
        gr = float(g64[name][j])
        # the quotient's rounding floor: a few ulps of L over 2h, ten times
        floor = 10 * 4 * 2.0 ** -52 * max(1.0, abs(float(Lv))) / (2 * h)
        err = abs(fd - gr) / (abs(fd) + 1e3 * floor)
        print(f"  d L / d {name}[{j}]: adjoint {gr:.10e}, central difference {fd:.10e}", flush=True)
        check(err, 1e-3, f"config-4 full size d/d{name}[{j}] vs central difference")


def test_config4_length_run_matches_oracle(coeffs16):
    """The differentiated workload's shape at its length: 2 planes, 256
    steps, checkpoints every K = 64, Boris; each plane a sin^2 pulse
    (L_p = 4 lambda0, head at 8 lambda0, a0 = 10^U(0,3), seed 4) with 32
    electrons at rest spread over 2 lambda0 ahead of it on the middle x2
    line; loss = mean final gamma + the vacuum phase error of E2 against the
    initial pulse moved on by the elapsed time.  Gradients with respect to
    C^E, C^B, the initial fields and the particles against the oracle's
    autograd (each step checkpointed on the CPU side so that 256 steps fit
    in memory), at the FP64 bound 1e-12 (norm-wise; about 1e-13 measured)."""
    from torch.utils.checkpoint import checkpoint

    from paper_2004_03754_amd import autograd as pa
    CE, CB = coeffs16
    n1, n2, nb, npb, nsteps, K = 512, 16, 2, 32, 256, 64
    L0 = wl.LAMBDA0
    a0 = 10.0 ** (3.0 * wl.rng(4).random(nb))
    planes = [wl.laser_fields((n1, n2, 1), DX, wl.Sin2Pulse(a0=float(a), Lp=4 * L0), x_head=8 * L0) for a in a0]
    refs = [wl.laser_fields((n1, n2, 1), DX, wl.Sin2Pulse(a0=float(a), Lp=4 * L0), x_head=8 * L0 + nsteps * wl.DT)
            for a in a0]
    E = [np.concatenate([pl[0][c] for pl in planes], 0) for c in range(3)]
    B = [np.concatenate([pl[1][c] for pl in planes], 0) for c in range(3)]
    Eref2 = np.concatenate([r[0][1] for r in refs], 0)
    x = np.zeros((3, nb * npb))
    x[0] = np.tile(8.5 * L0 + np.arange(npb) * (2 * L0 / npb), nb)
    x[1] = 0.5 * n2 * DX[1]
    x[2] = np.repeat(np.arange(nb) + 0.5, npb)
    u = np.zeros_like(x)
    leaves = [_t(CE).requires_grad_(), _t(CB).requires_grad_()] + \
             [dev(a).requires_grad_() for a in E + B] + [dev(x).requires_grad_(), dev(u).requires_grad_()]
    cfg = pa.RunConfig(DX, wl.DT, nsteps, K=K, ndim=2, q=QM)
    Ef, Bf, xf, uf = pa.run(leaves[0], leaves[1], leaves[2:5], leaves[5:8], leaves[8], leaves[9], cfg)
    den = float(np.sum(Eref2 ** 2))
    L = torch.mean(torch.sqrt(1.0 + torch.sum(uf * uf, 0))) + torch.sum((Ef[1] - dev(Eref2)) ** 2) / den
    L.backward()

    def one(*s):
        En, Bn, xn, un = ad.step(s[:3], s[3:6], s[6], s[7], s[8], s[9], DX, wl.DT, QM,
                                 (n1 * DX[0], n2 * DX[1], DX[2]), 2)
        return (*En, *Bn, xn, un)

    gsum = {"CE": 0, "CB": 0}
    for k in range(nb):
        ol = [_t(CE).requires_grad_(), _t(CB).requires_grad_()] + \
             [_t(a[k:k + 1]).requires_grad_() for a in E + B] + \
             [_t(x[:, k * npb:(k + 1) * npb]).requires_grad_(), _t(u[:, k * npb:(k + 1) * npb]).requires_grad_()]
        st = tuple(ol[2:])
        for _ in range(nsteps):
            st = checkpoint(one, *st, ol[0], ol[1], use_reentrant=False)
        gam = torch.sqrt(1.0 + torch.sum(st[7] * st[7], 0))
        Lk = torch.sum(gam) / (nb * npb) + torch.sum((st[1] - _t(Eref2[k:k + 1])) ** 2) / den
        gr = torch.autograd.grad(Lk, ol)
        gsum["CE"] = gsum["CE"] + gr[0].numpy()
        gsum["CB"] = gsum["CB"] + gr[1].numpy()
        for i in range(6):
            check(_rel(host(leaves[2 + i].grad)[k:k + 1], gr[2 + i].numpy()), 1e-12,
                  f"config-4 length field grad {i} plane {k}")
        sl = slice(k * npb, (k + 1) * npb)
        check(_rel(host(leaves[8].grad)[:2, sl], gr[8].numpy()[:2]), 1e-12, f"config-4 length x grad plane {k}")
        check(_rel(host(leaves[9].grad)[:, sl], gr[9].numpy()), 1e-12, f"config-4 length u grad plane {k}")
    check(_rel(leaves[0].grad.numpy(), gsum["CE"]), 1e-12, "config-4 length dL/dC^E")
    check(_rel(leaves[1].grad.numpy(), gsum["CB"]), 1e-12, "config-4 length dL/dC^B")


@pytest.mark.parametrize("n,npart,pusher", [((256, 10, 3), 300, "boris"), ((64, 5, 2), 100, "analytic"),
                                            ((384, 17, 1), 200, "boris"), ((448, 21, 3), 300, "analytic"),
                                            ((256, 24, 200), 400, "boris")])
def test_fused_2d_reverse_matches_in_place_stages(n, npart, pusher, coeffs16):
    """The fused 2D reverse sweep (out-of-place cotangents, forward state and
    B^{n+1/2} given, C^B = e1) against the three in-place stages on the same
    inputs: field, particle and coefficient cotangents to 1e-12 (norm-wise),
    on stacks of planes with tiles overhanging the mesh in x1 and x2, meshes
    narrower than a tile's halo (the general periodic wrap), and 400 work
    items over the 256 persistent workgroups (several items per workgroup)."""
    CE, CB = coeffs16
    E, B, x, u = _case(n, 31, npart, 2, scale=2.0)
    x[2] = np.floor(wl.rng(33).random(npart) * n[2]) + 0.5
    lE, lB, lx, lu = _cotangents(n, npart, 32)
    res = []
    for oop in (False, True):
        grid = b.Grid([dev(e) for e in E], [dev(v) for v in B], DX[:2], wl.DT, CE, CB, ndim=2)
        pn = b.Particles(dev(x), dev(u), q=QM, m=1.0)
        En = [torch.empty_like(a) for a in grid.E]
        Bn = [torch.empty_like(a) for a in grid.B]
        Bh = [torch.empty_like(a) for a in grid.B]
        grid.step_to([pn], En, Bn, pusher=pusher, B_half=Bh)
        p = b.Particles(dev(x), dev(u), q=QM, m=1.0)
        lEd, lBd = [dev(a) for a in lE], [dev(a) for a in lB]
        lxd, lud = dev(lx), dev(lu)
        lam = b.Particles(lxd, lud, q=QM, m=1.0)
        gCE = torch.zeros(16, dtype=torch.float64, device="cuda:0")
        gCB = torch.zeros(16, dtype=torch.float64, device="cuda:0")
        kw = dict(next_E=En, next_B=Bn, half_B=Bh)
        if oop:
            kw["out_E"] = [torch.empty_like(a) for a in lEd]
            kw["out_B"] = [torch.empty_like(a) for a in lBd]
        grid.adjoint_step(lEd, lBd, gCE, gCB, [p], [lam], pusher=pusher, **kw)
        grid.sync()
        f = (kw["out_E"] + kw["out_B"]) if oop else (lEd + lBd)
        res.append([host(a) for a in f] + [host(lxd)[:2], host(lud), host(gCE), host(gCB)])
        if oop:  # the inputs are left unchanged
            assert all(np.array_equal(host(a), c) for a, c in zip(lEd + lBd, list(lE) + list(lB)))
        grid.close()
    names = ["lE1", "lE2", "lE3", "lB1", "lB2", "lB3", "lx", "lu", "gCE", "gCB"]
    for name, g_, r in zip(names, res[1], res[0]):
        check(_rel(g_, r), 1e-12, f"fused 2D reverse {n} {pusher} {name}")
