"""GPU parity of the quadratic particle shape (the Sec. 4.2 run's shape):
gather/push, the global deposit, the tile-sorted plasma step and the 2D step
against the oracle, and Gauss's law on the GPU's own output."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import fdtd, particles as pt, pic  # noqa: E402
from paper_2004_03754_amd import binding as b, workloads as wl  # noqa: E402

torch = pytest.importorskip("torch")
from gpu_util import assert_fields_close, dev, host  # noqa: E402

DX = (wl.DX1, wl.DX2, wl.DX3)


def _box(n):
    return [n[d] * DX[d] for d in range(3)]


def _by_id(t, ids):
    order = np.argsort(host(ids).astype(np.int64))
    return host(t)[:, order]


def _edge_particles(n, npart, seed, u_th):
    L = _box(n)
    x, u = wl.uniform_particles(npart, [0, 0, 0], L, seed=seed, u_th=u_th)
    x[0, 0] = 0.0
    x[0, 1] = L[0] - 1e-12
    x[0, 2] = 2.5 * DX[0]          # half-way between nodes
    x[1, 3] = 0.5 * DX[1]
    x[2, 4] = L[2] - 1e-13
    return x, u


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("ndim", [3, 2])
def test_quadratic_gather_push(ndim, prec, coeffs16):
    n = (128, 6, 5) if ndim == 3 else (128, 6, 1)
    E, B = wl.random_fields(n, seed=61, scale=2.0)
    x, u = _edge_particles(n, 3000, seed=62, u_th=2.0)
    if ndim == 2:
        x[2] = 0.0
    dtype = torch.float64 if prec == "fp64" else torch.float32
    if prec == "fp32":
        E = [e.astype(np.float32).astype(np.float64) for e in E]
        B = [v.astype(np.float32).astype(np.float64) for v in B]
    CE, CB = coeffs16
    grid = b.Grid([dev(e, dtype) for e in E], [dev(v, dtype) for v in B], DX if ndim == 3 else DX[:2], wl.DT,
                  CE, CB, prec=prec, ndim=ndim)
    grid.set_shape(2)
    xd, ud = dev(x), dev(u)
    print(f"quadratic gather/push {ndim}D {prec}", flush=True)
    grid.gather_push(b.Particles(xd, ud, q=-1.0, m=1.0), "boris")
    grid.sync()
    Ep, Bp = pt.gather(E, B, x, DX, ndim, order=2)
    un = pt.boris(u, Ep, Bp, -1.0, wl.DT)
    assert np.max(np.abs(host(ud) - un) / np.maximum(1.0, np.abs(un))) <= 1e-12
    grid.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("ndim", [3, 2])
def test_quadratic_deposit(ndim, prec, coeffs16):
    n = (128, 6, 5) if ndim == 3 else (128, 6, 1)
    L = _box(n)
    x0, u = _edge_particles(n, 4000, seed=63, u_th=0.5)
    x1, _ = wl.small_moves(x0, DX, L, seed=64)
    x1[0, 0] = L[0] - 0.05
    x1[0, 1] = 0.05
    if ndim == 2:
        x0[2] = 0.0
        x1[2] = 0.0
    dtype = torch.float64 if prec == "fp64" else torch.float32
    CE, CB = coeffs16
    zeros = [np.zeros((n[2], n[1], n[0])) for _ in range(3)]
    Jd = [dev(z, dtype) for z in zeros]
    grid = b.Grid([dev(z, dtype) for z in zeros], [dev(z, dtype) for z in zeros], DX if ndim == 3 else DX[:2],
                  wl.DT, CE, CB, J=Jd, prec=prec, ndim=ndim)
    grid.set_shape(2)
    print(f"quadratic deposit {ndim}D {prec}", flush=True)
    grid.deposit_J(b.Particles(dev(x1), dev(u), q=-1.0, m=1.0, w=0.37), dev(x0), zero_first=True)
    grid.sync()
    ref = pt.deposit(x0, x1, -1.0, 0.37, DX, wl.DT, (n[2], n[1], n[0]), ndim, u=u, order=2)
    assert_fields_close(Jd, ref, 1e-12 if prec == "fp64" else 2e-6, "quadratic deposit J")
    grid.close()


@pytest.mark.parametrize("pusher,nsteps,prec", [("boris", 4, "fp64"), ("hc", 7, "fp64"), ("boris", 4, "fp32")])
def test_quadratic_plasma_step(pusher, nsteps, prec, coeffs16):
    """The tile-sorted 3D plasma step with quadratic gather and deposit (the
    on-chip current tile one node wider), against the oracle; 7 steps cross
    two re-sorts."""
    CE, CB = coeffs16
    n = (128, 16, 12)
    L = _box(n)
    pulse = wl.Sin2Pulse(a0=2.0, Lp=4 * wl.LAMBDA0, period=L[0])
    E, B = wl.laser_fields(n, DX, pulse, x_head=3 * wl.LAMBDA0, w0=2 * wl.LAMBDA0)
    x, u = wl.lattice_particles(n, DX, 1, seed=65, u_th=0.05)
    x[0, :4] = [0.0, L[0] - 1e-12, 8 * DX[0], 8.5 * DX[0]]
    w = 0.01
    dtype = torch.float64 if prec == "fp64" else torch.float32
    grid = b.Grid([dev(e, dtype) for e in E], [dev(v, dtype) for v in B], DX, wl.DT, CE, CB,
                  J=[dev(np.zeros_like(e), dtype) for e in E], prec=prec)
    grid.set_shape(2)
    xd, ud = dev(x), dev(u)
    ids = torch.arange(x.shape[1], device="cuda:0", dtype=torch.int64)
    print(f"quadratic plasma step {pusher} {nsteps} {prec}", flush=True)
    grid.step_n([b.Particles(xd, ud, q=-1.0, m=1.0, w=w, id=ids)], nsteps, pusher=pusher, deposit=True)
    grid.sync()
    if prec == "fp32":
        E = [e.astype(np.float32).astype(np.float64) for e in E]
        B = [v.astype(np.float32).astype(np.float64) for v in B]
    sp = {"x": x.copy(), "u": u.copy(), "q": -1.0, "m": 1.0, "w": w}
    Er, Br = pic.run(E, B, [sp], CE, CB, DX, wl.DT, nsteps, pusher=pusher, deposit=True, order=2)
    ftol, ptol = (1e-12, 1e-12) if prec == "fp64" else (1e-5, 1e-6)
    assert_fields_close(grid.E, Er, ftol, "quadratic step E", joint=prec == "fp32")
    assert_fields_close(grid.B, Br, ftol, "quadratic step B", joint=prec == "fp32")
    ug, xg = _by_id(ud, ids), _by_id(xd, ids)
    assert np.max(np.abs(ug - sp["u"]) / np.maximum(1, np.abs(sp["u"]))) < ptol
    d = xg - sp["x"]
    Lb = np.asarray(L)[:, None]
    assert np.max(np.abs((d + Lb / 2) % Lb - Lb / 2)) < ptol
    grid.close()


def test_quadratic_2d_step_and_gauss_law(coeffs16_quarter):
    """The 2D path (unsorted push, global deposit) with the quadratic shape at
    dt = dx1/4 (wide Ampere stencil, x1 current correction): parity with the
    oracle, and div_B E - rho kept on the GPU's output."""
    CE, CB = coeffs16_quarter
    dt = wl.DX1 / 4
    n = (256, 24, 1)
    shape = (n[2], n[1], n[0])
    L = _box(n)
    E, B = wl.random_fields(n, seed=66, scale=0.05)
    x, u = wl.uniform_particles(3000, [0, 0, 0], L, seed=67, u_th=0.2)
    x[2] = 0.0
    g0 = fdtd.div_ampere(E, CB, DX) - pt.charge_density(x, -1.0, 0.01, DX, shape, ndim=2, order=2)
    Ed = [dev(e) for e in E]
    grid = b.Grid(Ed, [dev(v) for v in B], DX, dt, CE, CB, J=[dev(np.zeros_like(e)) for e in E], ndim=2)
    grid.set_shape(2)
    xd, ud = dev(x), dev(u)
    grid.step_n([b.Particles(xd, ud, q=-1.0, m=1.0, w=0.01)], 6, pusher="boris", deposit=True)
    grid.sync()
    sp = {"x": x.copy(), "u": u.copy(), "q": -1.0, "m": 1.0, "w": 0.01}
    Er, Br = pic.run(E, B, [sp], CE, CB, DX, dt, 6, pusher="boris", deposit=True, ndim=2, order=2)
    assert_fields_close(grid.E, Er, 1e-12, "2D quadratic step E")
    assert_fields_close(grid.B, Br, 1e-12, "2D quadratic step B")
    Eg = [host(e) for e in Ed]
    g = fdtd.div_ampere(Eg, CB, DX) - pt.charge_density(host(xd), -1.0, 0.01, DX, shape, ndim=2, order=2)
    assert np.max(np.abs(g - g0)) < 1e-11 * np.max(np.abs(fdtd.div_ampere(Eg, CB, DX)))
    grid.close()


def test_stacked_2d_deposit(coeffs16):
    """A stack of 2D meshes (n3 planes, plane index in x3) deposits each
    particle into its own plane: equal to the oracle's 2D deposit per plane."""
    CE, CB = coeffs16
    n = (128, 6, 3)
    shape = (n[2], n[1], n[0])
    L = _box(n)
    x0, u = wl.uniform_particles(900, [0, 0, 0], [L[0], L[1], 1.0], seed=68, u_th=0.5)
    x1, _ = wl.small_moves(x0, DX, L, seed=69)
    plane = np.arange(900) % 3
    x0[2] = plane + 0.5
    x1[2] = plane + 0.5
    zeros = [np.zeros(shape) for _ in range(3)]
    Jd = [dev(z) for z in zeros]
    grid = b.Grid([dev(z) for z in zeros], [dev(z) for z in zeros], DX[:2], wl.DT, CE, CB, J=Jd, ndim=2)
    grid.deposit_J(b.Particles(dev(x1), dev(u), q=-1.0, m=1.0, w=0.37), dev(x0), zero_first=True)
    grid.sync()
    for k in range(3):
        sel = plane == k
        ref = pt.deposit(x0[:, sel], x1[:, sel], -1.0, 0.37, DX, wl.DT, (1, n[1], n[0]), 2, u=u[:, sel])
        assert_fields_close([host(j)[k:k + 1] for j in Jd], ref, 1e-12, f"plane {k}")
    grid.close()


def test_adjoint_refuses_quadratic_shape(coeffs16):
    CE, CB = coeffs16
    shape = (2, 4, 64)
    z = [dev(np.zeros(shape)) for _ in range(6)]
    grid = b.Grid(z[:3], z[3:], DX, wl.DT, CE, CB)
    grid.set_shape(2)
    lE = [dev(np.zeros(shape)) for _ in range(3)]
    lB = [dev(np.zeros(shape)) for _ in range(3)]
    g = [torch.zeros(16, dtype=torch.float64, device="cuda:0") for _ in range(2)]
    with pytest.raises(b.YeePICError) as e:
        grid.adjoint_step(lE, lB, g[0], g[1])
    assert e.value.code == -6
    with pytest.raises(b.YeePICError):
        grid.set_shape(3)
    grid.close()
