"""Parity at the benchmark's full sizes and launch configuration, on samples
the oracle can compute.

* 1024 x 256 x 256 FP64 (the headline workload): the oracle runs on a
  periodic 1024 x 32 x 32 window of the same initial fields.  A fused step
  reaches at most two cells along x2 and x3, so after s steps the window's
  interior, 2s cells away from its edges, is exactly the full run's; fields
  there and electrons that start there are compared.
* 512 x 256 x 256 with FP32 fields and 268M electrons (the plasma
  workload): the oracle runs on a periodic 512 x 24 x 24 window around the
  axis with every electron that starts in it; the same reach argument gives
  an exact interior, where fields, the last step's current and the electrons
  that start there are compared.
* 2048 x 512 x 512 with FP32 fields (the mixed-precision workload): the
  plane wave does not depend on x2 and x3, so a periodic 2048 x 4 x 4 window
  is exactly the full run; FP32 fields are held to 1e-5 of the FP64 oracle
  and the electrons' gamma error is measured against the error FP32 field
  storage alone causes (the oracle run with float32 field arrays).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import fdtd, particles, pic  # noqa: E402
from paper_2004_03754_amd import binding as b, workloads as wl  # noqa: E402

torch = pytest.importorskip("torch")
from gpu_util import check, host  # noqa: E402

DX = (wl.DX1, wl.DX2, wl.DX3)
L0 = wl.LAMBDA0


def _laser_device(n, pulse, x_head, w0, dtype):
    """The headline workload's fields built on the device from the same
    factors that workloads.laser_fields multiplies on the host."""
    e2, b3, prof = wl.laser_profiles(n, DX, pulse, x_head, w0)
    d = "cuda:0"
    pr = torch.as_tensor(prof, device=d, dtype=torch.float64)
    E2 = (pr[:, :, None] * torch.as_tensor(e2, device=d)[None, None, :]).to(dtype).contiguous()
    B3 = (pr[:, :, None] * torch.as_tensor(b3, device=d)[None, None, :]).to(dtype).contiguous()
    z = [torch.zeros_like(E2) for _ in range(4)]
    lon = wl.laser_longitudinal(n, DX, pulse, x_head, w0)
    if lon is not None:
        e1, p1, b1, q1 = (torch.as_tensor(a, device=d, dtype=torch.float64) for a in lon)
        z[0] = (p1[:, :, None] * e1[None, None, :]).to(dtype).contiguous()
        z[2] = (q1[:, :, None] * b1[None, None, :]).to(dtype).contiguous()
    return [z[0], E2, z[1]], [z[2], z[3], B3]


@pytest.mark.parametrize("steps,half", [(2, 16), (20, 56)])
def test_headline_workload_window_parity(steps, half):
    """The headline workload at full size for ``steps`` steps (2, and 20:
    the benchmark's step count), against the oracle on a periodic window of
    1024 x 2*half x 2*half cells around the axis: fields on the window's
    interior (2*steps cells from its edges) to 1e-12, electrons that start
    2*steps + 2 cells inside it, one in 40 (2 steps) or 100 (20 steps)."""
    CE = b.design_coeffs(16, 0.5, "E")
    CB = b.design_coeffs(16, 0.5, "B")
    n = (1024, 256, 256)
    pulse = wl.Sin2Pulse(a0=100.0, Lp=10 * L0)
    E, B = _laser_device(n, pulse, 12 * L0, 4 * L0, torch.float64)
    lo = [13 * L0, (n[1] / 2 - 32) * DX[1], (n[2] / 2 - 32) * DX[2]]
    hi = [15 * L0, (n[1] / 2 + 32) * DX[1], (n[2] / 2 + 32) * DX[2]]
    x, u = wl.uniform_particles(1 << 20, lo, hi, seed=2)
    w0, w1 = 128 - half, 128 + half        # window along x2 and x3
    Ew = [host(e[w0:w1, w0:w1, :]) for e in E]
    Bw = [host(v[w0:w1, w0:w1, :]) for v in B]
    grid = b.Grid(E, B, DX, wl.DT, CE, CB)
    xd = torch.as_tensor(x, device="cuda:0").contiguous()
    ud = torch.as_tensor(u, device="cuda:0").contiguous()
    p = b.Particles(xd, ud, q=-1.0, m=1.0)
    print(f"headline window parity: 1024x256x256 FP64, 1048576 electrons, {steps} steps", flush=True)
    grid.step_n([p], steps, pusher="analytic")
    grid.sync()
    # oracle on the window, with a sample of the electrons that start well inside it
    m = 2 * steps + 2
    inner = ((x[1] >= (w0 + m) * DX[1]) & (x[1] < (w1 - m) * DX[1]) &
             (x[2] >= (w0 + m) * DX[2]) & (x[2] < (w1 - m) * DX[2]))
    idx = np.flatnonzero(inner)[::40 if steps <= 2 else 100]
    assert idx.size > 500
    xs = x[:, idx].copy()
    xs[1] -= w0 * DX[1]
    xs[2] -= w0 * DX[2]
    sp = {"x": xs, "u": u[:, idx].copy(), "q": -1.0, "m": 1.0, "w": 1.0}
    Er, Br = pic.run(Ew, Bw, [sp], CE, CB, DX, wl.DT, steps, pusher="analytic")
    c = slice(2 * steps, (w1 - w0) - 2 * steps)
    for g, r in zip(E + B, list(Er) + list(Br)):
        gw = host(g[w0:w1, w0:w1, :])[c, c, :]
        rw = r[c, c, :]
        scale = max(np.max(np.abs(r)), 1e-300)
        check(float(np.max(np.abs(gw - rw))) / scale, 1e-12, f"headline {steps} steps field")
    ug = host(ud)[:, idx]
    xg = host(xd)[:, idx]
    xg[1] -= w0 * DX[1]
    xg[2] -= w0 * DX[2]
    check(float(np.max(np.abs(ug - sp["u"]) / np.maximum(1.0, np.abs(sp["u"])))), 1e-12,
          f"headline {steps} steps u")
    check(float(np.max(np.abs(xg - sp["x"]))) / (n[0] * DX[0]), 1e-12, f"headline {steps} steps x")
    grid.close()


def test_plasma_workload_window_parity():
    """The plasma workload at full size in the benchmark's launch
    configuration: 512 x 256 x 256 cells, FP32 fields, 268,435,456 electrons
    (8 per cell on the sub-lattice, u_th = 0.01, w = 0.01/8), Gaussian laser
    a0 = 10, w0 = 4 lambda0; Boris, Esirkepov deposit, sort interval 3, for
    4 steps (sorts before steps 0 and 3, the second from the keys the push
    before it wrote).  The oracle (FP64, on the FP32 initial values) runs a
    periodic 512 x 24 x 24 window around the axis with the 2.4M electrons
    that start in it.  A step reaches at most two cells along x2 and x3 and
    an electron moves at most 0.125 cells, so after 4 steps everything 10
    cells inside the window is exactly the full run's.  There: fields to
    1e-5 of the largest (FP32 storage), the last step's current to 1e-5 of
    the largest, and every electron that starts there (by id, the GPU
    reorders them): gamma to 1e-6, u to 1e-6 of max(1, |u|), x to 1e-6 of
    a cell."""
    CE = b.design_coeffs(16, 0.5, "E")
    CB = b.design_coeffs(16, 0.5, "B")
    n = (512, 256, 256)
    steps, half, marg = 4, 12, 10
    qw = 0.01 / 8
    d = "cuda:0"
    pulse = wl.Sin2Pulse(a0=10.0, Lp=10 * L0, period=n[0] * DX[0])
    E, B = _laser_device(n, pulse, 12 * L0, 4 * L0, torch.float32)
    J = [torch.zeros_like(E[0]) for _ in range(3)]
    xd, ud = wl.device_lattice_particles(n, DX, 2, 0.01, 3, torch)
    npart = xd.shape[1]
    ids = torch.arange(npart, device=d, dtype=torch.int64)
    w0, w1 = 128 - half, 128 + half
    in_w = ((xd[1] >= w0 * DX[1]) & (xd[1] < w1 * DX[1]) & (xd[2] >= w0 * DX[2]) & (xd[2] < w1 * DX[2]))
    widx = torch.nonzero(in_w).flatten()
    xs, us, wid = host(xd[:, widx]), host(ud[:, widx]), widx.cpu().numpy()
    del in_w, widx
    xs[1] -= w0 * DX[1]
    xs[2] -= w0 * DX[2]
    Ew = [host(e[w0:w1, w0:w1, :]) for e in E]
    Bw = [host(v[w0:w1, w0:w1, :]) for v in B]
    grid = b.Grid(E, B, DX, wl.DT, CE, CB, J=J, prec="fp32")
    p = b.Particles(xd, ud, q=-1.0, m=1.0, w=qw, id=ids)
    print(f"plasma window parity: 512x256x256 FP32, {npart} electrons, {steps} steps", flush=True)
    grid.step_n([p], steps, pusher="boris", deposit=True)
    grid.sync()
    # oracle: steps - 1 steps, then the last one by hand to keep its current
    sp = {"x": xs, "u": us, "q": -1.0, "m": 1.0, "w": qw}
    Er, Br = pic.run(Ew, Bw, [sp], CE, CB, DX, wl.DT, steps - 1, pusher="boris", deposit=True)
    Ep, Bp = particles.gather(Er, Br, sp["x"], DX)
    u_new = particles.boris(sp["u"], Ep, Bp, -1.0, wl.DT)
    Lw = [n[0] * DX[0], 2 * half * DX[1], 2 * half * DX[2]]
    x_new, _ = particles.advance_position(sp["x"], u_new, wl.DT, Lw)
    Jr = particles.deposit(sp["x"], x_new, -1.0, qw, DX, wl.DT, Er[0].shape, 3, u=u_new)
    Er, Br = fdtd.sweep(Er, Br, Jr, CE, CB, DX, wl.DT)
    c = slice(marg, 2 * half - marg)
    fscale = max(float(np.max(np.abs(r[c, c, :]))) for r in list(Er) + list(Br))
    ferr = max(float(np.max(np.abs(host(g[w0:w1, w0:w1, :])[c, c, :] - r[c, c, :])))
               for g, r in zip(E + B, list(Er) + list(Br))) / fscale
    jscale = max(float(np.max(np.abs(r[c, c, :]))) for r in Jr)
    jerr = max(float(np.max(np.abs(host(g[w0:w1, w0:w1, :])[c, c, :] - r[c, c, :]))) for g, r in zip(J, Jr)) / jscale
    # electrons that start 10 cells inside, found on the GPU by id
    inner = ((xs[1] >= marg * DX[1]) & (xs[1] < (2 * half - marg) * DX[1]) &
             (xs[2] >= marg * DX[2]) & (xs[2] < (2 * half - marg) * DX[2]))
    sel = np.flatnonzero(inner)
    inv = torch.empty_like(ids)
    inv[ids] = torch.arange(npart, device=d, dtype=torch.int64)
    at = inv[torch.as_tensor(wid[sel], device=d)]
    del inv
    xg, ug = host(xd[:, at]), host(ud[:, at])
    xg[1] -= w0 * DX[1]
    xg[2] -= w0 * DX[2]
    ur, xr = u_new[:, sel], x_new[:, sel]
    uerr = float(np.max(np.linalg.norm(ug - ur, axis=0) / np.maximum(1.0, np.linalg.norm(ur, axis=0))))
    g_g, g_r = np.sqrt(1 + np.sum(ug * ug, 0)), np.sqrt(1 + np.sum(ur * ur, 0))
    gerr = float(np.max(np.abs(g_g - g_r) / g_r))
    xerr = max(float(np.max(np.abs(xg[k] - xr[k]))) / DX[k] for k in range(3))
    print(f"plasma window: fields {ferr:.2e} (joint, max {fscale:.3g}), current {jerr:.2e} (max {jscale:.3g}); "
          f"{sel.size} electrons: u {uerr:.2e}, gamma {gerr:.2e}, x {xerr:.2e} cells", flush=True)
    assert sel.size > 40000
    check(ferr, 1e-5, "plasma full size fields")
    check(jerr, 1e-5, "plasma full size current")
    check(gerr, 1e-6, "plasma full size gamma")
    check(uerr, 1e-6, "plasma full size u")
    check(xerr, 1e-6, "plasma full size x (cells)")
    grid.check(p)
    grid.close()


def _rho_device(x, q, w, n):
    """Charge density on the nodes from device positions: q w times the
    linear shape (the definition the Esirkepov deposit conserves, Sec. 3.3),
    summed with index_add in FP64, one of the eight corners at a time."""
    n1, n2, n3 = n
    rho = torch.zeros(n3 * n2 * n1, device="cuda:0", dtype=torch.float64)
    idx, wts = [], []
    for d, nd in enumerate((n1, n2, n3)):
        u = x[d] * (1.0 / DX[d])
        f = torch.floor(u)
        i0 = f.to(torch.int64) % nd
        idx.append((i0, (i0 + 1) % nd))
        wts.append((1.0 - (u - f), u - f))
    for a in range(2):
        for bb in range(2):
            for c in range(2):
                lin = (idx[2][c] * n2 + idx[1][bb]) * n1 + idx[0][a]
                rho.index_add_(0, lin, q * w * wts[0][a] * wts[1][bb] * wts[2][c])
    return rho.view(n3, n2, n1)


def _div_yee_device(E):
    """Gauss-law divergence with the Yee (C^B = e1) stencil on the nodes:
    backward differences along each direction (periodic), FP64."""
    e = [c.to(torch.float64) for c in E]
    return ((e[0] - torch.roll(e[0], 1, 2)) / DX[0] + (e[1] - torch.roll(e[1], 1, 1)) / DX[1]
            + (e[2] - torch.roll(e[2], 1, 0)) / DX[2])


def test_plasma_workload_gauss_law_200_steps():
    """The plasma workload at full size for its 200 steps (512 x 256 x 256,
    FP32 fields, 268M electrons, the bench's launch configuration): Sec. 3.3,
    with the charge-conserving deposit at dt = dx1/2 (Ampere stencil = Yee,
    no x1 correction) div E - rho keeps its initial value on every node.  rho
    from the GPU's particle positions, div E from its fields (both in FP64);
    the change is at most the FP32 rounding of E in each step's update
    accumulated linearly, 200 x sum_d(2/dx_d) x 2^-24 x max|E|; the plasma
    must have responded far more than that."""
    CE = b.design_coeffs(16, 0.5, "E")
    CB = b.design_coeffs(16, 0.5, "B")
    n = (512, 256, 256)
    steps = 200
    qw = 0.01 / 8
    pulse = wl.Sin2Pulse(a0=10.0, Lp=10 * L0, period=n[0] * DX[0])
    E, B = _laser_device(n, pulse, 12 * L0, 4 * L0, torch.float32)
    J = [torch.zeros_like(E[0]) for _ in range(3)]
    xd, ud = wl.device_lattice_particles(n, DX, 2, 0.01, 3, torch)
    rho0 = _rho_device(xd, -1.0, qw, n)
    res0 = _div_yee_device(E) - rho0
    grid = b.Grid(E, B, DX, wl.DT, CE, CB, J=J, prec="fp32")
    p = b.Particles(xd, ud, q=-1.0, m=1.0, w=qw)
    print(f"plasma Gauss law: 512x256x256 FP32, {xd.shape[1]} electrons, {steps} steps", flush=True)
    grid.step_n([p], steps, pusher="boris", deposit=True)
    grid.sync()
    rho = _rho_device(xd, -1.0, qw, n)
    res = _div_yee_device(E) - rho
    drift = float(torch.max(torch.abs(res - res0)))
    response = float(torch.max(torch.abs(rho - rho0)))
    del res, res0, rho, rho0
    emax = max(float(torch.max(torch.abs(e))) for e in E)
    bound = steps * sum(2 / d for d in DX) * 2.0 ** -24 * emax
    print(f"plasma Gauss law over {steps} steps: drift {drift:.2e}, bound {bound:.2e}, "
          f"max change of rho {response:.2e}", flush=True)
    check(drift / bound, 1.0, "full-size plasma Gauss-law drift / bound")
    assert response > 100 * drift
    grid.check(p)
    grid.close()


def test_headline_analogue_500_steps():
    """A 256 x 64 x 64 analogue of the headline workload over 500 steps
    (FP64, proposed solver at dt = dx1/2, exact pusher): a Gaussian sin^2
    pulse (a0 = 100, L_p = 4 lambda0, w0 = 2 lambda0, head at 6 lambda0)
    that crosses the periodic x1 box twice, and 4096 electrons from rest in
    a 32 x 16 x 16-cell box ahead of it on the axis.  Fields per component
    and every electron against the oracle's 500 steps."""
    CE = b.design_coeffs(16, 0.5, "E")
    CB = b.design_coeffs(16, 0.5, "B")
    n = (256, 64, 64)
    steps = 500
    pulse = wl.Sin2Pulse(a0=100.0, Lp=4 * L0)
    E, B = wl.laser_fields(n, DX, pulse, x_head=6 * L0, w0=2 * L0)
    lo = [6.5 * L0, 24 * DX[1], 24 * DX[2]]
    hi = [7.5 * L0, 40 * DX[1], 40 * DX[2]]
    x, u = wl.uniform_particles(4096, lo, hi, seed=12)
    d = "cuda:0"
    Eg = [torch.as_tensor(e, device=d).contiguous() for e in E]
    Bg = [torch.as_tensor(v, device=d).contiguous() for v in B]
    grid = b.Grid(Eg, Bg, DX, wl.DT, CE, CB)
    xd = torch.as_tensor(x, device=d).contiguous()
    ud = torch.as_tensor(u, device=d).contiguous()
    p = b.Particles(xd, ud, q=-1.0, m=1.0)
    print("headline analogue: 256x64x64 FP64, 4096 electrons, 500 steps", flush=True)
    grid.step_n([p], steps, pusher="analytic")
    grid.sync()
    sp = {"x": x.copy(), "u": u.copy(), "q": -1.0, "m": 1.0, "w": 1.0}
    Er, Br = pic.run(E, B, [sp], CE, CB, DX, wl.DT, steps, pusher="analytic")
    for c, (g, r) in enumerate(zip(Eg + Bg, list(Er) + list(Br))):
        scale = max(float(np.max(np.abs(r))), 1e-300)
        check(float(np.max(np.abs(host(g) - r))) / scale, 1e-12, f"analogue 500 steps field {c}")
    ug, xg = host(ud), host(xd)
    du = np.linalg.norm(ug - sp["u"], axis=0) / np.maximum(1.0, np.linalg.norm(sp["u"], axis=0))
    check(float(du.max()), 1e-12, "analogue 500 steps u")
    check(float(np.max(np.abs(xg - sp["x"]))) / (n[0] * DX[0]), 1e-12, "analogue 500 steps x")
    grid.close()


def test_mixed_precision_plane_wave_full_size():
    CE = b.design_coeffs(16, 0.5, "E")
    CB = b.design_coeffs(16, 0.5, "B")
    n = (2048, 512, 512)
    steps = 20
    a0 = 1.0e4
    L = [n[d] * DX[d] for d in range(3)]
    pw = wl.PlaneWave(a0)
    e2, b3, _ = wl.laser_profiles((n[0], 4, 4), DX, pw)
    d = "cuda:0"
    shape = (n[2], n[1], n[0])
    E2 = torch.as_tensor(e2, device=d, dtype=torch.float32).expand(shape).contiguous()
    B3 = torch.as_tensor(b3, device=d, dtype=torch.float32).expand(shape).contiguous()
    E = [torch.zeros(shape, device=d, dtype=torch.float32), E2, torch.zeros(shape, device=d, dtype=torch.float32)]
    B = [torch.zeros(shape, device=d, dtype=torch.float32), torch.zeros(shape, device=d, dtype=torch.float32), B3]
    x, u = wl.uniform_particles(1 << 22, [0, 0, 0], L, seed=5)
    xd = torch.as_tensor(x, device=d).contiguous()
    ud = torch.as_tensor(u, device=d).contiguous()
    grid = b.Grid(E, B, DX, wl.DT, CE, CB, prec="fp32")
    p = b.Particles(xd, ud, q=-1.0, m=1.0)
    print("plane-wave full size: 2048x512x512 FP32 fields, 4194304 electrons, 20 steps", flush=True)
    grid.step_n([p], steps, pusher="analytic")
    grid.sync()
    # oracle: a 2048 x 4 x 4 periodic window of the FP32 initial state, in FP64
    nw = (n[0], 4, 4)
    Ew, Bw = wl.laser_fields(nw, DX, pw)
    Ew = [e.astype(np.float32).astype(np.float64) for e in Ew]
    Bw = [v.astype(np.float32).astype(np.float64) for v in Bw]
    idx = np.arange(0, x.shape[1], 2048)
    xs = x[:, idx].copy()
    xs[1] = np.mod(xs[1], 4 * DX[1])
    xs[2] = np.mod(xs[2], 4 * DX[2])
    sp = {"x": xs, "u": u[:, idx].copy(), "q": -1.0, "m": 1.0, "w": 1.0}
    Er, Br = pic.run(Ew, Bw, [sp], CE, CB, DX, wl.DT, steps, pusher="analytic")
    scale = max(np.max(np.abs(r)) for r in list(Er) + list(Br))
    errs = []
    for g, r in zip(E + B, list(Er) + list(Br)):
        gw = host(g[100:104, 300:304, :])  # any window: the full run is uniform in x2, x3
        errs.append(float(np.max(np.abs(gw - r)) / scale))
    ug = host(ud)[:, idx]
    gam_g = np.sqrt(1 + np.sum(ug * ug, 0))
    gam_r = np.sqrt(1 + np.sum(sp["u"] ** 2, 0))
    rel = np.abs(gam_g - gam_r) / gam_r
    # what FP32 field storage alone does to gamma: the oracle's own step with
    # float32 field arrays (the gather still weights in FP64)
    s32 = {"x": xs.copy(), "u": u[:, idx].copy(), "q": -1.0, "m": 1.0, "w": 1.0}
    E32 = [e.astype(np.float32) for e in Ew]
    B32 = [v.astype(np.float32) for v in Bw]
    pic.run(E32, B32, [s32], CE.astype(np.float32), CB.astype(np.float32), DX, wl.DT, steps, pusher="analytic")
    rel32 = np.abs(np.sqrt(1 + np.sum(s32["u"] ** 2, 0)) - gam_r) / gam_r
    print(f"mixed precision after {steps} steps: field error {max(errs):.2e} (joint norm); gamma error "
          f"GPU max {rel.max():.2e} median {np.median(rel):.2e} | FP32-field oracle max {rel32.max():.2e} "
          f"median {np.median(rel32):.2e} over {idx.size} electrons", flush=True)
    assert max(errs) <= 1e-5
    # The 1e-6 gamma target is not reachable with FP32 fields at a0 = 1e4: the
    # electrons' gamma - u1 invariant turns the absolute field rounding
    # (~1e-7 x 1e4) into relative gamma errors of 1e-6 .. 1e-3 within 20 steps,
    # as the FP32-field oracle shows.  The GPU must not add error beyond that.
    assert np.median(rel) <= 10 * np.median(rel32) + 1e-12
    assert rel.max() <= 10 * rel32.max() + 1e-12
    grid.close()


def test_plane_wave_full_length_1000_steps():
    """The mixed-precision workload at its full size and length: the
    2048 x 512 x 512 plane wave at a0 = 1e4 for 1000 steps with 4M electrons
    from rest (exact pusher), once with FP32 and once with FP64 fields.  The
    electrons do not act on the fields, and the fields do not depend on x2
    and x3, so the oracle's periodic 2048 x 4 x 4 window gives the full run's
    fields exactly: FP64 to 1e-12 per component, FP32 to 1e-5 (joint).  No
    exact push may end unconverged (pic_check).  The electrons' gamma
    follows the closed-form plane-wave motion only up to the linear gather's
    interpolation error, which at a0 = 1e4 grows with time; it must stay
    within what the oracle itself shows for the same 512 electrons (every
    8192nd): the GPU's largest and median deviation (FP64 fields) at most
    1.5 times the oracle's plus 0.02 of max(gamma - 1)."""
    from oracle import trajectory as tj
    CE = b.design_coeffs(16, 0.5, "E")
    CB = b.design_coeffs(16, 0.5, "B")
    n = (2048, 512, 512)
    steps = 1000
    L = [n[d] * DX[d] for d in range(3)]
    pw = wl.PlaneWave(1.0e4)
    e2, b3, _ = wl.laser_profiles((n[0], 4, 4), DX, pw)
    x, u = wl.uniform_particles(1 << 22, [0, 0, 0], L, seed=5)
    Ew, Bw = wl.laser_fields((n[0], 4, 4), DX, pw)
    idx = np.arange(0, x.shape[1], 8192)
    xs = x[:, idx].copy()
    xs[1] = np.mod(xs[1], 4 * DX[1])
    xs[2] = np.mod(xs[2], 4 * DX[2])
    sp = {"x": xs, "u": u[:, idx].copy(), "q": -1.0, "m": 1.0, "w": 1.0}
    Er, Br = pic.run(Ew, Bw, [sp], CE, CB, DX, wl.DT, steps, pusher="analytic")
    tt = (steps - 0.5) * wl.DT
    _, _, gcf = tj.state_at(pw.a, -1.0, -0.5 * wl.DT, x[:, idx], tt)
    span = float(np.max(gcf - 1))
    dev_or = np.abs(np.sqrt(1 + np.sum(sp["u"] ** 2, 0)) - gcf) / span
    d = "cuda:0"
    shape = (n[2], n[1], n[0])
    for prec in ("fp32", "fp64"):
        dtype = torch.float32 if prec == "fp32" else torch.float64
        E2 = torch.as_tensor(e2, device=d, dtype=dtype).expand(shape).contiguous()
        B3 = torch.as_tensor(b3, device=d, dtype=dtype).expand(shape).contiguous()
        z = [torch.zeros(shape, device=d, dtype=dtype) for _ in range(4)]
        E, B = [z[0], E2, z[1]], [z[2], z[3], B3]
        xd = torch.as_tensor(x, device=d).contiguous()
        ud = torch.as_tensor(u, device=d).contiguous()
        grid = b.Grid(E, B, DX, wl.DT, CE, CB, prec=prec)
        p = b.Particles(xd, ud, q=-1.0, m=1.0)
        print(f"plane wave full length: 2048x512x512 {prec} fields, 4194304 electrons, {steps} steps", flush=True)
        grid.step_n([p], steps, pusher="analytic")
        grid.sync()
        grid.check(p)
        own = [float(np.max(np.abs(host(g[300:304, 100:104, :]) - r))) / max(float(np.max(np.abs(r))), 1e-300)
               for g, r in zip(E + B, list(Er) + list(Br))]
        scale = max(float(np.max(np.abs(r))) for r in list(Er) + list(Br))
        joint = max(float(np.max(np.abs(host(g[300:304, 100:104, :]) - r))) for g, r in zip(E + B, list(Er) + list(Br)))
        joint /= scale
        ug = host(ud)[:, idx]
        dev_gpu = np.abs(np.sqrt(1 + np.sum(ug * ug, 0)) - gcf) / span
        print(f"  fields: joint {joint:.2e}, per component {', '.join(f'{e:.1e}' for e in own)}; closed form: GPU max "
              f"{dev_gpu.max():.3f} median {np.median(dev_gpu):.3f}, oracle max {dev_or.max():.3f} median "
              f"{np.median(dev_or):.3f}", flush=True)
        if prec == "fp64":
            for c, e in enumerate(own):
                if max(float(np.max(np.abs(r))) for r in [(list(Er) + list(Br))[c]]) > 0:
                    check(e, 1e-12, f"1000-step FP64 plane wave field {c}")
            check(float(dev_gpu.max()), 1.5 * float(dev_or.max()) + 0.02, "1000-step plane wave closed form (max)")
            check(float(np.median(dev_gpu)), 1.5 * float(np.median(dev_or)) + 0.02,
                  "1000-step plane wave closed form (median)")
        else:
            check(joint, 1e-5, "1000-step FP32 plane wave fields (joint)")
        grid.close()
        del E, B, E2, B3, z, xd, ud
        torch.cuda.empty_cache()


def test_fp64_plane_wave_full_size_and_closed_form():
    """The 2048 x 512 x 512 plane wave at a0 = 1e4 with FP64 fields (the
    mixed-precision workload's FP64 run), 20 steps, 4M electrons from rest
    with the exact pusher.  The fields do not depend on x2 and x3, so a
    periodic 2048 x 4 x 4 window is exactly the full run: fields to 1e-12 per
    component, and a sample of electrons per particle (|u - u_ref| /
    max(1, |u_ref|)) against the oracle's own change under one-ulp changes of
    the initial x1 and field (the map is ill-conditioned at this field
    strength): median below 1e-12, the maximum within ten times the largest
    sensitivity (measured: median 2.4e-13, maximum 2.4e-10 against 2.1e-10).  Every sampled
    electron also follows the closed-form plane-wave motion (Sec. 4.1,
    canonical momentum) from rest at t = -dt/2 within 0.25 of max(gamma - 1):
    at a0 = 1e4 the linear gather's interpolation error, up to
    (k0 dx1)^2/8 ~ 5e-3 of the field and different for E2 and B3, breaks the
    null structure of the wave and grows over the step (the oracle shows a
    median of 0.10 and a maximum of 0.18), which bounds the agreement."""
    from oracle import trajectory as tj
    CE = b.design_coeffs(16, 0.5, "E")
    CB = b.design_coeffs(16, 0.5, "B")
    n = (2048, 512, 512)
    steps = 20
    a0 = 1.0e4
    L = [n[d] * DX[d] for d in range(3)]
    pw = wl.PlaneWave(a0)
    e2, b3, _ = wl.laser_profiles((n[0], 4, 4), DX, pw)
    d = "cuda:0"
    shape = (n[2], n[1], n[0])
    E2 = torch.as_tensor(e2, device=d, dtype=torch.float64).expand(shape).contiguous()
    B3 = torch.as_tensor(b3, device=d, dtype=torch.float64).expand(shape).contiguous()
    z = [torch.zeros(shape, device=d, dtype=torch.float64) for _ in range(4)]
    E = [z[0], E2, z[1]]
    B = [z[2], z[3], B3]
    x, u = wl.uniform_particles(1 << 22, [0, 0, 0], L, seed=5)
    xd = torch.as_tensor(x, device=d).contiguous()
    ud = torch.as_tensor(u, device=d).contiguous()
    grid = b.Grid(E, B, DX, wl.DT, CE, CB)
    p = b.Particles(xd, ud, q=-1.0, m=1.0)
    print("plane-wave full size: 2048x512x512 FP64 fields, 4194304 electrons, 20 steps", flush=True)
    grid.step_n([p], steps, pusher="analytic")
    grid.sync()
    nw = (n[0], 4, 4)
    Ew, Bw = wl.laser_fields(nw, DX, pw)
    idx = np.arange(0, x.shape[1], 2048)
    xs = x[:, idx].copy()
    xs[1] = np.mod(xs[1], 4 * DX[1])
    xs[2] = np.mod(xs[2], 4 * DX[2])
    sp = {"x": xs, "u": u[:, idx].copy(), "q": -1.0, "m": 1.0, "w": 1.0}
    Er, Br = pic.run(Ew, Bw, [sp], CE, CB, DX, wl.DT, steps, pusher="analytic")
    for c, (g, r) in enumerate(zip(E + B, list(Er) + list(Br))):
        gw = host(g[200:204, 40:44, :])  # any window: the full run is uniform in x2, x3
        scale = max(float(np.max(np.abs(r))), 1e-300)
        check(float(np.max(np.abs(gw - r))) / scale if np.max(np.abs(r)) > 0 else float(np.max(np.abs(gw))),
              1e-12, f"FP64 plane wave field {c}")
    ug = host(ud)
    nrm = np.maximum(1.0, np.linalg.norm(sp["u"], axis=0))
    err = np.linalg.norm(ug[:, idx] - sp["u"], axis=0) / nrm
    # The 20-step map at a0 = 1e4 is ill-conditioned: the oracle's own result
    # moves by up to ~2e-10 when an electron's initial x1, or the initial
    # field, changes by one ulp (median ~1e-13).  The GPU's errors must
    # follow that distribution: median below 1e-12 and maximum within ten
    # times the largest one-ulp sensitivity.  (Per electron the sensitivity
    # to two perturbation directions underestimates the rest: 96% of the
    # electrons lie within ten times their own.)
    sens = np.zeros_like(err)
    for kind, sgn in (("x", 1.0), ("x", -1.0), ("f", 1.0), ("f", -1.0)):
        xp = xs.copy()
        Ep, Bp = Ew, Bw
        if kind == "x":
            xp[0] = xp[0] * (1 + sgn * 2.0 ** -52)
        else:
            Ep = [e * (1 + sgn * 2.0 ** -52) for e in Ew]
            Bp = [v * (1 + sgn * 2.0 ** -52) for v in Bw]
        spp = {"x": xp, "u": u[:, idx].copy(), "q": -1.0, "m": 1.0, "w": 1.0}
        pic.run(Ep, Bp, [spp], CE, CB, DX, wl.DT, steps, pusher="analytic")
        sens = np.maximum(sens, np.linalg.norm(spp["u"] - sp["u"], axis=0) / nrm)
    frac = float(np.mean(err <= np.maximum(1e-12, 10 * sens)))
    print(f"FP64 plane-wave electrons: error median {np.median(err):.1e} max {err.max():.1e}; "
          f"one-ulp sensitivity median {np.median(sens):.1e} max {sens.max():.1e}; "
          f"{100 * frac:.2f}% within max(1e-12, 10 x own sensitivity)", flush=True)
    check(float(np.median(err)), 1e-12, "FP64 plane wave electrons u (median)")
    check(float(err.max()), 10 * float(sens.max()), "FP64 plane wave electrons u (max) vs 10 x largest sensitivity")
    # closed form for every 256th electron (16384)
    cf = np.arange(0, x.shape[1], 256)
    g_gpu = np.sqrt(1 + np.sum(ug[:, cf] ** 2, axis=0))
    tt = (steps - 0.5) * wl.DT
    _, _, gcf = tj.state_at(pw.a, -1.0, -0.5 * wl.DT, x[:, cf], tt)
    dev_cf = np.abs(g_gpu - gcf) / np.max(gcf - 1)
    print(f"closed form over {cf.size} electrons: max {dev_cf.max():.3f}, median {np.median(dev_cf):.3f}", flush=True)
    check(float(dev_cf.max()), 0.25, "FP64 plane wave gamma vs closed form")
    grid.close()
