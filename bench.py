"""Benchmark of the dual-stencil PIC hot path on one MI355X.

Default workload (the one the headline metric is quoted on): 3D vacuum mesh
1024 x 256 x 256 cells, dx1 = lambda0/32, dx2 = dx3 = lambda0/8,
dt = dx1/2, FP64 fields and particles; Gaussian laser (w0 = 4 lambda0,
a0 = 100, sin^2 envelope of 10 cycles, head at x1 = 12 lambda0); 1,048,576
electrons at rest, uniform in a 64^3-cell box on the axis at
x1 in [13, 15] lambda0; M = 16 proposed-solver coefficients (App. B, fitted
by the library); exact constant-field pusher.  One step = gather + push +
position update of every electron + one fused B-half/E/B-half field sweep.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras] [--no-cpu]

Prints one JSON line.  ``value`` is cell-updates/s of the whole step with
inputs resident in HBM.  ``roofline`` is the fused sweep's algorithmic HBM
traffic per launch over its average launch time (HIP events on the stream
the kernel runs on).  ``cpu_baseline`` times the FP64 CPU oracle on a
bounded sample of the same workload, in a child process with one thread.
Extras: the same step with FP32 fields (mixed precision), and the 3D plane
wave a0 = 1e4 mesh 2048 x 512 x 512 in FP32 vs FP64 fields.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cell-updates/s + particle-pushes/s (FP64 vs FP32-field); fwd+adjoint step ms"
HBM_PEAK_GBS = 8000.0
FP64_VALU_PEAK_TFLOPS = 78.6  # MI355X vector FP64 (FMA counted as two flops)
# Algorithmic FP64 work per particle of the plasma step (Boris, linear shape):
# staggered gather 126 (six trilinear interpolations of 21 flops), Boris 60,
# position update 14, Esirkepov deposit about 300 (shape differences, 27
# weights of 7 flops, running sums and scaling), an FMA counted as two.
PLASMA_FLOPS_PER_PARTICLE = 500
# The exact pusher per particle: gather 126, invariants and three applications
# of the field tensor about 100, about five Newton iterations of the
# Cayley-Hamilton coefficients and t(tau) (about 150 each), the final
# exponential and position update about 30.
EXACT_FLOPS_PER_PARTICLE = 1000


def _device_fields(n, dx, pulse, x_head, w0, dtype, torch):
    from paper_2004_03754_amd import workloads as wl
    e2, b3, prof = wl.laser_profiles(n, dx, pulse, x_head, w0)
    n1, n2, n3 = n
    dev = "cuda:0"
    P = torch.as_tensor(prof, device=dev, dtype=torch.float64)
    E = [torch.zeros((n3, n2, n1), device=dev, dtype=dtype) for _ in range(3)]
    B = [torch.zeros((n3, n2, n1), device=dev, dtype=dtype) for _ in range(3)]
    E[1].copy_((P[:, :, None] * torch.as_tensor(e2, device=dev)[None, None, :]).to(dtype))
    B[2].copy_((P[:, :, None] * torch.as_tensor(b3, device=dev)[None, None, :]).to(dtype))
    lon = wl.laser_longitudinal(n, dx, pulse, x_head, w0)
    if lon is not None:  # the Gaussian beam's longitudinal E1, B1
        e1, p1, b1, q1 = (torch.as_tensor(a, device=dev, dtype=torch.float64) for a in lon)
        E[0].copy_((p1[:, :, None] * e1[None, None, :]).to(dtype))
        B[0].copy_((q1[:, :, None] * b1[None, None, :]).to(dtype))
    return E, B


def _device_plane_wave(n, dx, a0, dtype, torch):
    """Monochromatic plane wave a = a0 sin(t - x1) at t = 0, polarisation x2:
    E2 = B3 = -a0 cos(x_head - x1) sampled at the staggered x1 locations."""
    from paper_2004_03754_amd import workloads as wl
    return _device_fields(n, dx, wl.PlaneWave(a0=a0), 0.0, None, dtype, torch)


def _device_uniform_particles(npart, lo, hi, seed, torch):
    """Uniform positions in [lo, hi) from a seeded device generator; at rest."""
    g = torch.Generator(device="cuda:0")
    g.manual_seed(seed)
    lo = torch.tensor(lo, device="cuda:0", dtype=torch.float64)[:, None]
    hi = torch.tensor(hi, device="cuda:0", dtype=torch.float64)[:, None]
    x = lo + (hi - lo) * torch.rand((3, npart), generator=g, device="cuda:0", dtype=torch.float64)
    return x.contiguous(), torch.zeros_like(x)


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def run_vacuum(torch, b, wl, n, prec, pulse, x_head, w0, npart, box, steps, warmup, pusher, seed, CE, CB,
               sweep_reps=20):
    """Set up a vacuum run, time ``steps`` full steps and ``sweep_reps``
    field sweeps alone.  Returns a dict of measurements."""
    dx = (wl.DX1, wl.DX2, wl.DX3)
    dtype = torch.float64 if prec == "fp64" else torch.float32
    E, B = _device_fields(n, dx, pulse, x_head, w0, dtype, torch)
    x, u = wl.uniform_particles(npart, box[0], box[1], seed=seed)
    xd = torch.as_tensor(x, device="cuda:0").contiguous()
    ud = torch.as_tensor(u, device="cuda:0").contiguous()
    grid = b.Grid(E, B, dx, wl.DT, CE, CB, prec=prec)
    p = b.Particles(xd, ud, q=-1.0, m=1.0, w=1.0)
    grid.step_n([p], warmup, pusher=pusher)
    torch.cuda.synchronize()
    t0, t1 = _events(torch)
    t0.record()
    grid.step_n([p], steps, pusher=pusher)
    t1.record()
    torch.cuda.synchronize()
    ms_step = t0.elapsed_time(t1) / steps
    # the fused sweep alone (even count: no copy-back) and the particle step alone
    reps = sweep_reps + (sweep_reps & 1)
    s0, s1 = _events(torch)
    s0.record()
    grid.step_n([], reps)
    s1.record()
    torch.cuda.synchronize()
    ms_sweep = s0.elapsed_time(s1) / reps
    q0, q1 = _events(torch)
    q0.record()
    for _ in range(reps):
        grid.gather_push(p, pusher)
    q1.record()
    torch.cuda.synchronize()
    ms_push = q0.elapsed_time(q1) / reps
    grid.check(p)
    cells = n[0] * n[1] * n[2]
    elem = 8 if prec == "fp64" else 4
    out = dict(cells=cells, npart=npart, ms_step=ms_step, ms_sweep=ms_sweep, ms_push=ms_push,
               sweep_bytes=12 * elem * cells, push_bytes=96 * npart)
    grid.close()
    del E, B, xd, ud
    torch.cuda.empty_cache()
    return out


def run_plane_wave(torch, b, wl, CE, CB, steps):
    """Mixed-precision workload: 2048 x 512 x 512 cells, plane wave a0 = 1e4
    along x1 (exactly periodic over 64 lambda0), 4,194,304 electrons at rest
    spread over the box, exact pusher; FP32 fields, then FP64 fields."""
    dx = (wl.DX1, wl.DX2, wl.DX3)
    n = (2048, 512, 512)
    L = [n[d] * dx[d] for d in range(3)]
    out = {}
    keep = {}
    for prec in ("fp32", "fp64"):
        dtype = torch.float32 if prec == "fp32" else torch.float64
        E, B = _device_plane_wave(n, dx, 1.0e4, dtype, torch)
        xd, ud = _device_uniform_particles(1 << 22, [0, 0, 0], L, 5, torch)
        grid = b.Grid(E, B, dx, wl.DT, CE, CB, prec=prec)
        p = b.Particles(xd, ud, q=-1.0, m=1.0, w=1.0)
        grid.step_n([p], 2, pusher="analytic")
        torch.cuda.synchronize()
        t0, t1 = _events(torch)
        t0.record()
        grid.step_n([p], steps, pusher="analytic")
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / steps
        s0, s1 = _events(torch)
        s0.record()
        grid.step_n([], 4)
        s1.record()
        torch.cuda.synchronize()
        ms_sweep = s0.elapsed_time(s1) / 4
        cells = n[0] * n[1] * n[2]
        elem = 4 if prec == "fp32" else 8
        gbps = 12 * elem * cells / (ms_sweep * 1e-3) / 1e9
        out[prec] = {"ms_per_step": ms, "cell_updates_per_s": cells / (ms * 1e-3),
                     "particle_pushes_per_s": (1 << 22) / (ms * 1e-3), "sweep_ms": ms_sweep,
                     "sweep_GBps": gbps, "sweep_hbm_frac": gbps / HBM_PEAK_GBS}
        # state for the mixed-path error: every electron's gamma and one x2-x3
        # column of the fields (the plane wave is uniform across it)
        keep[prec] = (torch.sqrt(1.0 + torch.sum(ud * ud, 0)),
                      [f[0, 0, :].to(torch.float64).clone() for f in E + B])
        grid.close()
        del E, B, xd, ud, grid, p
        torch.cuda.empty_cache()
        # plain copies of six arrays of the same size, for the sweep's share of them
        ceil_gbps, _ = stream_ceiling(torch, cells, reps=2, dtype=dtype)
        out[prec]["stream_ceiling_GBps"] = ceil_gbps
        out[prec]["sweep_frac_of_stream_ceiling"] = gbps / ceil_gbps
    g32, f32 = keep["fp32"]
    g64, f64 = keep["fp64"]
    rel = (torch.abs(g32 - g64) / g64).cpu()
    fscale = max(float(torch.max(torch.abs(f))) for f in f64)
    ferr = max(float(torch.max(torch.abs(a - c))) for a, c in zip(f32, f64)) / fscale
    out["mixed_path_error_vs_fp64_path"] = {
        "steps": steps + 2, "field_joint_norm": ferr,
        "gamma_rel_median": float(torch.median(rel)), "gamma_rel_p99": float(torch.quantile(rel[::16], 0.99)),
        "gamma_rel_max": float(torch.max(rel)),
        "note": "FP32-field run against the FP64-field run of the same GPU from the same state, all 4M electrons"}
    out["fp32_speedup_step"] = out["fp64"]["ms_per_step"] / out["fp32"]["ms_per_step"]
    out["fp32_speedup_sweep"] = out["fp64"]["sweep_ms"] / out["fp32"]["sweep_ms"]
    return out


def run_plasma(torch, b, wl, CE, CB, steps, dt=None, order=1):
    """Plasma workload: 512 x 256 x 256 cells, electrons at n = 0.01 n_c with
    8 per cell (268,435,456), u_th = 0.01, Gaussian laser a0 = 10, w0 = 4
    lambda0; Boris pusher, Esirkepov deposit; FP32 fields, FP64 particles.
    ``dt`` defaults to dx1/2; at dt = dx1/4 the proposed solver's Ampere
    stencil is wide, so each step also runs the x1 current correction, which
    is then timed alone as well.  ``order`` 2 runs the quadratic particle
    shape (the Sec. 4.2 run's)."""
    dt = wl.DT if dt is None else dt
    dx = (wl.DX1, wl.DX2, wl.DX3)
    n = (512, 256, 256)
    L0 = wl.LAMBDA0
    pulse = wl.Sin2Pulse(a0=10.0, Lp=10 * L0, period=n[0] * dx[0])
    E, B = _device_fields(n, dx, pulse, 12 * L0, 4 * L0, torch.float32, torch)
    J = [torch.zeros_like(E[0]) for _ in range(3)]
    xd, ud = wl.device_lattice_particles(n, dx, 2, 0.01, 3, torch)
    npart = xd.shape[1]
    grid = b.Grid(E, B, dx, dt, CE, CB, J=J, prec="fp32")
    grid.set_shape(order)
    p = b.Particles(xd, ud, q=-1.0, m=1.0, w=0.01 / 8)
    grid.step_n([p], 2, pusher="boris", deposit=True)
    torch.cuda.synchronize()
    t0, t1 = _events(torch)
    t0.record()
    grid.step_n([p], steps, pusher="boris", deposit=True)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    xo = torch.empty_like(xd)
    q0, q1 = _events(torch)
    q0.record()
    grid.gather_push(p, "boris", x_old=xo)
    q1.record()
    torch.cuda.synchronize()
    d0, d1 = _events(torch)
    d0.record()
    grid.deposit_J(p, xo, zero_first=True)
    d1.record()
    torch.cuda.synchronize()
    grid.check(p)
    cells = n[0] * n[1] * n[2]
    step_bytes = 96 * npart + 60 * cells
    out = {"ms_per_step": ms, "particles": npart, "particle_pushes_per_s": npart / (ms * 1e-3),
           "cell_updates_per_s": cells / (ms * 1e-3),
           "gather_push_ms": q0.elapsed_time(q1), "deposit_ms": d0.elapsed_time(d1),
           "step_roofline": {
               "hbm_frac": step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
               "fp64_valu_frac": PLASMA_FLOPS_PER_PARTICLE * npart / (ms * 1e-3) / 1e12 / FP64_VALU_PEAK_TFLOPS,
               "note": "whole step (sort every 3 steps included) against 96 B/particle + 60 B/cell of HBM "
                       "and about 500 FP64 flops/particle"}}
    if abs(dt - wl.DT) > 1e-15:
        jc = torch.empty_like(J[0])
        grid.current_correction(jc)
        c0, c1 = _events(torch)
        c0.record()
        for _ in range(10):
            grid.current_correction(jc)
        c1.record()
        torch.cuda.synchronize()
        cms = c0.elapsed_time(c1) / 10
        cells = n[0] * n[1] * n[2]
        out["dt_over_dx1"] = dt / dx[0]
        out["current_correction_ms"] = cms
        out["current_correction_GBps"] = 8 * cells / (cms * 1e-3) / 1e9  # FP32: read J1 + write 4 B/cell
        del jc
    grid.close()
    del E, B, J, xd, ud, xo, grid, p
    torch.cuda.empty_cache()
    return out


def run_plasma_quarter(torch, b, wl, steps):
    """The plasma workload at dt = dx1/4 (the ratio of the paper's Sec. 4.1
    runs) with the proposed solver's coefficients for that ratio: a 16-wide
    Ampere stencil, the general fused sweep and the x1 current correction."""
    CE = b.design_coeffs(16, 0.25, "E")
    CB = b.design_coeffs(16, 0.25, "B")
    return run_plasma(torch, b, wl, CE, CB, steps, dt=wl.DX1 / 4)


def run_window(torch, b, wl, suite_steps=20000, moves=20):
    """Moving window along x1 (Sec. 4.1).  (1) The single-particle run: 2D
    window of 1024 x 4 cells, dx1 = 0.2, dx2 = 20, dt = 0.05 (r = 1/4), the
    proposed solver fitted for r = 1/4, flat-top plane wave a0 = 0.5, one
    electron drifting with gamma0 = 20, Higuera-Cary pusher, the window moving
    one cell every 4 steps (at c) with the electron passed to every move.
    (2) One-cell moves on the headline mesh (1024 x 256 x 256 FP64) with its
    1,048,576 electrons passed (count, scan and a host sync; nobody leaves)
    and without particles (the column clearing alone)."""
    dx1, dx2, dt = 0.2, 20.0, 0.05
    dx = (dx1, dx2, dx2)
    CE = b.design_coeffs(16, dt / dx1, "E")
    CB = b.design_coeffs(16, dt / dx1, "B")
    pulse = wl.FlatTopPulse(0.5)
    E, B = wl.laser_fields((1024, 4, 1), dx, pulse, x_head=180.0)
    Ed = [torch.as_tensor(e, device="cuda:0").contiguous() for e in E]
    Bd = [torch.as_tensor(v, device="cuda:0").contiguous() for v in B]
    grid = b.Grid(Ed, Bd, dx, dt, CE, CB, ndim=2)
    x = torch.tensor([[180.0 - (pulse.R + 16 * math.pi)], [0.5 * dx2], [0.0]], dtype=torch.float64,
                     device="cuda:0")
    u = torch.tensor([[math.sqrt(20.0 ** 2 - 1)], [0.0], [0.0]], dtype=torch.float64, device="cuda:0")
    p = b.Particles(x, u)
    for _ in range(25):
        grid.step_n([p], 4, pusher="hc")
        grid.move_window(1, [p])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(suite_steps // 4):
        grid.step_n([p], 4, pusher="hc")
        grid.move_window(1, [p])
    torch.cuda.synchronize()
    ms_suite = (time.perf_counter() - t0) * 1e3 / suite_steps
    grid.close()
    # one-cell moves on the headline mesh
    n = (1024, 256, 256)
    z = [torch.zeros((n[2], n[1], n[0]), dtype=torch.float64, device="cuda:0") for _ in range(6)]
    L = wl.LAMBDA0
    xs, us = wl.uniform_particles(1 << 20, [13 * L, 0.0, 0.0], [15 * L, n[1] * wl.DX2, n[2] * wl.DX3], seed=2)
    ph = b.Particles(torch.as_tensor(xs, device="cuda:0").contiguous(),
                     torch.as_tensor(us, device="cuda:0").contiguous())
    grid = b.Grid(z[:3], z[3:], (wl.DX1, wl.DX2, wl.DX3), wl.DT, [1.0], [1.0])
    grid.move_window(1, [ph])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(moves):
        grid.move_window(1, [ph])
    torch.cuda.synchronize()
    ms_move_p = (time.perf_counter() - t0) * 1e3 / moves
    e0, e1 = _events(torch)
    e0.record()
    for _ in range(moves):
        grid.move_window(1, [])
    e1.record()
    torch.cuda.synchronize()
    ms_move = e0.elapsed_time(e1) / moves
    grid.close()
    del z, ph
    torch.cuda.empty_cache()
    return {"suite_2d_1024x4_ms_per_step": ms_suite, "suite_steps": suite_steps,
            "headline_move_with_1M_electrons_ms": ms_move_p, "headline_move_fields_only_ms": ms_move,
            "survivors": int(p.np)}


def run_adjoint(torch, b, wl, CE, CB, steps, K=64):
    """Adjoint workload: a batch of 16 2D meshes of 2048 x 256 cells (stacked
    planes of one grid), one sin^2 envelope per plane with a0 = 10^U(0,3)
    (seed 4), L_p = 10 lambda0, head at 12 lambda0; 64 electrons per plane at
    rest, evenly spaced over 2 lambda0 ahead of the head on the middle x2
    line; Boris pusher, FP64, checkpoints every K steps.  Losses: mean final
    gamma and the vacuum phase error of E2 against the initial pulse moved on
    by the elapsed time; gradients of each with respect to C^E, C^B and
    (a0, L_p, head) of every plane.  Returns ms per step of the forward pass
    and of each backward pass (recomputation + adjoint)."""
    from paper_2004_03754_amd import autograd as pa

    n1, n2, nb, npb = 2048, 256, 16, 64
    dx = (wl.DX1, wl.DX2, wl.DX3)
    L0 = wl.LAMBDA0
    g = wl.rng(4)
    a0 = torch.tensor(10.0 ** (3.0 * g.random(nb)), dtype=torch.float64, requires_grad=True)
    Lp = torch.full((nb,), 10 * L0, dtype=torch.float64, requires_grad=True)
    head = torch.full((nb,), 12 * L0, dtype=torch.float64, requires_grad=True)
    x = torch.zeros((3, nb * npb), dtype=torch.float64)
    x[0] = (12.5 * L0 + torch.arange(npb, dtype=torch.float64) * (2 * L0 / npb)).repeat(nb)
    x[1] = 0.5 * n2 * dx[1]
    x[2] = torch.arange(nb, dtype=torch.float64).repeat_interleave(npb) + 0.5
    xd = x.to("cuda:0").contiguous()
    ud = torch.zeros_like(xd)
    ce = torch.tensor(CE, dtype=torch.float64, requires_grad=True)
    cb = torch.tensor(CB, dtype=torch.float64, requires_grad=True)
    cfg = pa.RunConfig(dx, wl.DT, steps, K=K, ndim=2)
    with torch.no_grad():
        Eref, _ = pa.sin2_pulse_fields(n1, n2, nb, dx, a0, Lp, head + steps * wl.DT)
    torch.cuda.synchronize()
    f0, f1 = _events(torch)
    f0.record()
    E0, B0 = pa.sin2_pulse_fields(n1, n2, nb, dx, a0, Lp, head)
    Ef, Bf, xf, uf = pa.run(ce, cb, E0, B0, xd, ud, cfg)
    f1.record()
    gam = torch.sqrt(1.0 + torch.sum(uf * uf, 0))
    L_gamma = torch.mean(gam)
    L_phase = torch.sum((Ef[1] - Eref[1]) ** 2) / torch.sum(Eref[1] ** 2)
    leaves = [ce, cb, a0, Lp, head]
    out = {"steps": steps, "checkpoint_every": K, "planes": nb, "cells_per_plane": n1 * n2, "electrons": nb * npb}
    times = []
    for name, loss in (("gamma", L_gamma), ("phase", L_phase)):
        torch.cuda.synchronize()
        b0, b1 = _events(torch)
        b0.record()
        grads = torch.autograd.grad(loss, leaves, retain_graph=(name == "gamma"))
        b1.record()
        torch.cuda.synchronize()
        times.append(b0.elapsed_time(b1))
        out[f"L_{name}"] = float(loss)
        out[f"grad_{name}"] = {k: [float(v) for v in gr.flatten()[:4]] + (["..."] if gr.numel() > 4 else [])
                               for k, gr in zip(("CE", "CB", "a0", "Lp", "head"), grads)}
        assert all(bool(torch.isfinite(gr).all()) for gr in grads), "non-finite gradient"
    ms_fwd = f0.elapsed_time(f1) / steps
    out.update({"fwd_ms_per_step": ms_fwd, "adjoint_ms_per_step": times[0] / steps,
                "fwd_plus_adjoint_ms_per_step": ms_fwd + times[0] / steps,
                "second_adjoint_ms_per_step": times[1] / steps,
                "fwd_plus_second_adjoint_ms_per_step": ms_fwd + times[1] / steps,
                "adjoint_note": "the first backward pass also allocates the segment's state buffers (about "
                                "40 GB, once per process through the caching allocator); the second, of the "
                                "same work, runs with them cached"})
    del Ef, Bf, xf, uf, E0, B0, Eref, grads
    torch.cuda.empty_cache()
    return out


def cpu_baseline_child():
    """Runs in a child process with one thread: the oracle's step on a
    sample of the default workload (a 1024 x 32 x 32 column of the mesh with
    the same electron density per cell), cell-updates/s."""
    import numpy as np

    from oracle import pic, stencil
    from paper_2004_03754_amd import workloads as wl

    dx = (wl.DX1, wl.DX2, wl.DX3)
    n = (1024, 32, 32)
    CE, CB = stencil.fit_pair(16, 0.5)
    pulse = wl.Sin2Pulse(a0=100.0, Lp=10 * wl.LAMBDA0)
    E, B = wl.laser_fields(n, dx, pulse, x_head=12 * wl.LAMBDA0, w0=4 * wl.LAMBDA0)
    cells = n[0] * n[1] * n[2]
    npart = int(round(1048576 * cells / (1024 * 256 * 256)))
    lo = [13 * wl.LAMBDA0, 0, 0]
    hi = [15 * wl.LAMBDA0, n[1] * dx[1], n[2] * dx[2]]
    x, u = wl.uniform_particles(npart, lo, hi, seed=2)
    sp = {"x": x, "u": u, "q": -1.0, "m": 1.0, "w": 1.0}
    E, B = pic.step(E, B, [sp], CE, CB, dx, wl.DT, pusher="analytic")  # warm-up
    steps = 48
    t = time.perf_counter()
    for _ in range(steps):
        E, B = pic.step(E, B, [sp], CE, CB, dx, wl.DT, pusher="analytic")
    dt = time.perf_counter() - t
    print(json.dumps({"value": cells * steps / dt, "seconds": dt, "cells": cells, "npart": npart,
                      "steps": steps}))


def cpu_baseline():
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "NUMEXPR_NUM_THREADS"):
        env[k] = "1"
    env["CUDA_VISIBLE_DEVICES"] = ""
    env["HIP_VISIBLE_DEVICES"] = ""
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-child"], capture_output=True,
                       text=True, env=env, timeout=600)
    if r.returncode != 0:
        return {"error": r.stderr[-400:]}
    d = json.loads(r.stdout.strip().splitlines()[-1])
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": d["value"], "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "cpu_model": model, "os_cpu_count": os.cpu_count(),
            "sample": f"oracle step (exact pusher) on a 1024x32x32 column with {d['npart']} electrons, "
                      f"{d['steps']} steps after 1 warm-up, {d['seconds']:.1f} s, NumPy FP64 single thread"}


def stream_ceiling(torch, nelem, reps=5, dtype=None):
    """The HBM rate of a plain device copy (STREAM copy) of six arrays of
    ``nelem`` elements (FP64 unless ``dtype``), one copy after another, timed
    over ``reps`` rounds: 12 array passes, the traffic of a sweep without its
    stencil."""
    dtype = torch.float64 if dtype is None else dtype
    src = [torch.empty(nelem, device="cuda:0", dtype=dtype) for _ in range(6)]
    dst = [torch.empty_like(a) for a in src]
    for a, c in zip(src, dst):
        c.copy_(a)
    torch.cuda.synchronize()
    t0, t1 = _events(torch)
    t0.record()
    for _ in range(reps):
        for a, c in zip(src, dst):
            c.copy_(a)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    elem = src[0].element_size()
    del src, dst
    torch.cuda.empty_cache()
    return 12 * elem * nelem / (ms * 1e-3) / 1e9, ms


def copy_calibration(nbytes=1 << 29, reps=3):
    """A plain device-to-device copy of ``nbytes`` (reads nbytes, writes
    nbytes), repeated ``reps`` times: the known traffic against which the HBM
    byte counters of a profiler run are scaled."""
    import torch

    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-baseline-child", action="store_true")
    ap.add_argument("--adjoint-steps", type=int, default=2048,
                    help="steps of the differentiated 2D batch run (checkpoint every 64)")
    ap.add_argument("--adjoint-only", action="store_true", help="run only the adjoint workload")
    ap.add_argument("--plasma-only", action="store_true", help="run only the plasma workload")
    ap.add_argument("--plasma-quadratic-only", action="store_true",
                    help="run only the plasma workload with the quadratic particle shape")
    ap.add_argument("--plasma-quarter-only", action="store_true",
                    help="run only the plasma workload at dt = dx1/4 (wide Ampere stencil, current correction)")
    ap.add_argument("--window-only", action="store_true",
                    help="run only the moving-window measurements (Sec. 4.1 single-particle run)")
    ap.add_argument("--plasma-steps", type=int, default=10, help="timed steps of the plasma workload")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain device copy of known size (HBM counter calibration)")
    args = ap.parse_args()
    if args.cpu_baseline_child:
        cpu_baseline_child()
        return
    if args.copy_calibration:
        copy_calibration()
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the library runs on one GPU; --gpus must be 1 (no multi-GPU slab "
              "decomposition is implemented)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2004_03754_amd import binding as b, workloads as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    r = 0.5
    CE = b.design_coeffs(16, r, "E")
    CB = b.design_coeffs(16, r, "B")
    if args.adjoint_only:
        print(json.dumps({"adjoint_2d_2048x256_x16": run_adjoint(torch, b, wl, CE, CB, steps=args.adjoint_steps)}))
        return
    if args.plasma_only:
        print(json.dumps({"plasma_512x256x256": run_plasma(torch, b, wl, CE, CB, steps=args.plasma_steps)}))
        return
    if args.plasma_quadratic_only:
        print(json.dumps({"plasma_512x256x256_quadratic": run_plasma(torch, b, wl, CE, CB, args.plasma_steps,
                                                                      order=2)}))
        return
    if args.window_only:
        print(json.dumps({"moving_window": run_window(torch, b, wl)}))
        return
    if args.plasma_quarter_only:
        print(json.dumps({"plasma_512x256x256_dt_quarter": run_plasma_quarter(torch, b, wl, args.plasma_steps)}))
        return
    L = wl.LAMBDA0
    n = (1024, 256, 256)
    dx = (wl.DX1, wl.DX2, wl.DX3)
    box = ([13 * L, (n[1] / 2 - 32) * dx[1], (n[2] / 2 - 32) * dx[2]],
           [15 * L, (n[1] / 2 + 32) * dx[1], (n[2] / 2 + 32) * dx[2]])
    pulse = wl.Sin2Pulse(a0=100.0, Lp=10 * L)
    main_run = run_vacuum(torch, b, wl, n, "fp64", pulse, 12 * L, 4 * L, 1 << 20, box, args.steps, args.warmup,
                          "analytic", 2, CE, CB)
    cells = main_run["cells"]
    value = cells / (main_run["ms_step"] * 1e-3)
    achieved = main_run["sweep_bytes"] / (main_run["ms_sweep"] * 1e-3) / 1e9
    traffic = None
    tf = os.path.join(ROOT, "profiles", "sweep_fp64_1024x256x256_traffic.json")
    if os.path.exists(tf):
        with open(tf) as f:
            traffic = json.load(f).get("bytes_per_launch")
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3D vacuum 1024x256x256 cells, FP64 fields and particles, Gaussian laser a0=100 "
                               "w0=4 lambda0, 1048576 electrons at rest, M=16 proposed solver, exact pusher",
                   "cells": cells, "electrons": main_run["npart"], "dt_over_dx1": r},
        "particle_pushes_per_s": main_run["npart"] / (main_run["ms_step"] * 1e-3),
        "kernels_ms": {"fused_sweep": main_run["ms_sweep"], "gather_push_analytic": main_run["ms_push"]},
        "gather_push_analytic_roofline": {
            "hbm_frac": main_run["push_bytes"] / (main_run["ms_push"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "fp64_valu_frac": EXACT_FLOPS_PER_PARTICLE * main_run["npart"] / (main_run["ms_push"] * 1e-3) / 1e12
            / FP64_VALU_PEAK_TFLOPS,
            "note": "96 B and about 1000 FP64 flops per exact push (estimate of the algorithm's work)"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "fused B-half/E/B-half sweep, 96 B/cell FP64"},
    }
    ceil_gbps, ceil_ms = stream_ceiling(torch, cells)
    res["stream_ceiling"] = {
        "GBps": ceil_gbps, "ms": ceil_ms, "sweep_frac_of_ceiling": achieved / ceil_gbps,
        "note": "plain device copies of six FP64 arrays of the headline mesh (STREAM copy, 12 array "
                "passes): the HBM rate a stencil-free stream reaches on this GPU"}
    if not args.no_extras:
        # mixed precision on the same workload
        fp32 = run_vacuum(torch, b, wl, n, "fp32", pulse, 12 * L, 4 * L, 1 << 20, box, max(50, args.steps // 5),
                          args.warmup, "analytic", 2, CE, CB)
        res["fp32_fields"] = {
            "cell_updates_per_s": cells / (fp32["ms_step"] * 1e-3), "ms_per_step": fp32["ms_step"],
            "sweep_ms": fp32["ms_sweep"],
            "sweep_GBps": fp32["sweep_bytes"] / (fp32["ms_sweep"] * 1e-3) / 1e9,
            "speedup_vs_fp64_step": main_run["ms_step"] / fp32["ms_step"],
            "speedup_vs_fp64_sweep": main_run["ms_sweep"] / fp32["ms_sweep"]}
        c32, _ = stream_ceiling(torch, cells, dtype=torch.float32)
        res["fp32_fields"]["stream_ceiling_GBps"] = c32
        res["fp32_fields"]["sweep_frac_of_stream_ceiling"] = res["fp32_fields"]["sweep_GBps"] / c32
        # the headline workload with the Higuera-Cary pusher (Sec. 4.1's default pusher)
        hc = run_vacuum(torch, b, wl, n, "fp64", pulse, 12 * L, 4 * L, 1 << 20, box, max(50, args.steps // 5),
                        args.warmup, "hc", 2, CE, CB)
        res["hc_pusher"] = {"cell_updates_per_s": cells / (hc["ms_step"] * 1e-3), "ms_per_step": hc["ms_step"],
                            "gather_push_ms": hc["ms_push"],
                            "particle_pushes_per_s": hc["npart"] / (hc["ms_push"] * 1e-3)}
        res["plane_wave_2048x512x512"] = run_plane_wave(torch, b, wl, CE, CB, steps=20)
        res["plasma_512x256x256"] = run_plasma(torch, b, wl, CE, CB, steps=args.plasma_steps)
        res["plasma_512x256x256_dt_quarter"] = run_plasma_quarter(torch, b, wl, args.plasma_steps)
        res["plasma_512x256x256_quadratic"] = run_plasma(torch, b, wl, CE, CB, args.plasma_steps, order=2)
        res["adjoint_2d_2048x256_x16"] = run_adjoint(torch, b, wl, CE, CB, steps=args.adjoint_steps)
        res["moving_window"] = run_window(torch, b, wl)
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline()
    print(json.dumps(res))


if __name__ == "__main__":
    main()
