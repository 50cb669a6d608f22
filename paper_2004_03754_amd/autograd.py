"""Differentiable vacuum PIC run: a torch.autograd.Function over the HIP
library's forward step loop and its hand-written adjoint.

Forward: ``nsteps`` steps of gather + push (Boris or exact) + position update + fused
field sweep (pic_step_n), keeping a checkpoint of the state (E, B, x, u)
every ``K`` steps.  Backward: the segments are walked in reverse; each one is
recomputed from its checkpoint one step at a time (pic_step_to, each state
written into its own buffer of K + 1, and each step's half-step field B^{n+1/2}
into one of K more), then reversed step by step with pic_adjoint_step, which
maps the cotangents of (E, B, x, u) from t^{n+1} to t^n, given both states and
B^{n+1/2}, and accumulates dL/dC^E and dL/dC^B.
The forward arithmetic is deterministic, so a recomputed state equals the
stored forward state bit for bit.

Only argument marshalling and buffer management happen here; every step of
the path runs in the library's kernels.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import binding as b


class RunConfig:
    """Grid and run constants: cell sizes, time step, number of dimensions
    (2D grids may stack independent planes along n3), species constants,
    step count, checkpoint interval and pusher ("boris" or "analytic": the
    pushers the hand-written adjoint covers)."""

    def __init__(self, dx, dt, nsteps, K=64, ndim=3, q=-1.0, m=1.0, w=1.0, pusher="boris"):
        self.dx, self.dt, self.nsteps, self.K = tuple(dx), float(dt), int(nsteps), int(K)
        self.ndim, self.q, self.m, self.w = int(ndim), float(q), float(m), float(w)
        self.pusher = str(pusher)
        assert self.nsteps >= 0 and self.K >= 1 and self.pusher in ("boris", "analytic")


def _clone_state(E, B, x, u):
    return [e.clone() for e in E], [v.clone() for v in B], x.clone(), u.clone()


class PICRun(torch.autograd.Function):
    """(C^E, C^B, E1, E2, E3, B1, B2, B3, x, u) -> the state after
    ``cfg.nsteps`` steps.  C^E and C^B are CPU float64 vectors of equal length
    M <= 16; fields are FP64 device tensors [n3][n2][n1]; x and u are FP64
    device tensors (3, np) at t^0 and t^{-1/2}."""

    @staticmethod
    def forward(ctx, CE, CB, E1, E2, E3, B1, B2, B3, x, u, cfg: RunConfig):
        E, B, x, u = _clone_state([E1, E2, E3], [B1, B2, B3], x, u)
        ce = CE.detach().cpu().numpy().astype(np.float64)
        cb = CB.detach().cpu().numpy().astype(np.float64)
        grid = b.Grid(E, B, cfg.dx, cfg.dt, ce, cb, ndim=cfg.ndim)
        p = b.Particles(x, u, q=cfg.q, m=cfg.m, w=cfg.w)
        checkpoints = []
        for s in range(0, cfg.nsteps, cfg.K):
            checkpoints.append(_clone_state(E, B, x, u))
            grid.step_n([p] if p.np else [], min(cfg.K, cfg.nsteps - s), pusher=cfg.pusher)
        grid.close()
        ctx.cfg, ctx.ce, ctx.cb, ctx.checkpoints = cfg, ce, cb, checkpoints
        ctx.coef_meta = (CE.dtype, CE.device, CE.shape[0])
        return (*E, *B, x, u)

    @staticmethod
    def backward(ctx, gE1, gE2, gE3, gB1, gB2, gB3, gx, gu):
        cfg, ce, cb = ctx.cfg, ctx.ce, ctx.cb
        ref = ctx.checkpoints[0] if ctx.checkpoints else None
        if ref is None:  # zero steps: the identity
            return (None, None, gE1, gE2, gE3, gB1, gB2, gB3, gx, gu, None)

        def start(g, like):
            return g.detach().clone().contiguous() if g is not None else torch.zeros_like(like)

        E0, B0, x0, u0 = ref
        lE = [start(g, e) for g, e in zip((gE1, gE2, gE3), E0)]
        lB = [start(g, v) for g, v in zip((gB1, gB2, gB3), B0)]
        lx, lu = start(gx, x0), start(gu, u0)
        dev = E0[0].device
        gCE = torch.zeros(b.PIC_MAX_M, dtype=torch.float64, device=dev)
        gCB = torch.zeros(b.PIC_MAX_M, dtype=torch.float64, device=dev)
        K = min(cfg.K, cfg.nsteps)
        # K + 1 state buffers: a segment's states t^{s0} .. t^{s0+n} (every
        # one is written before it is read: storage only, no copies)
        slots = [([torch.empty_like(v) for v in E0], [torch.empty_like(v) for v in B0], torch.empty_like(x0),
                  torch.empty_like(u0)) for _ in range(K + 1)]
        halves = [[torch.empty_like(v) for v in B0] for _ in range(K)]  # B^{n+1/2} of each step
        grid = b.Grid(slots[0][0], slots[0][1], cfg.dx, cfg.dt, ce, cb, ndim=cfg.ndim)
        lam = b.Particles(lx, lu, q=cfg.q, m=cfg.m, w=cfg.w)
        # the field cotangents alternate between two sets: each reverse step
        # reads one and writes the other (out of place, fused where possible)
        lE2 = [torch.empty_like(v) for v in lE]
        lB2 = [torch.empty_like(v) for v in lB]
        nseg = len(ctx.checkpoints)
        for seg in reversed(range(nseg)):
            s0 = seg * cfg.K
            n = min(cfg.K, cfg.nsteps - s0)
            # recompute the segment's states, each step written into the next
            # buffer (out of place: no field copies)
            cE, cB, cx, cu = ctx.checkpoints[seg]
            for a, c in zip(slots[0][0] + slots[0][1], cE + cB):
                a.copy_(c)
            slots[0][2].copy_(cx)
            slots[0][3].copy_(cu)
            for i in range(1, n + 1):
                prev, cur = slots[i - 1], slots[i]
                cur[2].copy_(prev[2])
                cur[3].copy_(prev[3])
                grid.set_fields(prev[0], prev[1])
                p = b.Particles(cur[2], cur[3], q=cfg.q, m=cfg.m, w=cfg.w)
                grid.step_to([p] if p.np else [], cur[0], cur[1], pusher=cfg.pusher, B_half=halves[i - 1])
            # reverse the segment (the particle adjoint needs x, u at t^n: the
            # previous buffer's, since step_to advanced the copies)
            for i in reversed(range(n)):
                st, nx = slots[i], slots[i + 1]
                grid.set_fields(st[0], st[1])
                p = b.Particles(st[2], st[3], q=cfg.q, m=cfg.m, w=cfg.w)
                sp, lp = ([p], [lam]) if p.np else ((), ())
                grid.adjoint_step(lE, lB, gCE, gCB, sp, lp, pusher=cfg.pusher, next_E=nx[0], next_B=nx[1],
                                  half_B=halves[i], out_E=lE2, out_B=lB2)
                lE, lE2 = lE2, lE
                lB, lB2 = lB2, lB
        grid.sync()
        grid.close()
        dtype, device, M = ctx.coef_meta
        gce = gCE[:M].to(device=device, dtype=dtype)
        gcb = gCB[:M].to(device=device, dtype=dtype)
        return (gce, gcb, *lE, *lB, lx, lu, None)


def run(CE, CB, E, B, x, u, cfg: RunConfig):
    """Differentiable run: returns (E, B, x, u) after cfg.nsteps steps."""
    out = PICRun.apply(CE, CB, *E, *B, x, u, cfg)
    return list(out[:3]), list(out[3:6]), out[6], out[7]


def sin2_pulse_fields(n1, n2, nplanes, dx, a0, Lp, x_head, dtype=torch.float64, device="cuda"):
    """Initial laser fields of a stack of 2D planes, one envelope per plane:
    a(s) = a0 sin^2(pi s/Lp) sin(s) on 0 <= s <= Lp (else 0), s = x_head - x1,
    E2 = B3 = -a'(s) sampled at the E2 (x1 = i dx1) and B3 (x1 = (i+1/2) dx1)
    locations, uniform along x2.  a0, Lp, x_head are tensors of length
    nplanes (differentiable); returns ([E1, E2, E3], [B1, B2, B3])."""
    i = torch.arange(n1, dtype=dtype, device=device)

    def da(s, a0_, Lp_):
        k = math.pi / Lp_
        inside = (s >= 0) & (s <= Lp_)
        v = a0_ * (k * torch.sin(2 * k * s) * torch.sin(s) + torch.sin(k * s) ** 2 * torch.cos(s))
        return torch.where(inside, v, torch.zeros_like(v))

    a0 = a0.to(device=device, dtype=dtype)[:, None]
    Lp = Lp.to(device=device, dtype=dtype)[:, None]
    xh = x_head.to(device=device, dtype=dtype)[:, None]
    e2 = -da(xh - i[None, :] * dx[0], a0, Lp)
    b3 = -da(xh - (i[None, :] + 0.5) * dx[0], a0, Lp)
    shape = (nplanes, n2, n1)
    E2 = e2[:, None, :].expand(shape).contiguous()
    B3 = b3[:, None, :].expand(shape).contiguous()
    z = torch.zeros(shape, dtype=dtype, device=device)
    return [z, E2, z.clone()], [z.clone(), z.clone(), B3]
