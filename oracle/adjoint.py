"""Reference gradients of the hot path: the forward step written in plain
PyTorch CPU FP64 ops, differentiated by torch.autograd.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The forward here restates, operation for operation, the NumPy oracle's field
sweep (Eq. maxwell with the App. B operators), linear-shape gather (App. A),
Boris and exact pushes (Sec. 1) and leapfrog position update (Sec. 4.1);
tests pin it to the NumPy oracle's values.  The exact push's root tau* of
t(tau) = dt is differentiated implicitly (see ``analytic``).  Its autograd gradient is then the plain
definition of the adjoint (the transposed Jacobian applied to a cotangent),
against which the GPU's hand-written adjoint is compared.

Losses (readings of the optimisation targets, which the paper does not
define):
  L_gamma = mean over electrons of the final gamma = sqrt(1 + |u|^2);
  L_phase = sum (E2 - E2_ref)^2 / sum E2_ref^2, E2_ref a reference field
            (the initial pulse translated by the elapsed time).
"""
from __future__ import annotations

import torch

X1, X2, X3 = 2, 1, 0


def d1_faraday(f, C, dx1):
    """App. B Faraday x1 operator: (1/dx1) sum_j C_j (f_{i+j} - f_{i-j+1})."""
    out = torch.zeros_like(f)
    for j in range(1, C.shape[0] + 1):
        out = out + C[j - 1] * (torch.roll(f, -j, X1) - torch.roll(f, j - 1, X1))
    return out / dx1


def d1_ampere(f, C, dx1):
    """App. B Ampere x1 operator: (1/dx1) sum_j C_j (f_{i+j-1} - f_{i-j})."""
    out = torch.zeros_like(f)
    for j in range(1, C.shape[0] + 1):
        out = out + C[j - 1] * (torch.roll(f, -(j - 1), X1) - torch.roll(f, j, X1))
    return out / dx1


def d_fwd(f, axis, d):
    """Yee forward difference (x2, x3 in Faraday's law, Sec. 3.1.1)."""
    return (torch.roll(f, -1, axis) - f) / d


def d_bwd(f, axis, d):
    """Yee backward difference (x2, x3 in Ampere's law, Sec. 3.1.1)."""
    return (f - torch.roll(f, 1, axis)) / d


def curl_E(E, CE, dx):
    """Curl in Faraday's law, Eq. maxwell (E locations -> B locations)."""
    E1, E2, E3 = E
    return (d_fwd(E3, X2, dx[1]) - d_fwd(E2, X3, dx[2]),
            d_fwd(E1, X3, dx[2]) - d1_faraday(E3, CE, dx[0]),
            d1_faraday(E2, CE, dx[0]) - d_fwd(E1, X2, dx[1]))


def curl_B(B, CB, dx):
    """Curl in Ampere's law, Eq. maxwell (B locations -> E locations)."""
    B1, B2, B3 = B
    return (d_bwd(B3, X2, dx[1]) - d_bwd(B2, X3, dx[2]),
            d_bwd(B1, X3, dx[2]) - d1_ampere(B3, CB, dx[0]),
            d1_ampere(B2, CB, dx[0]) - d_bwd(B1, X2, dx[1]))


def sweep(E, B, CE, CB, dx, dt):
    """B half step, E step, B half step (vacuum)."""
    c = curl_E(E, CE, dx)
    Bh = tuple(b - dt / 2 * ci for b, ci in zip(B, c))
    c = curl_B(Bh, CB, dx)
    En = tuple(e + dt * ci for e, ci in zip(E, c))
    c = curl_E(En, CE, dx)
    Bn = tuple(b - dt / 2 * ci for b, ci in zip(Bh, c))
    return En, Bn


E_OFF = ((0.5, 0.0, 0.0), (0.0, 0.5, 0.0), (0.0, 0.0, 0.5))
B_OFF = ((0.0, 0.5, 0.5), (0.5, 0.0, 0.5), (0.5, 0.5, 0.0))


def _axis(xd, dx, off, n):
    """Linear-shape nodes and weights along one direction (App. A); the cell
    coordinate is x * (1/dx), as in the FP64 oracle."""
    u = xd * (1.0 / dx) - off
    i0 = torch.floor(u.detach())
    w1 = u - i0
    i0 = i0.to(torch.int64)
    return i0 % n, (i0 + 1) % n, 1.0 - w1, w1


def gather_component(f, x, dx, off, ndim):
    """App. A: one component interpolated from its own staggered nodes."""
    n3, n2, n1 = f.shape
    a0, a1, wa0, wa1 = _axis(x[0], dx[0], off[0], n1)
    b0, b1, wb0, wb1 = _axis(x[1], dx[1], off[1], n2)
    if ndim == 2:
        g = f[0]
        return (wb0 * (wa0 * g[b0, a0] + wa1 * g[b0, a1]) + wb1 * (wa0 * g[b1, a0] + wa1 * g[b1, a1]))
    c0, c1, wc0, wc1 = _axis(x[2], dx[2], off[2], n3)
    return (wc0 * (wb0 * (wa0 * f[c0, b0, a0] + wa1 * f[c0, b0, a1]) + wb1 * (wa0 * f[c0, b1, a0] + wa1 * f[c0, b1, a1]))
            + wc1 * (wb0 * (wa0 * f[c1, b0, a0] + wa1 * f[c1, b0, a1]) + wb1 * (wa0 * f[c1, b1, a0] + wa1 * f[c1, b1, a1])))


def gather(E, B, x, dx, ndim):
    """Fields at the particles, (3, np) each (App. A)."""
    Ep = torch.stack([gather_component(E[c], x, dx, E_OFF[c], ndim) for c in range(3)])
    Bp = torch.stack([gather_component(B[c], x, dx, B_OFF[c], ndim) for c in range(3)])
    return Ep, Bp


def boris(u, Ep, Bp, qm, dt):
    """Sec. 1: half electric kick, magnetic rotation, half kick."""
    eps = qm * dt / 2
    um = u + eps * Ep
    g = torch.sqrt(1.0 + torch.sum(um * um, 0))
    t = eps * Bp / g
    s = 2 * t / (1.0 + torch.sum(t * t, 0))
    up = um + torch.cross(um, t, dim=0)
    upl = um + torch.cross(up, s, dim=0)
    return upl + eps * Ep


def field_tensor(Ep, Bp):
    """The 4x4 field matrix Lambda(E, B) acting on (gamma, u), per particle:
    shape (np, 4, 4) (Sec. 1, the exact pusher's equation of motion)."""
    E1, E2, E3 = Ep
    B1, B2, B3 = Bp
    z = torch.zeros_like(E1)
    rows = [torch.stack([z, E1, E2, E3], -1), torch.stack([E1, z, B3, -B2], -1),
            torch.stack([E2, -B3, z, B1], -1), torch.stack([E3, B2, -B1, z], -1)]
    return torch.stack(rows, -2)


def _exp_and_integral(F, tau):
    """expm(F tau) and int_0^tau expm(F s) ds from the 8x8 block exponential."""
    n = F.shape[0]
    aug = torch.zeros((n, 8, 8), dtype=F.dtype)
    aug[:, :4, :4] = F * tau[:, None, None]
    aug[:, :4, 4:] = torch.eye(4, dtype=F.dtype)[None] * tau[:, None, None]
    ex = torch.linalg.matrix_exp(aug)
    return ex[:, :4, :4], ex[:, :4, 4:]


def analytic(u, Ep, Bp, qm, dt, max_iter=20000):
    """Exact push for fields constant over the step (Sec. 1, Sec. 4.1): the
    proper-time exponential with t(tau*) = dt.  tau* is found without
    gradients (bracketed Newton); the returned momentum uses
    tau = tau* - (t(tau*) - dt)/gamma(tau*), whose value is tau* and whose
    derivative is the implicit-function one, -(dt/dtheta)/gamma."""
    F = qm * field_tensor(Ep, Bp)
    g0 = torch.sqrt(1.0 + torch.sum(u * u, 0))
    U0 = torch.cat([g0[None], u], 0).T  # (np, 4)
    with torch.no_grad():
        Fd, U0d = F.detach(), U0.detach()
        n = U0d.shape[0]
        lo = torch.full((n,), min(0.0, dt), dtype=u.dtype)
        hi = torch.full((n,), max(0.0, dt), dtype=u.dtype)
        tau = dt / U0d[:, 0]
        done = torch.zeros(n, dtype=torch.bool)
        for _ in range(max_iter):
            ex, it = _exp_and_integral(Fd, tau)
            tval = torch.einsum("pj,pj->p", it[:, 0, :], U0d)
            gam = torch.einsum("pj,pj->p", ex[:, 0, :], U0d)
            f = tval - dt
            finite = torch.isfinite(f) & torch.isfinite(gam)
            hit = finite & (torch.abs(f) <= 1e-16 * abs(dt))
            over = torch.where(finite, f > 0, torch.full_like(finite, dt > 0))
            hi = torch.where(over, tau, hi)
            lo = torch.where(over, lo, tau)
            newt = tau - f / gam
            bad = ~finite | ~((newt > lo) & (newt < hi))
            nxt = torch.where(bad, 0.5 * (lo + hi), newt)
            small = torch.abs(nxt - tau) <= 1e-15 * torch.abs(tau)
            tau = torch.where(done | hit, tau, nxt)
            done |= hit | small
            if bool(done.all()):
                break
        if not bool(done.all()):
            raise RuntimeError("exact pusher: t(tau) = dt not solved")
        ex, _ = _exp_and_integral(Fd, tau)
        gam_star = torch.einsum("pj,pj->p", ex[:, 0, :], U0d)
    _, it = _exp_and_integral(F, tau)
    t_star = torch.einsum("pj,pj->p", it[:, 0, :], U0)
    tau_g = tau - (t_star - dt) / gam_star
    ex, _ = _exp_and_integral(F, tau_g)
    U = torch.einsum("pij,pj->pi", ex, U0)
    return U[:, 1:].T


def advance_position(x, u, dt, L, ndim):
    """x + dt u/gamma, then the periodic wrap of the NumPy oracle (a
    piecewise-constant shift, so its derivative is the identity)."""
    g = torch.sqrt(1.0 + torch.sum(u * u, 0))
    rows = []
    for d in range(ndim):
        v = x[d] + dt * u[d] / g
        vd = v.detach()
        Ld = torch.tensor(L[d], dtype=v.dtype)
        shift = torch.where(vd < 0, -Ld, torch.where(vd >= Ld, Ld, torch.zeros_like(Ld)))
        v = v - shift
        v = torch.where((vd < 0) & (v.detach() >= L[d]), v - v.detach(), v)
        rows.append(v)
    if ndim == 2 and x.shape[0] == 3:
        rows.append(x[2])
    return torch.stack(rows)


def step(E, B, x, u, CE, CB, dx, dt, qm, L, ndim, pusher="boris"):
    """One vacuum step with test particles: gather + push + position, sweep."""
    Ep, Bp = gather(E, B, x, dx, ndim)
    u = boris(u, Ep, Bp, qm, dt) if pusher == "boris" else analytic(u, Ep, Bp, qm, dt)
    x = advance_position(x, u, dt, L, ndim)
    E, B = sweep(E, B, CE, CB, dx, dt)
    return E, B, x, u


def run(E, B, x, u, CE, CB, dx, dt, qm, nsteps, ndim, pusher="boris"):
    """``nsteps`` calls of ``step`` on a periodic mesh."""
    n3, n2, n1 = E[0].shape
    L = [n1 * dx[0], n2 * dx[1], n3 * dx[2]]
    for _ in range(nsteps):
        E, B, x, u = step(E, B, x, u, CE, CB, dx, dt, qm, L, ndim, pusher)
    return E, B, x, u


def loss_gamma(u):
    """Mean final gamma of the electrons (reading stated above)."""
    return torch.mean(torch.sqrt(1.0 + torch.sum(u * u, 0)))


def loss_phase(E2, E2_ref):
    """Normalised squared deviation of E2 from a reference (reading above)."""
    return torch.sum((E2 - E2_ref) ** 2) / torch.sum(E2_ref ** 2)
