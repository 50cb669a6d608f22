"""Closed-form motion of a charge starting at rest in a plane wave (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 4.1: for a plane wave moving along +x1 and polarised along x2, the
canonical momentum is conserved, p2 - a_L = const for an electron (the
theory curves of Figs. 5-8).  With the vector potential A2 = a(psi),
psi = t - x1, the fields are E2 = B3 = -a'(psi), and for charge q, mass m:
    u2(psi)    = -(q/m) (a(psi) - a(psi0))       (canonical momentum)
    gamma - u1 = 1                               (E2 = B3, start at rest)
    u1 = u2^2/2,  gamma = 1 + u2^2/2,  d psi/dt = 1/gamma
so  t - t0 = int gamma dpsi,  x1 - x1_0 = int u1 dpsi,  x2 - x2_0 = int u2 dpsi.
A start where a(psi0) = 0 gives u_perp = a, u_par = a^2/2, gamma = 1 + a^2/2
(for q/m = -1).  The integrals use composite Gauss-Legendre quadrature and
t(psi) = t is inverted by safeguarded Newton (t is increasing in psi).
"""
from __future__ import annotations

import numpy as np

_GX, _GW = np.polynomial.legendre.leggauss(16)


def _integrals(a, qm, psi0, psi, panels):
    """int_{psi0}^{psi} (gamma, u1, u2) dpsi' for arrays psi0, psi."""
    a0 = a(psi0)
    h = (psi - psi0) / panels
    tot = np.zeros((3,) + np.shape(psi))
    for p in range(panels):
        lo = psi0 + p * h
        for xg, wg in zip(_GX, _GW):
            s = lo + (xg + 1) * h / 2
            u2 = -qm * (a(s) - a0)
            u1 = 0.5 * u2 * u2
            tot[0] += wg * h / 2 * (1.0 + u1)
            tot[1] += wg * h / 2 * u1
            tot[2] += wg * h / 2 * u2
    return tot


def state_at(a, qm, t0, x0, t, max_iter=100):
    """Particles at rest at time t0 at positions x0 (shape (3, np)); returns
    (x (3, np), u (3, np), gamma (np,)) at time t (scalar)."""
    x0 = np.asarray(x0, dtype=np.float64)
    psi0 = t0 - x0[0]
    span = max(t - t0, 0.0)
    panels = max(8, int(np.ceil(span / 0.5)))
    lo = psi0.copy()
    hi = psi0 + span
    psi = psi0 + 0.5 * span
    for _ in range(max_iter):
        I = _integrals(a, qm, psi0, psi, panels)
        f = t0 + I[0] - t
        u2 = -qm * (a(psi) - a(psi0))
        g = 1.0 + 0.5 * u2 * u2
        hi = np.where(f > 0, psi, hi)
        lo = np.where(f <= 0, psi, lo)
        nxt = psi - f / g
        bad = (nxt <= lo) | (nxt >= hi)
        nxt = np.where(bad, 0.5 * (lo + hi), nxt)
        if np.all(np.abs(nxt - psi) <= 1e-15 * np.maximum(1.0, np.abs(psi))):
            psi = nxt
            break
        psi = nxt
    I = _integrals(a, qm, psi0, psi, panels)
    u2 = -qm * (a(psi) - a(psi0))
    u1 = 0.5 * u2 * u2
    x = np.stack([x0[0] + I[1], x0[1] + I[2], x0[2]])
    u = np.stack([u1, u2, np.zeros_like(u2)])
    return x, u, 1.0 + u1
