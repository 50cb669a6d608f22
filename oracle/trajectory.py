"""Closed-form motion of a charge in a plane wave, starting at rest or with a
drift along the wave (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 4.1: for a plane wave moving along +x1 and polarised along x2, the
canonical momentum is conserved, p2 - a_L = const for an electron (the
theory curves of Figs. 5-8).  With the vector potential A2 = a(psi),
psi = t - x1, the fields are E2 = B3 = -a'(psi).  Then d(gamma - u1)/dt = 0,
so h = gamma - u1 keeps its initial value (h = 1 from rest; h = gamma0 -
sqrt(gamma0^2 - 1) for a drift gamma0 along +x1 with u2 = u3 = 0 at a
point where a = a(psi0)), and for charge q, mass m:
    u2(psi)    = -(q/m) (a(psi) - a(psi0))       (canonical momentum)
    u1 = (1 + u2^2 - h^2)/(2h),  gamma = (1 + u2^2 + h^2)/(2h),
    d psi/dt = 1 - u1/gamma = h/gamma
so  t - t0 = int gamma/h dpsi,  x1 - x1_0 = int u1/h dpsi,
x2 - x2_0 = int u2/h dpsi.
A start at rest where a(psi0) = 0 gives u_perp = a, u_par = a^2/2,
gamma = 1 + a^2/2 (for q/m = -1).  The integrals use composite Gauss-Legendre
quadrature and t(psi) = t is inverted by safeguarded Newton (t is increasing
in psi).
"""
from __future__ import annotations

import numpy as np

_GX, _GW = np.polynomial.legendre.leggauss(16)


def _h(gamma0):
    """h = gamma - u1 of a start with drift gamma0 along +x1 (1 at rest)."""
    if gamma0 is None:
        return 1.0
    return float(gamma0) - np.sqrt(float(gamma0) ** 2 - 1.0)


def _momenta(a, qm, psi0, s, h):
    """(u1, u2, gamma) at phase s."""
    u2 = -qm * (a(s) - a(psi0))
    q = 1.0 + u2 * u2
    return (q - h * h) / (2 * h), u2, (q + h * h) / (2 * h)


def _integrals(a, qm, psi0, psi, panels, h=1.0):
    """int_{psi0}^{psi} (gamma, u1, u2)/h dpsi' for 1-D arrays psi0, psi:
    composite 16-point Gauss-Legendre over ``panels`` equal panels, with
    every node evaluated in one call of ``a``."""
    psi0 = np.atleast_1d(np.asarray(psi0, dtype=np.float64))
    step = (np.atleast_1d(np.asarray(psi, dtype=np.float64)) - psi0) / panels
    frac = np.arange(panels)[:, None] + (_GX[None, :] + 1) / 2  # (panels, 16)
    s = psi0 + frac[..., None] * step  # (panels, 16, np)
    u1, u2, g = _momenta(a, qm, psi0, s, h)
    w = _GW[None, :, None] / 2
    return np.stack([np.sum(w * q, axis=(0, 1)) for q in (g, u1, u2)]) * step / h


def state_at(a, qm, t0, x0, t, max_iter=100, gamma0=None):
    """Particles at time t0 at positions x0 (shape (3, np)), at rest or (with
    ``gamma0``) drifting along +x1 with Lorentz factor gamma0 and u2 = u3 = 0;
    returns (x (3, np), u (3, np), gamma (np,)) at time t (scalar, >= t0)."""
    x0 = np.asarray(x0, dtype=np.float64)
    h = _h(gamma0)
    psi0 = t0 - x0[0]
    span = max(t - t0, 0.0)
    # d psi/dt = h/gamma <= 1: psi - psi0 lies in [0, span]
    panels = max(8, int(np.ceil(span * h / 0.5)))
    lo = psi0.copy()
    hi = psi0 + span
    psi = psi0 + 0.5 * span * h
    for _ in range(max_iter):
        I = _integrals(a, qm, psi0, psi, panels, h)
        f = t0 + I[0] - t
        _, _, g = _momenta(a, qm, psi0, psi, h)
        hi = np.where(f > 0, psi, hi)
        lo = np.where(f <= 0, psi, lo)
        nxt = psi - f * h / g
        bad = (nxt <= lo) | (nxt >= hi)
        nxt = np.where(bad, 0.5 * (lo + hi), nxt)
        if np.all(np.abs(nxt - psi) <= 1e-15 * np.maximum(1.0, np.abs(psi))):
            psi = nxt
            break
        psi = nxt
    I = _integrals(a, qm, psi0, psi, panels, h)
    u1, u2, g = _momenta(a, qm, psi0, psi, h)
    x = np.stack([x0[0] + I[1], x0[1] + I[2], x0[2]])
    u = np.stack([u1, u2, np.zeros_like(u2)])
    return x, u, g
