"""The three pushers evaluated in high precision (mpmath), one particle at a time.

TEST INFRASTRUCTURE ONLY (see the package docstring).

In strong fields (|E|, |B| ~ 1e4 with dt ~ 0.1, the a0 = 1e4 runs of Sec. 4.1)
an FP64 evaluation of a push loses digits: the Boris and Higuera-Cary
formulas subtract quantities of order q E dt from each other, and the exact
push of ``particles.analytic`` exponentiates a field tensor of large norm.
These functions evaluate the same definitions from the same FP64 inputs at
``dps`` significant digits (50 by default) and round the result to FP64 once,
so that any FP64 implementation can be measured against the exact value of
the map at its own inputs.

Passages followed (the definitions are those of ``particles``)
-------------------------------------------------------------
* Sec. 1, Boris: u- = u + h E, t = h B/gamma(u-), s = 2t/(1 + t^2),
  u' = u- + u- x t, u+ = u- + u' x s, result u+ + h E, with h = q dt/(2m).
* Sec. 1 / Sec. 4.1, Higuera-Cary (cited there): u- = u + h E, tau = h B,
  sigma = 1 + u-^2 - tau^2, gamma_r^2 = (sigma + sqrt(sigma^2 + 4 (tau^2 +
  (u-.tau)^2)))/2, t = tau/gamma_r, u+ = (u- + (u-.t) t + u- x t)/(1 + t^2),
  result u+ + h E + u+ x t.
* Sec. 1 / Sec. 4.1, exact push for fields constant over the step: with
  F = (q/m) Lambda(E, B), (gamma, u)(tau) = expm(F tau) (gamma, u)(0) and
  t(tau) = e0 . [int_0^tau expm(F s) ds] (gamma, u)(0); both come from the
  8x8 block exponential expm([[F, I], [0, 0]] tau).  t(tau) = dt is solved by
  Newton's method (on log(t/dt) where t/dt is outside (1/2, 2), since t can
  grow like exp(kappa tau)), safeguarded by bisection on a bracket [lo, hi]
  of the root (t increases with tau and the root lies between 0 and dt),
  until |t - dt| is below 10^-(dps-5) |dt|.
"""
from __future__ import annotations

import mpmath as mp


def _vec(v):
    return [mp.mpf(float(c)) for c in v]


def _cross(a, b):
    return [a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]]


def _dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def boris(u, E, B, qm, dt, dps=50):
    """Sec. 1 Boris push of one particle; returns u^{n+1/2} as 3 floats."""
    with mp.workdps(dps):
        u, E, B = _vec(u), _vec(E), _vec(B)
        h = mp.mpf(float(qm)) * mp.mpf(float(dt)) / 2
        um = [u[i] + h * E[i] for i in range(3)]
        g = mp.sqrt(1 + _dot(um, um))
        t = [h * B[i] / g for i in range(3)]
        s = [2 * t[i] / (1 + _dot(t, t)) for i in range(3)]
        c1 = _cross(um, t)
        up = [um[i] + c1[i] for i in range(3)]
        c2 = _cross(up, s)
        return [float(um[i] + c2[i] + h * E[i]) for i in range(3)]


def higuera_cary(u, E, B, qm, dt, dps=50):
    """Sec. 1 / 4.1 Higuera-Cary push of one particle; returns 3 floats."""
    with mp.workdps(dps):
        u, E, B = _vec(u), _vec(E), _vec(B)
        h = mp.mpf(float(qm)) * mp.mpf(float(dt)) / 2
        um = [u[i] + h * E[i] for i in range(3)]
        tau = [h * B[i] for i in range(3)]
        tau2 = _dot(tau, tau)
        ust = _dot(um, tau)
        sigma = 1 + _dot(um, um) - tau2
        gr = mp.sqrt((sigma + mp.sqrt(sigma * sigma + 4 * (tau2 + ust * ust))) / 2)
        t = [c / gr for c in tau]
        s = 1 / (1 + _dot(t, t))
        ut = _dot(um, t)
        c1 = _cross(um, t)
        up = [s * (um[i] + ut * t[i] + c1[i]) for i in range(3)]
        c2 = _cross(up, t)
        return [float(up[i] + h * E[i] + c2[i]) for i in range(3)]


def field_tensor(E, B, qm):
    """(q/m) Lambda(E, B) as a 4x4 mpmath matrix (rows (0, E), (E1, 0, B3,
    -B2), (E2, -B3, 0, B1), (E3, B2, -B1, 0))."""
    E1, E2, E3 = E
    B1, B2, B3 = B
    rows = [[0, E1, E2, E3], [E1, 0, B3, -B2], [E2, -B3, 0, B1], [E3, B2, -B1, 0]]
    F = mp.matrix(4, 4)
    for i in range(4):
        for j in range(4):
            F[i, j] = qm * rows[i][j]
    return F


def _block_exp(F, tau):
    """expm([[F tau, I tau], [0, 0]]): the upper blocks are expm(F tau) and
    int_0^tau expm(F s) ds."""
    A = mp.zeros(8, 8)
    for i in range(4):
        for j in range(4):
            A[i, j] = F[i, j] * tau
        A[i, 4 + i] = tau
    return mp.expm(A)


def exact(u, E, B, qm, dt, dps=50, max_iter=2000):
    """Exact push of one particle for fields constant over the step (see the
    module docstring); returns u^{n+1/2} as 3 floats.  Raises if the root of
    t(tau) = dt is not found."""
    with mp.workdps(dps):
        u, E, B = _vec(u), _vec(E), _vec(B)
        qm = mp.mpf(float(qm))
        dt = mp.mpf(float(dt))
        F = field_tensor(E, B, qm)
        U0 = [mp.sqrt(1 + _dot(u, u))] + u
        lo, hi = min(mp.mpf(0), dt), max(mp.mpf(0), dt)
        tol = mp.mpf(10) ** (-(dps - 5)) * abs(dt)
        tau = dt / U0[0]
        for _ in range(max_iter):
            X = _block_exp(F, tau)
            t = sum(X[0, 4 + j] * U0[j] for j in range(4))
            gam = sum(X[0, j] * U0[j] for j in range(4))
            f = t - dt
            if abs(f) <= tol:
                break
            if f > 0:
                hi = tau
            else:
                lo = tau
            ratio = t / dt
            if ratio > 0 and not (mp.mpf(1) / 2 < ratio < 2):
                nxt = tau - mp.log(ratio) * t / gam
            else:
                nxt = tau - f / gam
            if not (lo < nxt < hi):
                nxt = (lo + hi) / 2
            tau = nxt
        else:
            raise RuntimeError("exact push: t(tau) = dt not solved")
        X = _block_exp(F, tau)
        return [float(sum(X[1 + i, j] * U0[j] for j in range(4))) for i in range(3)]
