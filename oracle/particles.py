"""Particle side of the hot path (FP64): gather, pushers, position, deposit.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Particles are SoA: x is (3, np) (or (2, np) in 2D) with positions at integer
time t^n in [0, L_d); u = gamma*beta is (3, np) at half time t^{n-1/2}.
Normalised units c = m_e = e = 1 (Sec. 2.1); a species has charge q, mass m.

Passages followed
-----------------
* App. A: each field component is interpolated from its own staggered grid
  points with the shape S, one factor per direction: the linear
  (first-order) shape, or the quadratic B-spline that the Sec. 4.2 run lists
  in its parameter table (three nodes around the nearest one).  Staggering offsets (in cells) of the components:
  E1 (1/2,0,0) E2 (0,1/2,0) E3 (0,0,1/2) B1 (0,1/2,1/2) B2 (1/2,0,1/2)
  B3 (1/2,1/2,0).
* Sec. 1 (Boris pusher): half electric kick, magnetic rotation, half kick.
* Sec. 1 and Sec. 4.1 (Higuera-Cary pusher, cited there): the Boris
  splitting with the rotation taken at the Lorentz factor that the published
  method derives from the half-kicked momentum and the rotation vector, which
  keeps relativistic E x B drift exact.
* Sec. 1 and Sec. 4.1 (analytic pusher): the proper velocity is advanced by
  the exact solution for fields held constant over the step, with a map
  between proper time and lab time; the position update is second order.
  The paper defers the details; the oracle states the plain definition:
      d(gamma, u)/d tau = (q/m) Lambda(E, B) (gamma, u)
      Lambda = [[0, E1, E2, E3], [E1, 0, B3, -B2], [E2, -B3, 0, B1],
                [E3, B2, -B1, 0]]
  so (gamma, u)(tau) = expm((q/m) Lambda tau) (gamma, u)(0) and lab time
  t(tau) = e0 . [int_0^tau expm((q/m) Lambda s) ds] (gamma, u)(0).  The step
  solves t(tau*) = dt (t is increasing, dt/dtau = gamma >= 1) and returns
  u(tau*).  scipy's expm supplies both matrices through the block matrix
  expm([[F, I], [0, 0]] tau) = [[expm(F tau), int_0^tau expm(F s) ds], [0, I]].
* Sec. 4.1: position  x^{n+1} = x^n + dt u^{n+1/2}/gamma^{n+1/2}.
* Sec. 3.3: charge-conserving deposit "similar to Esirkepov" (cited, not
  restated by the paper); the oracle uses Esirkepov's first-order
  decomposition W = dS_x (S0_y S0_z + dS_y S0_z/2 + S0_y dS_z/2 + dS_y dS_z/3)
  and its cyclic forms, with J_1 = -q w (dx1/dt) * running sum of W_1 along
  x1.  It satisfies d_t rho + d_Yee . J = 0 exactly.

Readings
--------
* Shape order: linear for every run (the paper's LWFA run uses quadratic).
* Cell coordinate of a position: x/dx is evaluated as x * (1/dx) (one
  rounding of the reciprocal, one of the product), the cell index is
  floor(x * (1/dx) - offset) and the weight the remainder.  The index is an
  integer that floating point decides, so the reading fixes one evaluation
  order for it (and for the weights that go with it), here and in the HIP
  library; x/dx correctly rounded would move the index across a face for
  positions within an ulp of it and the weights by an ulp of the cell
  coordinate, which random fields of large amplitude amplify.  Periodic wrap
  of a position: x < 0 -> x + L (then 0 if that rounds to L); x >= L -> x - L.
* The momentum-conserving choice S_E = S_J (Sec. 3.1.2) holds: both are the
  linear shape at the component's own location.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

E_OFF = ((0.5, 0.0, 0.0), (0.0, 0.5, 0.0), (0.0, 0.0, 0.5))
B_OFF = ((0.0, 0.5, 0.5), (0.5, 0.0, 0.5), (0.5, 0.5, 0.0))


def _axis_weights(xd, dx, off, n):
    """Linear-shape nodes and weights along one direction."""
    u = xd * (1.0 / dx) - off
    i0 = np.floor(u)
    w1 = u - i0
    i0 = i0.astype(np.int64)
    return i0 % n, (i0 + 1) % n, 1.0 - w1, w1


def _axis_nodes_quadratic(xd, dx, off, n):
    """Quadratic B-spline shape along one direction (the Sec. 4.2 run's
    choice): the three nodes around the nearest one, i = round(u), with
    weights (1/2 - d)^2/2, 3/4 - d^2, (1/2 + d)^2/2 for d = u - i."""
    u = xd * (1.0 / dx) - off
    i = np.floor(u + 0.5)
    d = u - i
    i = i.astype(np.int64)
    return [(i - 1) % n, i % n, (i + 1) % n], [0.5 * (0.5 - d) ** 2, 0.75 - d * d, 0.5 * (0.5 + d) ** 2]


def gather_component(f, x, dx, off, ndim, order=1):
    """App. A: sum over the component's own grid points of f S(X - x);
    ``order`` 1 is the linear shape, 2 the quadratic B-spline."""
    if order == 2:
        return _gather_quadratic(f, x, dx, off, ndim)
    n3, n2, n1 = f.shape
    a0, a1, wa0, wa1 = _axis_weights(x[0], dx[0], off[0], n1)
    b0, b1, wb0, wb1 = _axis_weights(x[1], dx[1], off[1], n2)
    if ndim == 2:
        g = f[0]
        return (wb0 * (wa0 * g[b0, a0] + wa1 * g[b0, a1])
                + wb1 * (wa0 * g[b1, a0] + wa1 * g[b1, a1]))
    c0, c1, wc0, wc1 = _axis_weights(x[2], dx[2], off[2], n3)
    return (wc0 * (wb0 * (wa0 * f[c0, b0, a0] + wa1 * f[c0, b0, a1])
                   + wb1 * (wa0 * f[c0, b1, a0] + wa1 * f[c0, b1, a1]))
            + wc1 * (wb0 * (wa0 * f[c1, b0, a0] + wa1 * f[c1, b0, a1])
                     + wb1 * (wa0 * f[c1, b1, a0] + wa1 * f[c1, b1, a1])))


def _gather_quadratic(f, x, dx, off, ndim):
    n3, n2, n1 = f.shape
    ia, wa = _axis_nodes_quadratic(x[0], dx[0], off[0], n1)
    ib, wb = _axis_nodes_quadratic(x[1], dx[1], off[1], n2)
    out = np.zeros(x.shape[1])
    if ndim == 2:
        for b in range(3):
            for a in range(3):
                out += wb[b] * wa[a] * f[0][ib[b], ia[a]]
        return out
    ic, wc = _axis_nodes_quadratic(x[2], dx[2], off[2], n3)
    for c in range(3):
        for b in range(3):
            for a in range(3):
                out += wc[c] * wb[b] * wa[a] * f[ic[c], ib[b], ia[a]]
    return out


def gather(E, B, x, dx, ndim=3, order=1):
    """Fields at the particles: (E_p, B_p), each (3, np)."""
    Ep = np.stack([gather_component(E[c], x, dx, E_OFF[c], ndim, order) for c in range(3)])
    Bp = np.stack([gather_component(B[c], x, dx, B_OFF[c], ndim, order) for c in range(3)])
    return Ep, Bp


# ----------------------------------------------------------------------------
# Pushers (u at t^{n-1/2} -> t^{n+1/2}, fields at t^n)
# ----------------------------------------------------------------------------


def boris(u, Ep, Bp, qm, dt):
    """Sec. 1: Boris push, half E kick, rotation, half E kick."""
    eps = qm * dt / 2
    um = u + eps * Ep
    g = np.sqrt(1.0 + np.sum(um * um, axis=0))
    t = eps * Bp / g
    s = 2 * t / (1.0 + np.sum(t * t, axis=0))
    up = um + np.cross(um, t, axis=0)
    upl = um + np.cross(up, s, axis=0)
    return upl + eps * Ep


def higuera_cary(u, Ep, Bp, qm, dt):
    """Sec. 1 / Sec. 4.1: the Higuera-Cary push (the cited published
    method).  With h = q dt/(2m): u- = u + h E; tau = h B;
    sigma = gamma(u-)^2 - tau^2; gamma_r^2 = (sigma + sqrt(sigma^2 +
    4 (tau^2 + (u- . tau)^2)))/2; t = tau/gamma_r; the Boris-type rotation
    u+ = (u- + (u- . t) t + u- x t)/(1 + t^2); then u+ + h E + u+ x t."""
    eps = qm * dt / 2
    um = u + eps * Ep
    tau = eps * Bp
    tau2 = np.sum(tau * tau, axis=0)
    ust = np.sum(um * tau, axis=0)
    sigma = 1.0 + np.sum(um * um, axis=0) - tau2
    gr = np.sqrt((sigma + np.sqrt(sigma * sigma + 4 * (tau2 + ust * ust))) / 2)
    t = tau / gr
    s = 1.0 / (1.0 + np.sum(t * t, axis=0))
    up = s * (um + np.sum(um * t, axis=0) * t + np.cross(um, t, axis=0))
    return up + eps * Ep + np.cross(up, t, axis=0)


def field_tensor(Ep, Bp):
    """The 4x4 matrix Lambda(E, B), batched: shape (np, 4, 4)."""
    npart = Ep.shape[1]
    L = np.zeros((npart, 4, 4))
    E1, E2, E3 = Ep
    B1, B2, B3 = Bp
    L[:, 0, 1], L[:, 0, 2], L[:, 0, 3] = E1, E2, E3
    L[:, 1, 0], L[:, 2, 0], L[:, 3, 0] = E1, E2, E3
    L[:, 1, 2], L[:, 1, 3] = B3, -B2
    L[:, 2, 1], L[:, 2, 3] = -B3, B1
    L[:, 3, 1], L[:, 3, 2] = B2, -B1
    return L


def _exp_and_integral(F, tau):
    """expm(F tau) and int_0^tau expm(F s) ds via the 8x8 block exponential."""
    npart = F.shape[0]
    aug = np.zeros((npart, 8, 8))
    aug[:, :4, :4] = F * tau[:, None, None]
    aug[:, :4, 4:] = np.eye(4)[None] * tau[:, None, None]
    ex = scipy.linalg.expm(aug)
    return ex[:, :4, :4], ex[:, :4, 4:]


def analytic(u, Ep, Bp, qm, dt, max_iter=20000):
    """Exact push for E, B constant over the step (plain definition, see the
    module docstring): proper-time exponential plus a safeguarded Newton
    solve of t(tau) = dt between 0 and dt.  A non-finite t(tau) (overflow of
    the exponential far above the root) counts as an overshoot; the solve
    raises if some root is not found."""
    npart = u.shape[1]
    F = qm * field_tensor(Ep, Bp)
    g0 = np.sqrt(1.0 + np.sum(u * u, axis=0))
    U0 = np.concatenate([g0[None], u], axis=0).T  # (np, 4)
    # t(tau) is increasing with |t(tau)| >= |tau|: the root lies between 0
    # and dt (dt < 0 runs the map backwards in time)
    lo = np.full(npart, min(0.0, dt))
    hi = np.full(npart, max(0.0, dt))
    tau = dt / g0
    done = np.zeros(npart, dtype=bool)
    for _ in range(max_iter):
        ex, it = _exp_and_integral(F, tau)
        tval = np.einsum("pj,pj->p", it[:, 0, :], U0)
        gam = np.einsum("pj,pj->p", ex[:, 0, :], U0)
        f = tval - dt
        finite = np.isfinite(f) & np.isfinite(gam)
        hit = finite & (np.abs(f) <= 1e-16 * abs(dt))      # root found: keep tau
        # a non-finite t(tau) lies beyond the root, on the far side from 0
        over = np.where(finite, f > 0, dt > 0)
        hi = np.where(over, tau, hi)
        lo = np.where(over, lo, tau)
        with np.errstate(invalid="ignore"):
            newt = tau - f / gam
        bad = ~finite | ~((newt > lo) & (newt < hi))
        nxt = np.where(bad, 0.5 * (lo + hi), newt)
        small = np.abs(nxt - tau) <= 1e-15 * np.abs(tau)
        tau = np.where(done | hit, tau, nxt)
        done |= hit | small
        if done.all():
            break
    if not done.all():
        raise RuntimeError("exact pusher: t(tau) = dt not solved")
    ex, _ = _exp_and_integral(F, tau)
    U = np.einsum("pij,pj->pi", ex, U0)
    return U[:, 1:].T.copy()


def advance_position(x, u, dt, L, ndim=3):
    """Sec. 4.1: x^{n+1} = x^n + dt u/gamma, then periodic wrap.
    Returns (x_new_wrapped, displacement)."""
    g = np.sqrt(1.0 + np.sum(u * u, axis=0))
    disp = dt * u[:ndim] / g
    xn = x[:ndim] + disp
    out = np.empty_like(xn)
    for d in range(ndim):
        v = xn[d].copy()
        neg = v < 0
        v[neg] = v[neg] + L[d]
        v[neg & (v >= L[d])] = 0.0
        big = (~neg) & (v >= L[d])
        v[big] = v[big] - L[d]
        out[d] = v
    return out, disp


def min_image(x_new, x_old, L):
    """Displacement x_new - x_old undoing one periodic wrap."""
    d = x_new - x_old
    Lb = np.asarray(L)[:, None]
    d = np.where(d > Lb / 2, d - Lb, d)
    d = np.where(d < -Lb / 2, d + Lb, d)
    return d


# ----------------------------------------------------------------------------
# Charge-conserving deposit (Sec. 3.3, Esirkepov first order)
# ----------------------------------------------------------------------------


def _shapes_quadratic(x0, x1, dx):
    """Local 4-node quadratic shapes before/after a move of less than one
    cell (the nearest nodes differ by at most one)."""
    X0 = x0 * (1.0 / dx)
    X1 = x1 * (1.0 / dx)
    i0 = np.floor(X0 + 0.5)
    i1 = np.floor(X1 + 0.5)
    d0 = X0 - i0
    d1 = X1 - i1
    base = np.minimum(i0, i1) - 1
    a0 = (i0 - 1 - base).astype(np.int64)
    a1 = (i1 - 1 - base).astype(np.int64)
    npart = x0.shape[0]
    S0 = np.zeros((npart, 4))
    S1 = np.zeros((npart, 4))
    r = np.arange(npart)
    for k, (w0, w1) in enumerate(zip((0.5 * (0.5 - d0) ** 2, 0.75 - d0 * d0, 0.5 * (0.5 + d0) ** 2),
                                     (0.5 * (0.5 - d1) ** 2, 0.75 - d1 * d1, 0.5 * (0.5 + d1) ** 2))):
        S0[r, a0 + k] = w0
        S1[r, a1 + k] = w1
    return base.astype(np.int64), S0, S1


def _shapes(x0, x1, dx, order=1):
    """Local 3-node linear shapes before/after a move of less than one cell
    (``order`` 2: the 4-node quadratic ones)."""
    if order == 2:
        return _shapes_quadratic(x0, x1, dx)
    X0 = x0 * (1.0 / dx)
    X1 = x1 * (1.0 / dx)
    i0 = np.floor(X0)
    i1 = np.floor(X1)
    f0 = X0 - i0
    f1 = X1 - i1
    base = np.minimum(i0, i1)
    a0 = (i0 - base).astype(np.int64)
    a1 = (i1 - base).astype(np.int64)
    npart = x0.shape[0]
    S0 = np.zeros((npart, 3))
    S1 = np.zeros((npart, 3))
    r = np.arange(npart)
    S0[r, a0] = 1.0 - f0
    S0[r, a0 + 1] = f0
    S1[r, a1] = 1.0 - f1
    S1[r, a1 + 1] = f1
    return base.astype(np.int64), S0, S1


def deposit(x_old, x_new, q, w, dx, dt, shape, ndim=3, u=None, order=1):
    """Current J^{n+1/2} (3 arrays, E staggering) of particles moving
    x_old -> x_new (wrapped positions; the move is unwrapped by minimum
    image).  In 2D the out-of-plane current is q w v3 times the time-averaged
    in-plane shape (needs ``u``).  ``order`` 2: quadratic shapes (the same
    Esirkepov decomposition on 4-node stencils)."""
    n3, n2, n1 = shape
    L = [n1 * dx[0], n2 * dx[1], n3 * dx[2]][:ndim]
    disp = min_image(x_new[:ndim], x_old[:ndim], L)
    J = [np.zeros(shape) for _ in range(3)]
    bases, S0s, S1s = [], [], []
    for d in range(ndim):
        b, s0, s1 = _shapes(x_old[d], x_old[d] + disp[d], dx[d], order)
        bases.append(b)
        S0s.append(s0)
        S1s.append(s1)
    dS = [s1 - s0 for s0, s1 in zip(S0s, S1s)]
    qw = q * w
    ns = (n1, n2, n3)
    if ndim == 3:
        S0x, S0y, S0z = S0s
        dSx, dSy, dSz = dS
        ex = np.einsum
        W1 = dSx[:, :, None, None] * (ex("pb,pc->pbc", S0y, S0z) + 0.5 * ex("pb,pc->pbc", dSy, S0z)
                                       + 0.5 * ex("pb,pc->pbc", S0y, dSz)
                                       + ex("pb,pc->pbc", dSy, dSz) / 3.0)[:, None, :, :]
        W2 = dSy[:, None, :, None] * (ex("pa,pc->pac", S0x, S0z) + 0.5 * ex("pa,pc->pac", dSx, S0z)
                                       + 0.5 * ex("pa,pc->pac", S0x, dSz)
                                       + ex("pa,pc->pac", dSx, dSz) / 3.0)[:, :, None, :]
        W3 = dSz[:, None, None, :] * (ex("pa,pb->pab", S0x, S0y) + 0.5 * ex("pa,pb->pab", dSx, S0y)
                                       + 0.5 * ex("pa,pb->pab", S0x, dSy)
                                       + ex("pa,pb->pab", dSx, dSy) / 3.0)[:, :, :, None]
        C1 = -qw * dx[0] / dt * np.cumsum(W1, axis=1)
        C2 = -qw * dx[1] / dt * np.cumsum(W2, axis=2)
        C3 = -qw * dx[2] / dt * np.cumsum(W3, axis=3)
        K = S0x.shape[1]
        for comp, Cc in enumerate((C1, C2, C3)):
            for a in range(K):
                for b in range(K):
                    for c in range(K):
                        ia = (bases[0] + a) % ns[0]
                        ib = (bases[1] + b) % ns[1]
                        ic = (bases[2] + c) % ns[2]
                        np.add.at(J[comp], (ic, ib, ia), Cc[:, a, b, c])
        return J
    # 2D3V: x3 is ignorable
    S0x, S0y = S0s
    dSx, dSy = dS
    W1 = dSx[:, :, None] * (S0y + 0.5 * dSy)[:, None, :]
    W2 = dSy[:, None, :] * (S0x + 0.5 * dSx)[:, :, None]
    W3 = (S0x[:, :, None] * S0y[:, None, :] + 0.5 * dSx[:, :, None] * S0y[:, None, :]
          + 0.5 * S0x[:, :, None] * dSy[:, None, :] + dSx[:, :, None] * dSy[:, None, :] / 3.0)
    g = np.sqrt(1.0 + np.sum(u * u, axis=0))
    v3 = u[2] / g
    C1 = -qw * dx[0] / dt * np.cumsum(W1, axis=1)
    C2 = -qw * dx[1] / dt * np.cumsum(W2, axis=2)
    C3 = qw * v3[:, None, None] * W3
    K = S0x.shape[1]
    for comp, Cc in enumerate((C1, C2, C3)):
        for a in range(K):
            for b in range(K):
                ia = (bases[0] + a) % ns[0]
                ib = (bases[1] + b) % ns[1]
                np.add.at(J[comp], (np.zeros_like(ia), ib, ia), Cc[:, a, b])
    return J


def charge_density(x, q, w, dx, shape, ndim=3, order=1):
    """rho on the nodes: q w times the linear shape (Sec. 3.3 continuity);
    ``order`` 2: the quadratic B-spline."""
    n3, n2, n1 = shape
    rho = np.zeros(shape)
    ns = (n1, n2, n3)
    if order == 2:
        nodes = [_axis_nodes_quadratic(x[d], dx[d], 0.0, ns[d]) for d in range(ndim)]
        if ndim == 2:
            for a in range(3):
                for b in range(3):
                    np.add.at(rho, (np.zeros_like(nodes[0][0][a]), nodes[1][0][b], nodes[0][0][a]),
                              q * w * nodes[0][1][a] * nodes[1][1][b])
            return rho
        for a in range(3):
            for b in range(3):
                for c in range(3):
                    np.add.at(rho, (nodes[2][0][c], nodes[1][0][b], nodes[0][0][a]),
                              q * w * nodes[0][1][a] * nodes[1][1][b] * nodes[2][1][c])
        return rho
    idx, wts = [], []
    for d in range(ndim):
        i0, i1, w0, w1 = _axis_weights(x[d], dx[d], 0.0, ns[d])
        idx.append((i0, i1))
        wts.append((w0, w1))
    if ndim == 2:
        for a in range(2):
            for b in range(2):
                np.add.at(rho, (np.zeros_like(idx[0][a]), idx[1][b], idx[0][a]),
                          q * w * wts[0][a] * wts[1][b])
        return rho
    for a in range(2):
        for b in range(2):
            for c in range(2):
                np.add.at(rho, (idx[2][c], idx[1][b], idx[0][a]),
                          q * w * wts[0][a] * wts[1][b] * wts[2][c])
    return rho
