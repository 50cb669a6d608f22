"""One PIC step in the paper's order (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Per step (Eq. pusher time levels; Sec. 3.3 for the source):
  1. gather E^n, B^n at x^n (App. A) and push u^{n-1/2} -> u^{n+1/2}
  2. advance x^n -> x^{n+1} (second order, Sec. 4.1)
  3. deposit J^{n+1/2} from (x^n, x^{n+1}) (charge conserving, Sec. 3.3),
     then the x1 current correction of Eq. (correction) (``current``), which
     is the identity when [k]_B1 equals the Yee symbol (the proposed solver
     at dt = dx1/2) and is skipped there.
  4. field sweep (E^n, B^n) -> (E^{n+1}, B^{n+1}) with J^{n+1/2}.
  5. optionally, the absorbing layers at the two x1 ends of the window
     (``absorb``; off by default).
"""
from __future__ import annotations

import numpy as np

from . import absorb as absorb_mod, current, fdtd, particles


def _ampere_is_yee(CB):
    """[k]_B1 is the Yee symbol when C^B = e1; coefficients left over at the
    1e-20 level by the fit's rounding are far below FP64 resolution."""
    CB = np.asarray(CB, dtype=np.float64)
    return abs(CB[0] - 1.0) <= 1e-20 and bool(np.all(np.abs(CB[1:]) <= 1e-20))


def step(E, B, species, CE, CB, dx, dt, *, pusher="boris", deposit=False, ndim=3, order=1, absorb=None):
    """Advance fields and every species by one step; species entries are
    dicts with keys x, u, q, m, w (x and u are replaced).  ``order``: shape
    function of gather and deposit, 1 linear, 2 quadratic.  ``absorb``:
    (W, sigma) or (W, sigma, origin) of the x1 absorbing layers, applied
    after the field sweep."""
    shape = E[0].shape
    n3, n2, n1 = shape
    L = [n1 * dx[0], n2 * dx[1], n3 * dx[2]][:ndim]
    J = [np.zeros(shape) for _ in range(3)] if deposit else None
    for sp in species:
        Ep, Bp = particles.gather(E, B, sp["x"], dx, ndim, order)
        qm = sp["q"] / sp["m"]
        if pusher == "boris":
            u = particles.boris(sp["u"], Ep, Bp, qm, dt)
        elif pusher == "analytic":
            u = particles.analytic(sp["u"], Ep, Bp, qm, dt)
        elif pusher == "hc":
            u = particles.higuera_cary(sp["u"], Ep, Bp, qm, dt)
        else:
            raise ValueError(pusher)
        x_old = sp["x"]
        x_new, _ = particles.advance_position(x_old, u, dt, L, ndim)
        if ndim == 2 and x_old.shape[0] == 3:
            x_new = np.concatenate([x_new, x_old[2:3]], axis=0)
        if deposit:
            Js = particles.deposit(x_old, x_new, sp["q"], sp["w"], dx, dt, shape, ndim, u=u, order=order)
            J = [a + b for a, b in zip(J, Js)]
        sp["x"], sp["u"] = x_new, u
    if deposit and not _ampere_is_yee(CB):
        J[0] = current.correct_x1(J[0], CB, dx[0])
    E, B = fdtd.sweep(E, B, J, CE, CB, dx, dt)
    if absorb is not None:
        E, B = absorb_mod.damp(E, B, *absorb)
    return E, B


def run(E, B, species, CE, CB, dx, dt, nsteps, **kw):
    """``nsteps`` calls of ``step``."""
    for _ in range(nsteps):
        E, B = step(E, B, species, CE, CB, dx, dt, **kw)
    return E, B
