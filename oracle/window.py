"""Moving window along x1 (Sec. 4.1, the single-particle runs) (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The single-particle runs of Sec. 4.1 follow the laser with a window that moves
along +x1 (x2 stays periodic).  Reading taken here: the window advances by
whole cells.  Moving it by s cells means
  * every field value at window cell i takes the value that was at window cell
    i + s (for i < n1 - s), and the s cells entering at the front hold vacuum
    (all fields zero);
  * every particle position x1 drops by s dx1, and particles that fall behind
    the window's back edge (x1 < 0 afterwards) leave the run; the others keep
    their order.
A window that moves at c advances one cell each time t passes a multiple of
dx1 (``cells_due``).
"""
from __future__ import annotations

import numpy as np


def shift_field(f, s):
    """One field array [n3][n2][n1] seen from a window moved by s cells."""
    f = np.asarray(f)
    n1 = f.shape[-1]
    if not 0 <= s < n1:
        raise ValueError("shift must satisfy 0 <= s < n1")
    out = np.zeros_like(f)
    out[..., : n1 - s] = f[..., s:]
    return out


def move(E, B, species, s, dx1, J=None):
    """Move the window by s cells: returns (E, B) (and J if given) in the new
    window; each species dict has its x, u (and optional id) replaced by the
    particles still inside, in their original order."""
    E = [shift_field(e, s) for e in E]
    B = [shift_field(b, s) for b in B]
    for sp in species:
        x = np.array(sp["x"], dtype=np.float64, copy=True)
        x[0] = x[0] - s * dx1
        keep = x[0] >= 0.0
        sp["x"] = x[:, keep]
        sp["u"] = np.asarray(sp["u"])[:, keep]
        if sp.get("id") is not None:
            sp["id"] = np.asarray(sp["id"])[keep]
    if J is not None:
        return E, B, [shift_field(j, s) for j in J]
    return E, B


def cells_due(nsteps, dt, dx1):
    """Cells a window moving at c has advanced after ``nsteps`` steps:
    floor(nsteps dt / dx1), with a tolerance of 1e-9 for a ratio that is an
    integer up to rounding."""
    return int(np.floor(nsteps * dt / dx1 + 1e-9))
