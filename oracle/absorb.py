"""Absorbing layers at the two x1 ends of the window (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The moving-window runs of Sec. 4.1 and Sec. 4.2 follow the laser along x1 with
a window whose x2 boundaries are periodic; the paper names no boundary
condition for the two x1 ends.  On a mesh that is periodic along x1, light
leaving through one end would re-enter through the other.  The absorber taken
here is the graded damping layer of Cerjan, Kosloff, Kosloff and Reshef
(Geophysics 50, 1985), a published method for finite-difference wave
equations: in a strip of W cells at each end, every field value is multiplied
after each step by a factor that falls smoothly from 1 at the strip's inner
edge to its minimum at the outer edge,

    g(s) = exp(-sigma (d(s)/W)^2),   d(s) = depth of x1 position s (in
                                     cells, window coordinates) into the
                                     nearest strip, 0 outside both,

so that a wave entering the strip is attenuated gradually (a steep profile
would reflect it).  Each component is damped at its own staggered x1 location
(E1, B2, B3 at i + 1/2; E2, E3, B1 at i).  Readings: the profile exponent 2 is
Cerjan's Gaussian grading; the depth is measured in cells from the strip's
inner edge at s = W (back strip) and s = n1 - W (front strip); the current is
not damped (the layers act on the field solution only).
"""
from __future__ import annotations

import numpy as np

# staggering of each component along x1, in cells (E1, E2, E3, B1, B2, B3)
X1_OFF = (0.5, 0.0, 0.0, 0.0, 0.5, 0.5)


def depth(s, n1, W):
    """Depth (cells) of window position s into the nearest end strip."""
    s = np.asarray(s, dtype=np.float64)
    back = np.where(s < W, W - s, 0.0)
    front = np.where(s > n1 - W, s - (n1 - W), 0.0)
    return np.maximum(back, front)


def profile(n1, W, sigma, off):
    """Damping factor g at positions i + off, i = 0..n1-1 (window cells)."""
    if W <= 0:
        return np.ones(n1)
    d = depth(np.arange(n1) + off, n1, W)
    return np.exp(-sigma * (d / W) ** 2)


def damp(E, B, W, sigma, origin=0):
    """Fields after one application of the layers.  ``origin``: array column
    of window cell 0 when the x1 axis is a ring (moving window); window cell
    i lives in array column (origin + i) mod n1."""
    n1 = E[0].shape[-1]
    out = []
    for c, f in enumerate(list(E) + list(B)):
        g = np.roll(profile(n1, W, sigma, X1_OFF[c]), origin)
        out.append(f * g)
    return tuple(out[:3]), tuple(out[3:])


def field_energy(E, B, dx):
    """Sum over the mesh of (E^2 + B^2)/2 times the cell volume (used to
    measure what the layers absorb and reflect)."""
    vol = float(np.prod(dx))
    return 0.5 * vol * float(sum(np.sum(f * f) for f in list(E) + list(B)))
