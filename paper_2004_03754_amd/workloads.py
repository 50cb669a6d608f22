"""Seeded synthetic inputs shared by the tests, the oracle checks and the
benchmark.  Holds none of the solver's arithmetic: only grid constants, laser
vector potentials sampled onto the staggered mesh, and particle loads.

Grid (all workloads): dx1 = lambda0/32, dx2 = dx3 = lambda0/8, dt = dx1/2,
k0 = omega0 = 1 (normalised units of Sec. 2.1, lambda0 = 2 pi).

Laser: a plane wave along +x1 polarised along x2, given by its normalised
vector potential a(s) with the local phase s = t - x1 + x_head (s = 0 at the
pulse head).  At t = 0 both E and B are sampled at their own staggered
locations (E2 = B3 = -a'(s), times an optional transverse Gaussian profile).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

LAMBDA0 = 2.0 * np.pi
DX1 = LAMBDA0 / 32.0
DX2 = LAMBDA0 / 8.0
DX3 = LAMBDA0 / 8.0
DT = DX1 / 2.0


def rng(seed: int) -> np.random.Generator:
    """The one random source of every workload (PCG64, seeded)."""
    return np.random.Generator(np.random.PCG64(seed))


# ----------------------------------------------------------------------------
# laser vector potentials a(s) and their derivatives
# ----------------------------------------------------------------------------


@dataclass
class Sin2Pulse:
    """a(s) = a0 sin^2(pi s/Lp) sin(s) for 0 <= s <= Lp, else 0; optionally
    periodic with period ``period`` (a box length)."""
    a0: float
    Lp: float
    period: float | None = None

    def _s(self, s):
        s = np.asarray(s, dtype=np.float64)
        return np.mod(s, self.period) if self.period else s

    def a(self, s):
        s = self._s(s)
        inside = (s >= 0) & (s <= self.Lp)
        return np.where(inside, self.a0 * np.sin(np.pi * s / self.Lp) ** 2 * np.sin(s), 0.0)

    def da(self, s):
        s = self._s(s)
        inside = (s >= 0) & (s <= self.Lp)
        k = np.pi / self.Lp
        v = self.a0 * (k * np.sin(2 * k * s) * np.sin(s) + np.sin(k * s) ** 2 * np.cos(s))
        return np.where(inside, v, 0.0)


@dataclass
class PlaneWave:
    """a(s) = a0 sin(s): monochromatic, exactly periodic over whole lambda0."""
    a0: float

    def a(self, s):
        return self.a0 * np.sin(np.asarray(s, dtype=np.float64))

    def da(self, s):
        return self.a0 * np.cos(np.asarray(s, dtype=np.float64))


@dataclass
class FlatTopPulse:
    """Plane-wave pulse with a flat top (the single-particle runs of Sec. 4.1):
    a(s) = a0 env(s) sin(s - R), env = 1 on the flat top R <= s <= R + Lf,
    exp(-((R - s)/sigma)^4) before it and exp(-((s - R - Lf)/sigma)^4) after
    it, and a = 0 outside 0 <= s <= 2R + Lf.  Inside the flat top the vector
    potential vanishes at s = R + m pi, where E2 = -a' is extremal."""
    a0: float
    Lf: float = 100.0
    sigma: float = 10.0
    R: float = 30.0

    def _env(self, s):
        lo = (self.R - s) / self.sigma
        hi = (s - self.R - self.Lf) / self.sigma
        env = np.where(s < self.R, np.exp(-lo ** 4), np.where(s > self.R + self.Lf, np.exp(-hi ** 4), 1.0))
        denv = np.where(s < self.R, 4 * lo ** 3 / self.sigma * np.exp(-lo ** 4),
                        np.where(s > self.R + self.Lf, -4 * hi ** 3 / self.sigma * np.exp(-hi ** 4), 0.0))
        inside = (s >= 0) & (s <= 2 * self.R + self.Lf)
        return np.where(inside, env, 0.0), np.where(inside, denv, 0.0)

    def a(self, s):
        s = np.asarray(s, dtype=np.float64)
        env, _ = self._env(s)
        return self.a0 * env * np.sin(s - self.R)

    def da(self, s):
        s = np.asarray(s, dtype=np.float64)
        env, denv = self._env(s)
        return self.a0 * (denv * np.sin(s - self.R) + env * np.cos(s - self.R))


def laser_profiles(n, dx, pulse, x_head=0.0, w0=None, centre=None):
    """Factors of the t = 0 laser fields: E2 = e2[i] prof[k, j] and
    B3 = b3[i] prof[k, j], with e2 = b3 = -a'(x_head - x1) sampled at the E2
    (x1 = i dx1) and B3 (x1 = (i+1/2) dx1) locations and prof the transverse
    Gaussian exp(-r_perp^2/w0^2) at (j+1/2, k) (ones without ``w0``)."""
    n1, n2, n3 = n
    i = np.arange(n1, dtype=np.float64)
    e2 = -pulse.da(x_head - i * dx[0])
    b3 = -pulse.da(x_head - (i + 0.5) * dx[0])
    if w0 is None:
        prof = np.ones((n3, n2))
    else:
        c2, c3 = centre if centre is not None else (n2 * dx[1] / 2, n3 * dx[2] / 2)
        y = (np.arange(n2) + 0.5) * dx[1] - c2
        z = np.arange(n3) * dx[2] - c3
        prof = np.exp(-(z[:, None] ** 2 + y[None, :] ** 2) / w0 ** 2)
    return e2, b3, prof


def laser_longitudinal(n, dx, pulse, x_head=0.0, w0=None, centre=None):
    """Factors of the first-order longitudinal fields of the Gaussian beam,
    E1 = e1[i] p1[k, j] and B1 = b1[i] q1[k, j], or None without ``w0``.

    With E2 = f(x1) g and B3 = f(x1) g, f = -a'(x_head - x1) and g =
    exp(-r_perp^2/w0^2), the longitudinal components that make both fields
    divergence-free are E1 = -a(x_head - x1) dg/dx2 and B1 = -a(x_head - x1)
    dg/dx3 (d/dx1 of a(x_head - x1) is f), i.e. a(x_head - x1) (2 x2/w0^2) g
    and a(x_head - x1) (2 x3/w0^2) g: the paraxial beam's first-order terms.
    Each is sampled at its own staggered location: E1 at ((i+1/2), j, k),
    B1 at (i, j+1/2, k+1/2) cells."""
    if w0 is None:
        return None
    n1, n2, n3 = n
    i = np.arange(n1, dtype=np.float64)
    e1 = pulse.a(x_head - (i + 0.5) * dx[0])
    b1 = pulse.a(x_head - i * dx[0])
    c2, c3 = centre if centre is not None else (n2 * dx[1] / 2, n3 * dx[2] / 2)
    yj = np.arange(n2) * dx[1] - c2
    zk = np.arange(n3) * dx[2] - c3
    yh = yj + 0.5 * dx[1]
    zh = zk + 0.5 * dx[2]
    p1 = (2 * yj[None, :] / w0 ** 2) * np.exp(-(zk[:, None] ** 2 + yj[None, :] ** 2) / w0 ** 2)
    q1 = (2 * zh[:, None] / w0 ** 2) * np.exp(-(zh[:, None] ** 2 + yh[None, :] ** 2) / w0 ** 2)
    return e1, p1, b1, q1


def laser_fields(n, dx, pulse, x_head=0.0, w0=None, centre=None, dtype=np.float64):
    """(E, B) at t = 0 on the (n3, n2, n1) mesh: E2 = B3 = -a'(x_head - x1),
    times exp(-r_perp^2/w0^2) with the longitudinal E1, B1 of
    ``laser_longitudinal`` if ``w0``; every other component zero."""
    n1, n2, n3 = n
    e2, b3, prof = laser_profiles(n, dx, pulse, x_head, w0, centre)
    E = [np.zeros((n3, n2, n1), dtype=dtype) for _ in range(3)]
    B = [np.zeros((n3, n2, n1), dtype=dtype) for _ in range(3)]
    E[1][...] = (prof[:, :, None] * e2[None, None, :]).astype(dtype)
    B[2][...] = (prof[:, :, None] * b3[None, None, :]).astype(dtype)
    lon = laser_longitudinal(n, dx, pulse, x_head, w0, centre)
    if lon is not None:
        e1, p1, b1, q1 = lon
        E[0][...] = (p1[:, :, None] * e1[None, None, :]).astype(dtype)
        B[0][...] = (q1[:, :, None] * b1[None, None, :]).astype(dtype)
    return E, B


def random_fields(n, seed, scale=1.0, dtype=np.float64):
    """Six independent uniform(-scale, scale) arrays (parity inputs)."""
    g = rng(seed)
    n1, n2, n3 = n
    comps = [(scale * (2 * g.random((n3, n2, n1)) - 1)).astype(dtype) for _ in range(6)]
    return comps[:3], comps[3:]


def uniform_particles(npart, lo, hi, seed, u_th=0.0):
    """x uniform in the box [lo, hi) (per direction), u ~ N(0, u_th^2) per
    component (zeros for u_th = 0)."""
    g = rng(seed)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    x = lo[:, None] + (hi - lo)[:, None] * g.random((3, npart))
    u = u_th * g.standard_normal((3, npart)) if u_th > 0 else np.zeros((3, npart))
    return x, u


def lattice_particles(n, dx, ppc_per_dim, seed, u_th):
    """Plasma load: ppc_per_dim^3 particles per cell on a regular sub-lattice
    (cell-centred offsets), thermal u ~ N(0, u_th^2)."""
    n1, n2, n3 = n
    p = ppc_per_dim
    off = (np.arange(p) + 0.5) / p
    cells = [np.arange(m, dtype=np.float64) for m in (n1, n2, n3)]
    coords = []
    for d in range(3):
        c = (cells[d][:, None] + off[None, :]).ravel() * dx[d]
        coords.append(c)
    z, y, x = np.meshgrid(coords[2], coords[1], coords[0], indexing="ij")
    X = np.stack([x.ravel(), y.ravel(), z.ravel()])
    g = rng(seed)
    U = u_th * g.standard_normal(X.shape)
    return X, U


def device_lattice_particles(n, dx, ppc_per_dim, u_th, seed, torch):
    """The plasma load of ``lattice_particles`` built on cuda:0 (no host copy
    of a full-size load): ppc_per_dim^3 particles per cell on the cell-centred
    sub-lattice, x1 fastest, then x2, then x3; momenta N(0, u_th^2) per
    component from a seeded device generator.  ``torch`` is passed in so that
    this module does not import it."""
    n1, n2, n3 = n
    dev = "cuda:0"
    off = (torch.arange(ppc_per_dim, device=dev, dtype=torch.float64) + 0.5) / ppc_per_dim
    cx = ((torch.arange(n1, device=dev, dtype=torch.float64)[:, None] + off[None, :]).reshape(-1)) * dx[0]
    cy = ((torch.arange(n2, device=dev, dtype=torch.float64)[:, None] + off[None, :]).reshape(-1)) * dx[1]
    cz = ((torch.arange(n3, device=dev, dtype=torch.float64)[:, None] + off[None, :]).reshape(-1)) * dx[2]
    npart = cx.numel() * cy.numel() * cz.numel()
    x = torch.empty((3, npart), device=dev, dtype=torch.float64)
    x[0].view(cz.numel(), cy.numel(), cx.numel()).copy_(cx[None, None, :].expand(cz.numel(), cy.numel(), -1))
    x[1].view(cz.numel(), cy.numel(), cx.numel()).copy_(cy[None, :, None].expand(cz.numel(), -1, cx.numel()))
    x[2].view(cz.numel(), cy.numel(), cx.numel()).copy_(cz[:, None, None].expand(-1, cy.numel(), cx.numel()))
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    u = u_th * torch.randn((3, npart), generator=g, device=dev, dtype=torch.float64)
    return x, u


def small_moves(x, dx, L, seed, frac=0.9):
    """New positions within ``frac`` cells of ``x`` (periodic), for deposit
    checks."""
    g = rng(seed)
    d = (2 * g.random(x.shape) - 1) * frac * np.asarray(dx)[:, None]
    return np.mod(x + d, np.asarray(L)[:, None]), d
