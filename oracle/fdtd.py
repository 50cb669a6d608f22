"""Leapfrog FDTD field step on the staggered Yee mesh (FP64, periodic).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Layout: every component is an array of shape (n3, n2, n1) (x1 fastest; axis 2
is x1, axis 1 is x2, axis 0 is x3).  Index (k, j, i) holds the component at
its own staggered location (App. A and the standard Yee mesh):
    E1 (i+1/2, j, k)   E2 (i, j+1/2, k)   E3 (i, j, k+1/2)
    B1 (i, j+1/2, k+1/2)  B2 (i+1/2, j, k+1/2)  B3 (i+1/2, j+1/2, k)
Boundaries are periodic in every direction.  A 2D run is n3 = 1 (every x3
difference then vanishes identically).

Passages followed
-----------------
* Eq. (maxwell): d_t B = -d_E x E,  d_t E = d_B x B - J.
* App. B: the x1 operators
      Faraday  d^E f_i = (1/dx1) sum_j C^E_j (f_{i+j}   - f_{i-j+1})
      Ampere   d^B f_i = (1/dx1) sum_j C^B_j (f_{i+j-1} - f_{i-j})
* Sec. 3.1.1: x2 (and x3) operators are the Yee ones for every solver.
* Eq. (pusher) and Sec. 2.2: fields are needed at integer time; E and B are
  both kept at t^n and B passes through two half steps,
      B^{n+1/2} = B^n - (dt/2) curl_E E^n
      E^{n+1}   = E^n + dt (curl_B B^{n+1/2} - J^{n+1/2})
      B^{n+1}   = B^{n+1/2} - (dt/2) curl_E E^{n+1}
  so that B^n equals the average (B^{n-1/2} + B^{n+1/2})/2 of Eq. (pusher).
* Sec. 3.3: Gauss's law with the Ampere operator, i [k]_B . E = -rho.
"""
from __future__ import annotations

import numpy as np

X1, X2, X3 = 2, 1, 0  # array axes of the three directions


def d1_faraday(f, C, dx1):
    """App. B: (1/dx1) sum_j C_j (f_{i+j} - f_{i-j+1}) along x1."""
    out = np.zeros_like(f)
    for j, c in enumerate(C, start=1):
        out = out + c * (np.roll(f, -j, axis=X1) - np.roll(f, j - 1, axis=X1))
    return out / dx1


def d1_ampere(f, C, dx1):
    """App. B: (1/dx1) sum_j C_j (f_{i+j-1} - f_{i-j}) along x1."""
    out = np.zeros_like(f)
    for j, c in enumerate(C, start=1):
        out = out + c * (np.roll(f, -(j - 1), axis=X1) - np.roll(f, j, axis=X1))
    return out / dx1


def d_fwd(f, axis, d):
    """Yee forward difference (f_{j+1} - f_j)/d (Faraday, x2 and x3)."""
    return (np.roll(f, -1, axis=axis) - f) / d


def d_bwd(f, axis, d):
    """Yee backward difference (f_j - f_{j-1})/d (Ampere, x2 and x3)."""
    return (f - np.roll(f, 1, axis=axis)) / d


def curl_E(E, CE, dx):
    """The curl used in Faraday's law, d_E x E (Eq. maxwell)."""
    E1, E2, E3 = E
    dx1, dx2, dx3 = dx
    return (d_fwd(E3, X2, dx2) - d_fwd(E2, X3, dx3),
            d_fwd(E1, X3, dx3) - d1_faraday(E3, CE, dx1),
            d1_faraday(E2, CE, dx1) - d_fwd(E1, X2, dx2))


def curl_B(B, CB, dx):
    """The curl used in Ampere's law, d_B x B (Eq. maxwell)."""
    B1, B2, B3 = B
    dx1, dx2, dx3 = dx
    return (d_bwd(B3, X2, dx2) - d_bwd(B2, X3, dx3),
            d_bwd(B1, X3, dx3) - d1_ampere(B3, CB, dx1),
            d1_ampere(B2, CB, dx1) - d_bwd(B1, X2, dx2))


def advance_B(E, B, CE, dx, h):
    """B <- B - h curl_E E  (Faraday over a time h; h = dt/2 is a half step)."""
    c = curl_E(E, CE, dx)
    return tuple(b - h * ci for b, ci in zip(B, c))


def advance_E(E, B, J, CB, dx, dt):
    """E <- E + dt (curl_B B - J)  (Ampere; J may be None for vacuum)."""
    c = curl_B(B, CB, dx)
    if J is None:
        return tuple(e + dt * ci for e, ci in zip(E, c))
    return tuple(e + dt * (ci - j) for e, ci, j in zip(E, c, J))


def sweep(E, B, J, CE, CB, dx, dt):
    """One full field step (E^n, B^n) -> (E^{n+1}, B^{n+1}):
    B half step, E full step, B half step (Eq. maxwell, Eq. pusher)."""
    Bh = advance_B(E, B, CE, dx, dt / 2)
    En = advance_E(E, Bh, J, CB, dx, dt)
    Bn = advance_B(En, Bh, CE, dx, dt / 2)
    return En, Bn


def div_faraday(B, CE, dx):
    """Divergence annihilating curl_E (x1 part with the C^E operator); it is
    constant in time under Faraday's law."""
    return (d1_faraday(B[0], CE, dx[0]) + d_fwd(B[1], X2, dx[1])
            + d_fwd(B[2], X3, dx[2]))


def div_ampere(E, CB, dx):
    """Sec. 3.3: the Gauss-law divergence i[k]_B . E (x1 part with C^B),
    evaluated on the nodes (i, j, k)."""
    return (d1_ampere(E[0], CB, dx[0]) + d_bwd(E[1], X2, dx[1])
            + d_bwd(E[2], X3, dx[2]))


def amplification_matrix(k, CE, CB, dx, dt, n=(64, 4, 4)):
    """The 6x6 complex matrix G of one sweep acting on the Fourier amplitudes
    of a single mode exp(i k . X) (X = grid index times dx), measured by
    stepping each unit amplitude through ``sweep`` on a periodic grid whose
    size ``n`` (n1, n2, n3) must contain the mode."""
    n1, n2, n3 = n
    i3, i2, i1 = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
    phase = np.exp(1j * (k[0] * i1 * dx[0] + k[1] * i2 * dx[1] + k[2] * i3 * dx[2]))
    G = np.zeros((6, 6), dtype=np.complex128)
    for c in range(6):
        comps = [np.zeros((n3, n2, n1), dtype=np.complex128) for _ in range(6)]
        comps[c] = phase.copy()
        En, Bn = sweep(tuple(comps[:3]), tuple(comps[3:]), None, CE, CB, dx, dt)
        for r, f in enumerate(En + Bn):
            G[r, c] = np.mean(f * np.conj(phase))
    return G
