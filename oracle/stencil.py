"""Stencil coefficients and k-space analysis of the dual-operator FDTD solver.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper passages followed
-----------------------
* Sec. 2.1, Eq. (maxwell_fourier) and Eq. (dispersion): vacuum numerical
  dispersion  [omega]_t^2 = [k]_B . [k]_E,  [omega]_t = sin(omega dt/2)/(dt/2).
* Eq. (v_phi): phase velocity of a wave along x1.
* Sec. 2.1: the staggered x1 symbol  [k] = sum_j C_j sin((2j-1) k dx/2)/(dx/2).
* Eq. (f2_q) and the definition of F in the caption of Fig. 2: the
  cancellation factor  F = sqrt([k]_E1/[k]_B1) cos(omega dt/2).
* Eq. (new_op): the targets [k]_E1 = [k]_{1,t}/cos(k1 dt/2),
  [k]_B1 = [k]_{1,t} cos(k1 dt/2), [k]_{1,t} = sin(k1 dt/2)/(dt/2).
* Sec. 3.1.1, Eq. (vphi_ob) and the definition of kappa: obliquely
  travelling waves, x2 operators are Yee for every solver.
* Sec. 3.2: exact and sufficient CFL conditions.
* App. B: constrained weighted least squares for the customized coefficients;
  objective, constraint matrix M_ij = (2j-1)^(2i-1)/(2i-1)!, the KKT matrix
  equation, the integrals A_ij and b_i, and the super-Gaussian weight.

Readings taken where the paper is silent
----------------------------------------
* Weight: the printed form w = exp[-ln2 (2 kappa / w_k1)^n], n = 10,
  w_k1 = 0.4 (upper end of the quoted 0.3-0.4 range).  ``width_factor`` is the
  "2" in front of kappa and may be set to 1 to study the other reading.
* Quadrature: composite Gauss-Legendre over [0, 1/2]; the KKT system is solved
  in mpmath at 60 significant digits, because the system is extremely
  ill-conditioned (condition number ~1e19 at M = 16).
* Normalisation: k1 and the operators are divided by k_g1 = 2 pi/dx1, so the
  j-th basis function is sin((2j-1) pi kappa)/pi and, with r = dt/dx1, the
  targets are T_E = tan(pi kappa r)/(pi r) and T_B = sin(2 pi kappa r)/(2 pi r).
"""
from __future__ import annotations

from fractions import Fraction
from math import factorial

import mpmath as mp
import numpy as np

# ----------------------------------------------------------------------------
# App. B: constraint matrix and textbook (M = p/2) staggered coefficients
# ----------------------------------------------------------------------------


def constraint_matrix(p: int, M: int):
    """App. B: M_ij = (2j-1)^(2i-1) / (2i-1)!,  i = 1..p/2, j = 1..M (exact)."""
    if p % 2 or p < 2:
        raise ValueError("order p must be even and >= 2")
    return [[Fraction((2 * j - 1) ** (2 * i - 1), factorial(2 * i - 1))
             for j in range(1, M + 1)] for i in range(1, p // 2 + 1)]


def _solve_fraction(a, b):
    """Gaussian elimination over the rationals (square, non-singular)."""
    n = len(a)
    m = [list(row) + [rhs] for row, rhs in zip(a, b)]
    for c in range(n):
        piv = next(r for r in range(c, n) if m[r][c] != 0)
        m[c], m[piv] = m[piv], m[c]
        for r in range(n):
            if r != c and m[r][c] != 0:
                f = m[r][c] / m[c][c]
                m[r] = [x - f * y for x, y in zip(m[r], m[c])]
    return [m[i][n] / m[i][i] for i in range(n)]


def standard_coeffs(p: int):
    """Standard p-th order staggered coefficients: M = p/2, so the App. B
    constraint M C = e1 alone fixes C.  Returned as exact fractions."""
    M = p // 2
    a = constraint_matrix(p, M)
    e1 = [Fraction(1)] + [Fraction(0)] * (M - 1)
    return _solve_fraction(a, e1)


# ----------------------------------------------------------------------------
# Eq. (new_op): targets, normalised to k_g1
# ----------------------------------------------------------------------------


def target(kind: str, kappa, r):
    """Normalised target operator at kappa = k1/k_g1 for r = dt/dx1.

    kind 'E': [k]_E1 / k_g1 = tan(pi kappa r)/(pi r)      (Eq. new_op)
    kind 'B': [k]_B1 / k_g1 = sin(2 pi kappa r)/(2 pi r)  (Eq. new_op)
    kind 'xu': [k]_{1,t} / k_g1 = sin(pi kappa r)/(pi r)  (Xu solver, Sec. 4)
    kind 'yeet_E', 'yeet_B': the Yee t-stagger solver (Sec. 4, third solver
        of the comparison), read as Eq. (new_op) with [k]_{1,t} replaced by
        the Yee symbol, so that [k]_E1 [k]_B1 = [k]_Yee^2 (Yee dispersion) and
        [k]_E1/[k]_B1 = 1/cos^2(k1 dt/2) (time-stagger correction):
        [k]_E1/k_g1 = sin(pi kappa)/(pi cos(pi kappa r)),
        [k]_B1/k_g1 = sin(pi kappa) cos(pi kappa r)/pi.
    Works for mpmath or numpy arguments.
    """
    lib = mp if isinstance(kappa, mp.mpf) or isinstance(r, mp.mpf) else np
    pi = lib.pi
    if kind == "E":
        return lib.tan(pi * kappa * r) / (pi * r)
    if kind == "B":
        return lib.sin(2 * pi * kappa * r) / (2 * pi * r)
    if kind == "xu":
        return lib.sin(pi * kappa * r) / (pi * r)
    if kind == "yeet_E":
        return lib.sin(pi * kappa) / (pi * lib.cos(pi * kappa * r))
    if kind == "yeet_B":
        return lib.sin(pi * kappa) * lib.cos(pi * kappa * r) / pi
    raise ValueError(kind)


# ----------------------------------------------------------------------------
# App. B: weighted least squares with the constraint, in mpmath
# ----------------------------------------------------------------------------


def _gauss_legendre_nodes(G: int, dps: int):
    """Gauss-Legendre nodes and weights on [-1, 1] at ``dps`` digits (Newton
    refinement of numpy's double-precision nodes on the Legendre recurrence)."""
    x0, _ = np.polynomial.legendre.leggauss(G)
    nodes, weights = [], []
    with mp.workdps(dps + 10):
        for xi in x0:
            x = mp.mpf(xi)
            for _ in range(100):
                p0, p1 = mp.mpf(1), x
                for k in range(2, G + 1):
                    p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
                dp = G * (x * p1 - p0) / (x * x - 1)
                dx = p1 / dp
                x -= dx
                if abs(dx) < mp.mpf(10) ** (-(dps + 5)):
                    break
            p0, p1 = mp.mpf(1), x
            for k in range(2, G + 1):
                p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
            dp = G * (x * p1 - p0) / (x * x - 1)
            nodes.append(x)
            weights.append(2 / ((1 - x * x) * dp * dp))
    return nodes, weights


def fit_coeffs(M: int, r, kind: str, *, p: int = 2, n: int = 10, wk1=0.4,
               width_factor: int = 2, panels: int = 48, G: int = 40,
               dps: int = 60):
    """App. B: customized coefficients C (length M) fitting target ``kind``.

    Minimises  int_0^{1/2} w(kappa) (sum_j C_j sin((2j-1) pi kappa)/pi - T)^2
    subject to  M C = e1  (order-p accuracy), by solving the KKT system
        [[A, M^T], [M, 0]] [C; lambda] = [b; e1]
    with  A_ij = (2/pi^2) int w sin((2i-1) pi kappa) sin((2j-1) pi kappa),
          b_i  = (2/pi)   int w sin((2i-1) pi kappa) T(kappa),
          w    = exp[-ln2 (width_factor kappa / w_k1)^n].
    Returns a list of mpmath numbers (``dps`` digits).
    """
    with mp.workdps(dps):
        r = mp.mpf(r)
        wk1 = mp.mpf(wk1)
        gx, gw = _gauss_legendre_nodes(G, dps)
        A = mp.zeros(M, M)
        b = mp.zeros(M, 1)
        h = mp.mpf(1) / 2 / panels
        ln2 = mp.log(2)
        for pnl in range(panels):
            a0 = pnl * h
            for xi, wi in zip(gx, gw):
                kap = a0 + (xi + 1) * h / 2
                q = wi * h / 2 * mp.exp(-ln2 * (width_factor * kap / wk1) ** n)
                # sin((2j-1) pi kappa), j = 1..M, by the three-term recurrence
                s1 = mp.sin(mp.pi * kap)
                c2 = 2 * mp.cos(2 * mp.pi * kap)
                s = [s1]
                prev = -s1
                for _ in range(M - 1):
                    s.append(c2 * s[-1] - prev)
                    prev = s[-2]
                t = target(kind, kap, r)
                for i in range(M):
                    qi = q * s[i]
                    b[i] += qi * t
                    for j in range(i, M):
                        A[i, j] += qi * s[j]
        for i in range(M):
            b[i] *= 2 / mp.pi
            for j in range(i, M):
                A[i, j] *= 2 / mp.pi ** 2
                A[j, i] = A[i, j]
        cons = constraint_matrix(p, M)
        nc = len(cons)
        K = mp.zeros(M + nc, M + nc)
        rhs = mp.zeros(M + nc, 1)
        for i in range(M):
            for j in range(M):
                K[i, j] = A[i, j]
            rhs[i] = b[i]
        for ci, row in enumerate(cons):
            for j, v in enumerate(row):
                K[M + ci, j] = mp.mpf(v.numerator) / v.denominator
                K[j, M + ci] = K[M + ci, j]
        rhs[M] = 1
        sol = mp.lu_solve(K, rhs)
        return [sol[i] for i in range(M)]


def fit_pair(M: int, r, **kw):
    """(C^E, C^B) as float64 arrays: the proposed solver's coefficients
    (Eq. new_op targets fitted by App. B)."""
    ce = np.array([float(c) for c in fit_coeffs(M, r, "E", **kw)])
    cb = np.array([float(c) for c in fit_coeffs(M, r, "B", **kw)])
    return ce, cb


# ----------------------------------------------------------------------------
# Sec. 2.1 / 3.1: symbols, dispersion, phase velocity, F, oblique waves
# ----------------------------------------------------------------------------


def symbol(C, k, dx):
    """Sec. 2.1: [k] = sum_j C_j sin((2j-1) k dx/2) / (dx/2)  (numpy, FP64)."""
    k = np.asarray(k, dtype=np.float64)
    out = np.zeros_like(k)
    for j, c in enumerate(np.asarray(C, dtype=np.float64), start=1):
        out = out + c * np.sin((2 * j - 1) * k * dx / 2) / (dx / 2)
    return out


def yee_symbol(k, dx):
    """[k]_Yee = sin(k dx/2)/(dx/2)."""
    return np.sin(np.asarray(k, dtype=np.float64) * dx / 2) / (dx / 2)


def omega_from_symbols(kEkB, dt):
    """Eq. (dispersion) with [omega]_t = sin(omega dt/2)/(dt/2):
    omega = (2/dt) arcsin((dt/2) sqrt([k]_E.[k]_B)).  NaN where unstable."""
    arg = (dt / 2) * np.sqrt(np.asarray(kEkB, dtype=np.float64))
    with np.errstate(invalid="ignore"):
        return (2 / dt) * np.arcsin(arg)


def phase_velocity(CE, CB, k, dx, dt):
    """Eq. (v_phi): v_phi = (2/(k dt)) arcsin((dt/2) sqrt([k]_B1 [k]_E1))."""
    k = np.asarray(k, dtype=np.float64)
    return omega_from_symbols(symbol(CE, k, dx) * symbol(CB, k, dx), dt) / k


def f_factor(CE, CB, k, dx, dt):
    """Fig. 2 caption / Eq. (f2_q): F = sqrt([k]_E1/[k]_B1) cos(omega dt/2),
    omega under numerical dispersion."""
    kE, kB = symbol(CE, k, dx), symbol(CB, k, dx)
    w = omega_from_symbols(kE * kB, dt)
    return np.sqrt(kE / kB) * np.cos(w * dt / 2)


def oblique(CE, CB, k0, theta, dx1, dx2, dt):
    """Sec. 3.1.1: a plane wave with |k| = k0 at angle theta to x1 in the
    x1-x2 plane; x2 operators are Yee.  Returns (v_phi, kappa_factor)."""
    theta = np.asarray(theta, dtype=np.float64)
    k1, k2 = k0 * np.cos(theta), k0 * np.sin(theta)
    kE1, kB1 = symbol(CE, k1, dx1), symbol(CB, k1, dx1)
    kE2 = kB2 = yee_symbol(k2, dx2)
    s = kE1 * kB1 + kE2 * kB2
    w = omega_from_symbols(s, dt)
    vphi = w / k0
    kap = (kE1 * np.cos(theta) + kE2 * np.sin(theta)) / np.sqrt(s) * np.cos(w * dt / 2)
    return vphi, kap


def oblique_vphi_formula(k0, theta, dx1, dx2, dt, eta):
    """Eq. (vphi_ob): the unified closed form for the proposed (eta = 1) and
    Yee (eta = dx1/dt) solvers."""
    theta = np.asarray(theta, dtype=np.float64)
    a = np.sin(eta * k0 * dt * np.cos(theta) / 2) / (eta * dt / 2)
    b = np.sin(k0 * dx2 * np.sin(theta) / 2) / (dx2 / 2)
    return (2 / (k0 * dt)) * np.arcsin((dt / 2) * np.sqrt(a * a + b * b))


def oblique_leading_term(k0, dt, eta):
    """Sec. 3.1.1: theta -> 0 limit of Eq. (vphi_ob),
    (2/(k0 dt)) arcsin[eta^-1 sin(eta k0 dt/2)]."""
    return (2 / (k0 * dt)) * np.arcsin(np.sin(eta * k0 * dt / 2) / eta)


# ----------------------------------------------------------------------------
# Sec. 3.2: CFL
# ----------------------------------------------------------------------------


def cfl_sufficient_dt(CE, CB, dx):
    """Sec. 3.2 sufficient condition, extended to 3D by adding 1/dx3^2:
    dt <= 1/sqrt(sum|C^B| sum|C^E| / dx1^2 + sum_{d>=2} 1/dx_d^2)."""
    sE = float(np.sum(np.abs(CE)))
    sB = float(np.sum(np.abs(CB)))
    s = sB * sE / dx[0] ** 2 + sum(1.0 / d ** 2 for d in dx[1:])
    return 1.0 / np.sqrt(s)


def cfl_exact_max(CE, CB, dx, dt, nk: int = 4097):
    """Sec. 3.2 exact condition: the maximum over real k of
    (dt/2) sqrt(sum C^B s_1 * sum C^E s_1 + sum_{d>=2} s_d^2); stable iff <= 1.
    The x2/x3 terms peak at k_d = pi/dx_d; the x1 product is maximised on a
    grid over [0, pi/dx1] (it can be negative, which only helps)."""
    k1 = np.linspace(0.0, np.pi / dx[0], nk)
    prod = symbol(CE, k1, dx[0]) * symbol(CB, k1, dx[0])
    trans = sum((2.0 / d) ** 2 for d in dx[1:])
    return float((dt / 2) * np.sqrt(np.max(prod) + trans))
