"""Pins of the high-precision pushers (oracle.precise) and the FP64 oracle's
own accuracy in strong fields (CPU only)."""
import json
import os

import numpy as np
import pytest

from oracle import particles as pt, precise as pr

HERE = os.path.dirname(__file__)
DT = 2 * np.pi / 64


def test_pure_electric_field_kick_is_exact():
    """Sec. 1 / 4.1: with B = 0, du/dt = (q/m) E, so every pusher gives
    u + (q/m) E dt exactly (Boris and Higuera-Cary by construction, the exact
    push because it solves the equation of motion), also at 1e4."""
    g = np.random.default_rng(1)
    for s in (1.0, 1e4):
        for _ in range(3):
            u, E = 3 * g.standard_normal(3), s * g.standard_normal(3)
            want = u - E * DT
            for f in (pr.boris, pr.higuera_cary, pr.exact):
                got = np.array(f(u, E, np.zeros(3), -1.0, DT))
                assert np.linalg.norm(got - want) <= 2e-16 * np.linalg.norm(want)


def test_pure_magnetic_field_rotation_angles():
    """Sec. 1 / 4.1: with E = 0, du/dt = (q/m) u x B/gamma = Omega x u with
    Omega = -(q/m) B/gamma, so |u| and gamma are conserved; the exact push
    rotates u about B by -(q/m)|B| dt/gamma, the Boris push by
    2 arctan(-(q/m)|B| dt/(2 gamma)); Higuera-Cary keeps |u|."""
    g = np.random.default_rng(2)
    for s in (1.0, 1e4):
        B = s * g.standard_normal(3)
        u = 5 * g.standard_normal(3)
        b = B / np.linalg.norm(B)
        gam = np.sqrt(1 + u @ u)
        up = u - (u @ b) * b
        w = np.linalg.norm(B) / gam  # -(q/m) |B|/gamma with q/m = -1
        for f, ang in ((pr.exact, w * DT), (pr.boris, 2 * np.arctan(w * DT / 2)), (pr.higuera_cary, None)):
            got = np.array(f(u, np.zeros(3), B, -1.0, DT))
            assert abs(np.linalg.norm(got) - np.linalg.norm(u)) <= 1e-15 * np.linalg.norm(u)
            if ang is None:
                continue
            # rotation of u_perp by ang about b (right-handed)
            want = (u @ b) * b + np.cos(ang) * up + np.sin(ang) * np.cross(b, up)
            assert np.linalg.norm(got - want) <= 1e-13 * np.linalg.norm(u)


def test_exact_push_null_field_from_rest():
    """A null crossed field (E along x2, B along x3, |E| = |B|) from rest:
    the orbit solves u2 + u2^3/6 = |q E| t in lab time, with u1 = u2^2/2
    (gamma - u1 = 1), reached in one exact push of length dt for any |E|."""
    for e in (0.5, 30.0, 1e4):
        u = np.array(pr.exact(np.zeros(3), [0.0, e, 0.0], [0.0, 0.0, e], -1.0, DT))
        u2 = abs(u[1])
        assert abs(u2 + u2 ** 3 / 6 - e * DT) <= 1e-15 * max(1.0, e * DT)
        assert abs(u[0] - u2 ** 2 / 2) <= 1e-15 * max(1.0, u2 ** 2)
        assert abs(u[2]) <= 1e-15 * max(1.0, u2)


def test_exact_push_semigroup_and_reversal():
    """Constant fields: two pushes of dt/2 equal one of dt, and a push of
    -dt undoes one of dt, to the FP64 rounding of the intermediate state
    (times its conditioning)."""
    g = np.random.default_rng(3)
    for s in (1.0, 30.0):
        E, B = s * g.standard_normal(3), s * g.standard_normal(3)
        u = 2 * g.standard_normal(3)
        one = np.array(pr.exact(u, E, B, -1.0, DT))
        two = np.array(pr.exact(pr.exact(u, E, B, -1.0, DT / 2), E, B, -1.0, DT / 2))
        back = np.array(pr.exact(one, E, B, -1.0, -DT))
        assert np.linalg.norm(one - two) <= 1e-13 * max(1.0, np.linalg.norm(one))
        assert np.linalg.norm(back - u) <= 1e-13 * max(1.0, np.linalg.norm(u))


def test_precision_is_converged():
    """50 and 80 significant digits round to the same FP64 result."""
    g = np.random.default_rng(4)
    E, B, u = 1e4 * g.standard_normal(3), 1e4 * g.standard_normal(3), 3 * g.standard_normal(3)
    for f in (pr.boris, pr.higuera_cary, pr.exact):
        assert f(u, E, B, -1.0, DT) == f(u, E, B, -1.0, DT, dps=80)


@pytest.fixture(scope="module")
def strong():
    with open(os.path.join(HERE, "golden", "strong_push.json")) as f:
        return json.load(f)


def test_fp64_oracle_accuracy_in_strong_fields(strong):
    """The FP64 oracle's pushers against the 50-digit values of the strong
    field cases (uniform fields of 1e2 to 1e5): per particle
    |u - u_exact| / max(1, |u_exact|).  Measured: Boris 6e-16, the exact push
    (8x8 expm) 6e-14, Higuera-Cary 8e-14 (it loses digits to the
    cancellation in sigma = 1 + u-^2 - tau^2, |tau| ~ 500 at 1e4).  These are
    the oracle's own errors at these inputs; the GPU is measured against the
    50-digit values, not against the FP64 oracle."""
    funcs = {"boris": pt.boris, "hc": pt.higuera_cary, "analytic": pt.analytic}
    worst = {}
    for p in strong["planes"]:
        u = np.array(p["u"]).T
        E = np.repeat(np.array(p["E"])[:, None], u.shape[1], axis=1)
        B = np.repeat(np.array(p["B"])[:, None], u.shape[1], axis=1)
        for name, f in funcs.items():
            got = f(u, E, B, strong["qm"], strong["dt"])
            ref = np.array(p[name]).T
            err = np.linalg.norm(got - ref, axis=0) / np.maximum(1.0, np.linalg.norm(ref, axis=0))
            worst[name] = max(worst.get(name, 0.0), float(err.max()))
    assert worst["boris"] <= 1e-14, worst
    assert worst["analytic"] <= 1e-12, worst
    assert worst["hc"] <= 1e-12, worst
