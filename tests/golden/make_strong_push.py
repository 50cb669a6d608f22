"""Writes strong_push.json: single pushes in uniform fields of 1e2 to 1e5
(the field strengths of the Sec. 4.1 runs at a0 up to 1e4) evaluated at 50
significant digits by oracle.precise, for the GPU strong-field push test.

    python tests/golden/make_strong_push.py

Every field value and position is a short binary fraction, so the staggered
linear gather of a uniform field is exact in FP64 on any implementation: the
test then measures each pusher's own arithmetic against the exact map at the
same FP64 inputs.  Calls only the oracle.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import precise  # noqa: E402

DT = 2 * np.pi / 64  # the workloads' dt = dx1/2 with dx1 = lambda0/32
QM = -1.0


def short(v, bits=8):
    """Round to a multiple of 2^-bits (so that |v| < 2^44 keeps <= 52 bits)."""
    return np.round(np.asarray(v, dtype=np.float64) * 2.0 ** bits) / 2.0 ** bits


def cases():
    g = np.random.default_rng(2024)
    out = []
    for e in (1e2, 1e3, 1e4, 1e5):
        out.append((np.array([e, 0.0, 0.0]), np.zeros(3), "pure E"))
    for d in (1e-4, 1e-2, 0.5):
        out.append((np.array([0.0, 1e4, 0.0]), np.array([0.0, 0.0, short(1e4 * (1 - d))]), f"crossed, |B| = (1 - {d:g}) |E|"))
    for s in (1e2, 1e2, 1e3, 1e3, 1e4, 1e4, 1e4, 1e4, 1e4):
        out.append((short(s * g.standard_normal(3)), short(s * g.standard_normal(3)), f"random {s:g}"))
    return out, g


def main():
    planes, g = cases()
    per = 4
    rec = {"dt": DT, "qm": QM, "per_plane": per, "planes": []}
    for E, B, what in planes:
        us = [np.zeros(3)] + [short(10.0 * g.standard_normal(3), 20) for _ in range(per - 1)]
        p = {"what": what, "E": E.tolist(), "B": B.tolist(), "u": [u.tolist() for u in us]}
        for name, f in (("boris", precise.boris), ("hc", precise.higuera_cary), ("analytic", precise.exact)):
            p[name] = [f(u, E, B, QM, DT) for u in us]
        rec["planes"].append(p)
        print(what, flush=True)
    with open(os.path.join(HERE, "strong_push.json"), "w") as f:
        json.dump(rec, f, indent=1)


if __name__ == "__main__":
    main()
