"""Invariants of the oracle's full PIC step with plasma (CPU only)."""
import numpy as np
import pytest

from oracle import fdtd, particles as pt, pic
from paper_2004_03754_amd import workloads as wl


@pytest.mark.parametrize("pusher", ["boris", "analytic"])
def test_gauss_law_preserved_with_deposit(pusher, coeffs16):
    """Sec. 3.3: with the charge-conserving deposit and the Ampere operator
    equal to Yee along x1 (the proposed solver at dt = dx1/2), the Gauss
    residual div_B E - rho stays at its initial value to roundoff, and so
    does Faraday's divergence of B."""
    CE, CB = coeffs16
    n = (24, 6, 5)
    dx = (wl.DX1, wl.DX2, wl.DX3)
    shape = (n[2], n[1], n[0])
    L = [n[d] * dx[d] for d in range(3)]
    E, B = wl.random_fields(n, seed=31, scale=0.05)
    x, u = wl.uniform_particles(400, [0, 0, 0], L, seed=32, u_th=0.3)
    sp = {"x": x, "u": u, "q": -1.0, "m": 1.0, "w": 0.01}
    gauss0 = fdtd.div_ampere(E, CB, dx) - pt.charge_density(sp["x"], -1.0, 0.01, dx, shape)
    divb0 = fdtd.div_faraday(B, CE, dx)
    for _ in range(8):
        E, B = pic.step(E, B, [sp], CE, CB, dx, wl.DT, pusher=pusher, deposit=True)
    gauss = fdtd.div_ampere(E, CB, dx) - pt.charge_density(sp["x"], -1.0, 0.01, dx, shape)
    scale = np.max(np.abs(fdtd.div_ampere(E, CB, dx)))
    assert np.max(np.abs(gauss - gauss0)) < 1e-12 * scale
    assert np.max(np.abs(fdtd.div_faraday(B, CE, dx) - divb0)) < 1e-12 * np.max(np.abs(divb0))
