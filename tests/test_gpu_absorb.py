"""GPU parity of the absorbing layers at the x1 ends of the window (graded
damping of Cerjan et al. 1985, pic_set_absorber) against the oracle, with and
without window moves, and the reflection of a laser pulse entering them."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import absorb, pic, window  # noqa: E402
from paper_2004_03754_amd import binding as b, workloads as wl  # noqa: E402

torch = pytest.importorskip("torch")
from gpu_util import assert_fields_close, check, dev, host  # noqa: E402

DX = (wl.DX1, wl.DX2, wl.DX3)
TOL = {"fp64": 1e-12, "fp32": 1e-5}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("ndim", [3, 2])
def test_absorber_steps_match_oracle(ndim, prec, coeffs16):
    """Five vacuum steps with 16-cell layers (sigma = 1.5) on random fields,
    through pic_step_n, pic_field_sweep and pic_step_to, against the
    oracle's steps followed by its damping."""
    CE, CB = coeffs16
    n = (256, 6, 5) if ndim == 3 else (256, 10, 1)
    dtype = torch.float64 if prec == "fp64" else torch.float32
    E, B = wl.random_fields(n, seed=91)
    if prec == "fp32":
        E = [e.astype(np.float32).astype(np.float64) for e in E]
        B = [v.astype(np.float32).astype(np.float64) for v in B]
    dx = DX if ndim == 3 else DX[:2]
    grid = b.Grid([dev(e, dtype) for e in E], [dev(v, dtype) for v in B], dx, wl.DT, CE, CB, prec=prec, ndim=ndim)
    grid.set_absorber(16, 1.5)
    grid.step_n([], 3)
    grid.sweep()
    Eo = [torch.empty_like(a) for a in grid.E]
    Bo = [torch.empty_like(a) for a in grid.B]
    grid.step_to([], Eo, Bo)
    grid.sync()
    Er, Br = pic.run(E, B, [], CE, CB, DX, wl.DT, 5, ndim=ndim, absorb=(16, 1.5))
    assert_fields_close(Eo, Er, TOL[prec], "absorber steps E", joint=prec == "fp32")
    assert_fields_close(Bo, Br, TOL[prec], "absorber steps B", joint=prec == "fp32")
    grid.close()


def test_absorber_follows_the_moving_window(coeffs16):
    """Steps and window moves (11, 0, 40 cells) with 24-cell layers: the ring
    fields, seen from the window origin, equal the oracle's shifted window
    with the layers at its own ends (FP64 1e-12)."""
    CE, CB = coeffs16
    n = (256, 6, 4)
    E, B = wl.random_fields(n, seed=92)
    grid = b.Grid([dev(e) for e in E], [dev(v) for v in B], DX, wl.DT, CE, CB)
    grid.set_absorber(24, 1.0)
    for s in (11, 0, 40):
        grid.step_n([], 3)
        grid.move_window(s)
        E, B = pic.run(E, B, [], CE, CB, DX, wl.DT, 3, absorb=(24, 1.0))
        E, B = window.move(E, B, [], s, DX[0])
    grid.step_n([], 2)
    E, B = pic.run(E, B, [], CE, CB, DX, wl.DT, 2, absorb=(24, 1.0))
    grid.sync()
    origin, _ = grid.window()
    got = [np.roll(host(a), -origin, axis=-1) for a in grid.E + grid.B]
    assert_fields_close(got[:3], E, 1e-12, "window + absorber E")
    assert_fields_close(got[3:], B, 1e-12, "window + absorber B")
    grid.close()


@pytest.mark.parametrize("direction", [1, -1])
def test_pulse_is_absorbed_on_gpu(direction, coeffs16):
    """A sin^2 pulse of 4 lambda0 on a 768-cell periodic strip runs 928 steps
    into the 32-cell layer at the end it moves to (sigma = 1), on the GPU:
    the energy left in the interior (whatever the layer reflected) and the
    total are below 1e-7 of the incident energy, as in the oracle."""
    CE, CB = coeffs16
    n = (768, 2, 1)
    E, B = wl.laser_fields(n, DX, wl.Sin2Pulse(a0=1.0, Lp=4 * wl.LAMBDA0), x_head=448 * DX[0])
    if direction < 0:
        E = (E[0], E[1][..., ::-1].copy(), E[2])
        B = (B[0], B[1], -B[2][..., ::-1].copy())
    e0 = absorb.field_energy(E, B, DX)
    grid = b.Grid([dev(e) for e in E], [dev(v) for v in B], DX[:2], wl.DT, CE, CB, ndim=2)
    grid.set_absorber(32, 1.0)
    grid.step_n([], 928)
    grid.sync()
    Eg, Bg = [host(a) for a in grid.E], [host(a) for a in grid.B]
    s = slice(32, n[0] - 32)
    inner = absorb.field_energy([e[..., s] for e in Eg], [v[..., s] for v in Bg], DX)
    check(inner / e0, 1e-7, f"pulse reflected by the layer (direction {direction})")
    check(absorb.field_energy(Eg, Bg, DX) / e0, 1e-7, f"pulse energy left (direction {direction})")
    grid.close()


def test_adjoint_refuses_absorber(coeffs16):
    CE, CB = coeffs16
    shape = (2, 4, 64)
    z = [dev(np.zeros(shape)) for _ in range(6)]
    grid = b.Grid(z[:3], z[3:], DX, wl.DT, CE, CB)
    grid.set_absorber(8, 1.0)
    lE = [dev(np.zeros(shape)) for _ in range(3)]
    lB = [dev(np.zeros(shape)) for _ in range(3)]
    g = [torch.zeros(16, dtype=torch.float64, device="cuda:0") for _ in range(2)]
    with pytest.raises(b.YeePICError) as e:
        grid.adjoint_step(lE, lB, g[0], g[1])
    assert e.value.code == -6
    with pytest.raises(b.YeePICError):
        grid.set_absorber(40, 1.0)  # 2W > n1
    grid.close()
