"""The allocation-free adjoint step (pic_adjoint_step_noalloc) against
pic_adjoint_step, through the C ABI: two calls in a row on one device, the
second on a smaller mesh, each compared with the allocating entry point on
the same inputs, plus the refusal of a mesh beyond the fixed scratch."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_2004_03754_amd import binding as b, workloads as wl  # noqa: E402

torch = pytest.importorskip("torch")
from gpu_util import check, dev, host  # noqa: E402

DX = (wl.DX1, wl.DX2, wl.DX3)


def _run(n, ndim, npart, seed, pusher, noalloc, CE, CB, with_next, out_of_place=False):
    E, B = wl.random_fields(n, seed=seed, scale=0.3)
    L = [n[d] * DX[d] for d in range(3)]
    x, u = wl.uniform_particles(npart, [0, 0, 0], L, seed=seed + 1, u_th=0.3)
    if ndim == 2:
        x[2] = np.floor(x[2] / DX[2]) + 0.5 if n[2] > 1 else 0.5
    g = np.random.default_rng(seed + 2)
    shape = (n[2], n[1], n[0])
    lE = [dev(g.standard_normal(shape)) for _ in range(3)]
    lB = [dev(g.standard_normal(shape)) for _ in range(3)]
    lx, lu = dev(g.standard_normal((3, npart))), dev(g.standard_normal((3, npart)))
    grid = b.Grid([dev(e) for e in E], [dev(v) for v in B], DX if ndim == 3 else DX[:2], wl.DT, CE, CB, ndim=ndim)
    p = b.Particles(dev(x), dev(u), q=-1.0, m=1.0)
    lam = b.Particles(lx, lu, q=-1.0, m=1.0)
    gCE = torch.full((16,), 0.25, dtype=torch.float64, device="cuda:0")
    gCB = torch.full((16,), -0.5, dtype=torch.float64, device="cuda:0")
    nxt = {}
    if with_next:
        pn = b.Particles(dev(x), dev(u), q=-1.0, m=1.0)
        En = [torch.empty_like(a) for a in grid.E]
        Bn = [torch.empty_like(a) for a in grid.B]
        Bh = [torch.empty_like(a) for a in grid.B]
        grid.step_to([pn], En, Bn, pusher=pusher, B_half=Bh)
        nxt = {"next_E": En, "next_B": Bn, "half_B": Bh}
    if out_of_place:
        nxt["out_E"] = [torch.empty_like(a) for a in lE]
        nxt["out_B"] = [torch.empty_like(a) for a in lB]
    grid.adjoint_step(lE, lB, gCE, gCB, [p], [lam], pusher=pusher, noalloc=noalloc, **nxt)
    grid.sync()
    fo = (nxt["out_E"] + nxt["out_B"]) if out_of_place else (lE + lB)
    out = [host(a) for a in fo] + [host(lx), host(lu), host(gCE), host(gCB)]
    grid.close()
    return out


@pytest.mark.parametrize("pusher", ["boris", "analytic"])
def test_noalloc_adjoint_matches_allocating_entry_point(pusher, coeffs16):
    """Two allocation-free calls in a row (a 2D stack of 16 planes of
    2048 x 64 on the fused out-of-place path, then a smaller 3D mesh in
    place), each against pic_adjoint_step on the same inputs: field,
    particle and coefficient cotangents to 1e-12 (norm-wise; the particle scatter uses atomics, so the last bits of the
    field cotangents may differ between any two runs)."""
    CE, CB = coeffs16
    cases = [((2048, 64, 16), 2, 3000, 31, True, True), ((256, 8, 6), 3, 500, 41, False, False)]
    for n, ndim, npart, seed, with_next, oop in cases:
        ref = _run(n, ndim, npart, seed, pusher, False, CE, CB, with_next, oop)
        got = _run(n, ndim, npart, seed, pusher, True, CE, CB, with_next, oop)
        names = ["lE1", "lE2", "lE3", "lB1", "lB2", "lB3", "lx", "lu", "gCE", "gCB"]
        for name, g_, r in zip(names, got, ref):
            if name == "lx" and ndim == 2:
                g_, r = g_[:2], r[:2]
            scale = max(float(np.max(np.abs(r))), 1e-300)
            check(float(np.max(np.abs(g_ - r))) / scale, 1e-12, f"noalloc adjoint {pusher} {n} {name}")


def test_noalloc_adjoint_refuses_meshes_beyond_its_scratch(coeffs16):
    """A mesh needing more than the fixed 2^17 doubles of partial sums on
    the in-place path (8192 blocks of 1024 x 8 cells) is refused with
    PIC_EUNSUPPORTED before any launch; the allocating entry point takes
    it."""
    CE, CB = coeffs16
    n = (1024, 256, 264)  # 8448 blocks of 1024 x 8 cells (69M cells)
    shape = (n[2], n[1], n[0])
    z = [torch.zeros(shape, dtype=torch.float64, device="cuda:0") for _ in range(6)]
    grid = b.Grid(z[:3], z[3:], DX, wl.DT, CE, CB)
    lE = [torch.zeros(shape, dtype=torch.float64, device="cuda:0") for _ in range(3)]
    lB = [torch.zeros(shape, dtype=torch.float64, device="cuda:0") for _ in range(3)]
    g = [torch.zeros(16, dtype=torch.float64, device="cuda:0") for _ in range(2)]
    with pytest.raises(b.YeePICError) as e:
        grid.adjoint_step(lE, lB, g[0], g[1], noalloc=True)
    assert e.value.code == -6
    grid.adjoint_step(lE, lB, g[0], g[1])
    grid.sync()
    assert float(host(g[0]).max()) == 0.0
    grid.close()
