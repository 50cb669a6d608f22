"""Pins of the adjoint oracle (CPU only).

The reference gradients are torch autograd over a plain torch restatement of
the forward step.  That restatement is pinned to the NumPy oracle's values,
its gradients to central finite differences, and the operator transposition
that the GPU adjoint is built on to the NumPy oracle's own curls.
"""
import numpy as np
import pytest
import torch

from oracle import adjoint as ad, fdtd, pic
from paper_2004_03754_amd import workloads as wl

DX = (wl.DX1, wl.DX2, wl.DX3)


def _t(a):
    return torch.tensor(np.asarray(a), dtype=torch.float64)  # a copy: the tests modify it in place


def _case(n, seed, npart, ndim, scale=0.3, u_th=0.2):
    E, B = wl.random_fields(n, seed=seed, scale=scale)
    L = [n[d] * DX[d] for d in range(3)]
    x, u = wl.uniform_particles(npart, [0, 0, 0], L, seed=seed + 1, u_th=u_th)
    if ndim == 2:
        x[2] = 0.5 * DX[2]
    return E, B, x, u


@pytest.mark.parametrize("ndim,n", [(3, (20, 6, 5)), (2, (32, 8, 1))])
def test_torch_forward_matches_numpy_oracle(ndim, n, coeffs16):
    """The torch restatement reproduces the NumPy oracle's step (fields,
    positions and momenta) to roundoff, Boris pusher, 10 steps, with
    electrons crossing the periodic seam of every direction both ways (the
    wrap must be exact in FP64)."""
    CE, CB = coeffs16
    E, B, x, u = _case(n, 71, 50, ndim, u_th=0.5)
    L = [n[d] * DX[d] for d in range(3)]
    for d in range(ndim):
        x[d, 2 * d] = L[d] - 1e-3 * DX[d]
        u[d, 2 * d] = 2.0
        x[d, 2 * d + 1] = 1e-3 * DX[d]
        u[d, 2 * d + 1] = -2.0
    sp = {"x": x.copy(), "u": u.copy(), "q": -1.0, "m": 1.0, "w": 1.0}
    Er, Br = pic.run(E, B, [sp], CE, CB, DX, wl.DT, 10, pusher="boris", ndim=ndim)
    Et, Bt, xt, ut = ad.run([_t(e) for e in E], [_t(b) for b in B], _t(x), _t(u), _t(CE), _t(CB), DX, wl.DT,
                            -1.0, 10, ndim)
    for a, r in zip(list(Et) + list(Bt), list(Er) + list(Br)):
        assert np.max(np.abs(a.numpy() - r)) <= 1e-13 * max(1.0, np.max(np.abs(r)))
    assert np.max(np.abs(xt.numpy() - sp["x"])) < 1e-12
    assert np.max(np.abs(ut.numpy() - sp["u"])) < 1e-13


@pytest.mark.parametrize("ndim,n", [(3, (12, 5, 4)), (2, (24, 6, 1))])
def test_curl_transposition(ndim, n):
    """App. B operators: the transpose of Faraday's x1 operator is minus
    Ampere's with the same coefficients, and Yee's forward difference is
    minus the backward one, so <curl_E[C] e, b> = <e, curl_B[C] b> for any
    C; the adjoint field step is built on this."""
    g = np.random.default_rng(5)
    C = g.standard_normal(16)
    E, _ = wl.random_fields(n, seed=81)
    _, B = wl.random_fields(n, seed=82)
    cE = fdtd.curl_E(E, C, DX)
    cB = fdtd.curl_B(B, C, DX)
    lhs = sum(np.vdot(a, b) for a, b in zip(cE, B))
    rhs = sum(np.vdot(a, b) for a, b in zip(E, cB))
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + np.sqrt(sum(np.vdot(a, a) for a in cE)) * np.sqrt(
        sum(np.vdot(b, b) for b in B)))
    # and the transpose is not the identity map (a wrong sign would fail here)
    assert abs(lhs) > 1e-3


def test_torch_exact_pusher_matches_numpy_and_differences():
    """The torch exact push equals the NumPy oracle's (weak to strong fields,
    including near-null crossed fields of 1e4), and its implicit-function
    gradient with respect to u, E and B matches central differences."""
    from oracle import particles as pt
    g = np.random.default_rng(11)
    n = 12
    E = g.standard_normal((3, n)) * np.repeat([0.3, 5.0, 50.0], 4)
    B = g.standard_normal((3, n)) * np.repeat([0.3, 5.0, 50.0], 4)
    E[:, -1] = [0, 1e4, 0]
    B[:, -1] = [0, 0, 0.99e4]
    u = g.standard_normal((3, n)) * 2
    u[:, -1] = 0
    ref = pt.analytic(u, E, B, -1.0, wl.DT)
    got = ad.analytic(_t(u), _t(E), _t(B), -1.0, wl.DT).detach().numpy()
    assert np.max(np.abs(got - ref) / np.maximum(1.0, np.abs(ref))) <= 1e-12
    lam = _t(g.standard_normal((3, n)))
    leaves = [_t(u).requires_grad_(), _t(E).requires_grad_(), _t(B).requires_grad_()]
    L = torch.sum(ad.analytic(*leaves, -1.0, wl.DT) * lam)
    grads = torch.autograd.grad(L, leaves)
    h = 1e-6
    for which in range(3):
        for (d, p) in [(0, 0), (1, 5), (2, 9), (1, n - 1)]:
            vals = []
            for sgn in (1, -1):
                args = [_t(u), _t(E), _t(B)]
                step = h * max(1.0, abs(float(args[which][d, p])))
                args[which][d, p] += sgn * step
                with torch.no_grad():
                    vals.append(float(torch.sum(ad.analytic(*args, -1.0, wl.DT) * lam)))
            fd = (vals[0] - vals[1]) / (2 * step)
            gr = float(grads[which][d, p])
            assert abs(fd - gr) <= 1e-5 * max(1.0, abs(fd)), (which, d, p, fd, gr)


def _loss(E, B, x, u, CE, CB, nsteps, ndim, w):
    Ef, Bf, xf, uf = ad.run(E, B, x, u, CE, CB, DX, wl.DT, -1.0, nsteps, ndim)
    # a mix of the two losses plus position and B terms so every cotangent is non-zero
    return (ad.loss_gamma(uf) + ad.loss_phase(Ef[1], w[0]) + torch.sum(w[1] * Bf[2]) + torch.sum(w[2] * Ef[0])
            + 0.1 * torch.sum(torch.sin(xf[0])))


@pytest.mark.parametrize("ndim,n", [(3, (12, 5, 4)), (2, (24, 6, 1))])
def test_autograd_matches_central_differences(ndim, n, coeffs16):
    """Gradients of a scalar loss after 4 steps with respect to C^E, C^B,
    one field value and one momentum, against central differences."""
    CE, CB = coeffs16
    E, B, x, u = _case(n, 91, 30, ndim, scale=0.5, u_th=0.5)
    g = np.random.default_rng(3)
    shape = (n[2], n[1], n[0])
    w = [_t(g.standard_normal(shape)), _t(g.standard_normal(shape)), _t(g.standard_normal(shape))]
    leaves = dict(E=[_t(e).requires_grad_() for e in E], B=[_t(b).requires_grad_() for b in B],
                  x=_t(x).requires_grad_(), u=_t(u).requires_grad_(), CE=_t(CE).requires_grad_(),
                  CB=_t(CB).requires_grad_())
    nsteps = 4
    L = _loss(leaves["E"], leaves["B"], leaves["x"], leaves["u"], leaves["CE"], leaves["CB"], nsteps, ndim, w)
    L.backward()

    def value(mod):
        with torch.no_grad():
            a = dict(E=[_t(e) for e in E], B=[_t(b) for b in B], x=_t(x), u=_t(u), CE=_t(CE), CB=_t(CB))
            mod(a)
            return float(_loss(a["E"], a["B"], a["x"], a["u"], a["CE"], a["CB"], nsteps, ndim, w))

    checks = [
        ("CE", 0, lambda a, h: a["CE"].__setitem__(0, a["CE"][0] + h), leaves["CE"].grad[0]),
        ("CE", 3, lambda a, h: a["CE"].__setitem__(3, a["CE"][3] + h), leaves["CE"].grad[3]),
        ("CB", 0, lambda a, h: a["CB"].__setitem__(0, a["CB"][0] + h), leaves["CB"].grad[0]),
        ("CB", 2, lambda a, h: a["CB"].__setitem__(2, a["CB"][2] + h), leaves["CB"].grad[2]),
        ("E2", 0, lambda a, h: a["E"][1].view(-1).__setitem__(7, a["E"][1].view(-1)[7] + h),
         leaves["E"][1].grad.view(-1)[7]),
        ("B3", 0, lambda a, h: a["B"][2].view(-1).__setitem__(11, a["B"][2].view(-1)[11] + h),
         leaves["B"][2].grad.view(-1)[11]),
        ("u", 0, lambda a, h: a["u"].__setitem__((1, 4), a["u"][1, 4] + h), leaves["u"].grad[1, 4]),
        ("x", 0, lambda a, h: a["x"].__setitem__((0, 5), a["x"][0, 5] + h), leaves["x"].grad[0, 5]),
    ]
    h = 1e-6
    for name, j, mod, gr in checks:
        fd = (value(lambda a: mod(a, h)) - value(lambda a: mod(a, -h))) / (2 * h)
        assert abs(fd - float(gr)) <= 2e-6 * max(1.0, abs(fd)), (name, j, fd, float(gr))
