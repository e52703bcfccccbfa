"""Pins of the oracle's pullbacks: the finite-difference adjoint identity of Sec. 3.4.

<fbar, (K(u + eps v) - K(u - eps v)) / (2 eps)> = <K_u^T fbar, v>.
For the linear operators and the quadratic convection kernel the central
difference is exact up to rounding, so the check is tight; for the RK4 step
(a polynomial in u0) the central difference carries an O(eps^2) error.
A torch-CPU float64 autograd of the step gives an independent second check.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
import synth as S

GRIDS = [(6, 8), (5, 4, 6)]


def _dot(a, b):
    return float(np.sum(a * b))


def _h(n):
    return tuple([1.0, 1.6, 0.9][a] * 2 * math.pi / n[a] for a in range(len(n)))


def _central(fn, u, v, eps):
    return (fn(u + eps * v) - fn(u - eps * v)) / (2 * eps)


@pytest.mark.parametrize("n", GRIDS)
def test_divergence_vjp(n):
    h = _h(n)
    u, v = S.random_field(n, 1), S.random_field(n, 2)
    rbar = S.random_scalar(n, 3)
    jv = _central(lambda x: O.divergence(x, h), u, v, 0.5)
    assert abs(_dot(rbar, jv) - _dot(O.divergence_vjp(rbar, h), v)) < 1e-12 * np.abs(jv).sum()
    # and D^T = -G on the uniform periodic grid
    np.testing.assert_allclose(O.divergence_vjp(rbar, h), -O.gradient(rbar, h), atol=1e-13)


@pytest.mark.parametrize("n", GRIDS)
def test_gradient_vjp(n):
    h = _h(n)
    p, q = S.random_scalar(n, 4), S.random_scalar(n, 5)
    gbar = S.random_field(n, 6)
    jv = _central(lambda x: O.gradient(x, h), p, q, 0.5)
    assert abs(_dot(gbar, jv) - _dot(O.gradient_vjp(gbar, h), q)) < 1e-12 * np.abs(jv).sum()
    np.testing.assert_allclose(O.gradient_vjp(gbar, h), -O.divergence(gbar, h), atol=1e-13)


@pytest.mark.parametrize("n", GRIDS)
def test_diffusion_vjp(n):
    h = _h(n)
    u, v, fbar = S.random_field(n, 7), S.random_field(n, 8), S.random_field(n, 9)
    jv = _central(lambda x: O.diffusion(x, h, 0.3), u, v, 0.5)
    assert abs(_dot(fbar, jv) - _dot(O.diffusion_vjp(fbar, h, 0.3), v)) < 1e-12 * np.abs(jv).sum()


@pytest.mark.parametrize("n", GRIDS + [(3, 3), (3, 3, 3)])
def test_convection_vjp_exact_central_difference(n):
    h = _h(n)
    u, v, fbar = S.random_field(n, 10), S.random_field(n, 11), S.random_field(n, 12)
    jv = _central(lambda x: O.convection(x, h), u, v, 0.25)
    lhs = _dot(fbar, jv)
    rhs = _dot(O.convection_vjp(u, fbar, h), v)
    assert abs(lhs - rhs) < 1e-12 * np.abs(fbar * jv).sum()


def test_convection_vjp_gather_components():
    """Element-wise: each ubar entry equals the derivative of <fbar, C(u)> w.r.t. that entry."""
    n = (3, 4, 3)
    h = _h(n)
    u, fbar = S.random_field(n, 13), S.random_field(n, 14)
    g = O.convection_vjp(u, fbar, h)
    rng = np.random.default_rng(0)
    for _ in range(12):
        idx = tuple(rng.integers(0, s) for s in u.shape)
        e = np.zeros_like(u)
        e[idx] = 1.0
        fd = _dot(fbar, _central(lambda x: O.convection(x, h), u, e, 0.5))
        assert abs(fd - g[idx]) < 1e-12 * (1 + abs(fd))


@pytest.mark.parametrize("n", GRIDS)
def test_rhs_vjp(n):
    h = _h(n)
    u, v, fbar = S.random_field(n, 15), S.random_field(n, 16), S.random_field(n, 17)
    jv = _central(lambda x: O.rhs(x, h, 0.05), u, v, 0.25)
    assert abs(_dot(fbar, jv) - _dot(O.rhs_vjp(u, fbar, h, 0.05), v)) < 1e-12 * np.abs(fbar * jv).sum()


@pytest.mark.parametrize("n", GRIDS)
def test_poisson_and_projection_self_adjoint(n):
    h = _h(n)
    r, s = S.random_scalar(n, 18), S.random_scalar(n, 19)
    assert abs(_dot(O.poisson_solve(r, h), s) - _dot(r, O.poisson_solve_vjp(s, h))) < 1e-11 * np.abs(r).sum()
    u, v = S.random_field(n, 20), S.random_field(n, 21)
    assert abs(_dot(O.project(u, h)[0], v) - _dot(u, O.project_vjp(v, h))) < 1e-11 * np.abs(u).sum()


def _torch_step(u0, h, nu, dt):
    """RK4 step written with torch ops (roll/fft), used only for autograd."""
    d = u0.shape[0]

    def nxt(f, a):
        return torch.roll(f, -1, dims=d - 1 - a)

    def prv(f, a):
        return torch.roll(f, 1, dims=d - 1 - a)

    def div(u):
        return sum((u[a] - prv(u[a], a)) / h[a] for a in range(d))

    def grad(p):
        return torch.stack([(nxt(p, a) - p) / h[a] for a in range(d)])

    def F(u):
        outs = []
        for a in range(d):
            acc = torch.zeros_like(u[a])
            for b in range(d):
                flux = 0.25 * (u[a] + nxt(u[a], b)) * (u[b] + nxt(u[b], a))
                acc = acc - (flux - prv(flux, b)) / h[b]
                acc = acc + nu * (nxt(u[a], b) - 2 * u[a] + prv(u[a], b)) / h[b] ** 2
            outs.append(acc)
        return torch.stack(outs)

    n = tuple(reversed(u0.shape[1:]))
    lam = torch.zeros(u0.shape[1:], dtype=torch.float64)
    for a in range(d):
        k = torch.arange(n[a], dtype=torch.float64)
        shp = [1] * d
        shp[d - 1 - a] = n[a]
        lam = lam - (4 * torch.sin(math.pi * k / n[a]) ** 2 / h[a] ** 2).reshape(shp)
    lam[(0,) * d] = 1.0

    def P(u):
        p = torch.real(torch.fft.ifftn(torch.fft.fftn(div(u)) / lam))
        return u - grad(p)

    u = u0
    fs = []
    for i, c in enumerate((0.5, 0.5, 1.0, None)):
        fs.append(F(u))
        if c is not None:
            u = P(u0 + dt * c * fs[i])
    return P(u0 + dt * (fs[0] + 2 * fs[1] + 2 * fs[2] + fs[3]) / 6)


@pytest.mark.parametrize("n", [(8, 6), (4, 6, 5)])
def test_step_vjp_against_torch_autograd_and_fd(n):
    h = S.spacing(n)
    nu, dt = 0.05, 0.05
    u0 = S.turbulence_ic(n, seed=1, k0=2)
    ubar = S.random_field(n, 22)
    g = O.step_rk4_vjp(u0, ubar, h, nu, dt)
    t = torch.tensor(u0, requires_grad=True)
    out = _torch_step(t, h, nu, dt)
    np.testing.assert_allclose(out.detach().numpy(), O.step_rk4(u0, h, nu, dt), atol=1e-13)
    (out * torch.tensor(ubar)).sum().backward()
    np.testing.assert_allclose(g, t.grad.numpy(), atol=1e-12 * np.abs(g).max())
    for seed in (30, 31, 32):
        v = S.random_field(n, seed)
        fd = _dot(ubar, _central(lambda x: O.step_rk4(x, h, nu, dt), u0, v, 1e-4))
        assert abs(fd - _dot(g, v)) < 1e-7 * np.abs(g * v).sum()


def test_rollout_loss_gradient_central_difference():
    n = (8, 6)
    h = S.spacing(n)
    nu, dt = 0.05, 0.05
    u0 = S.turbulence_ic(n, seed=3, k0=2)
    refs = [S.turbulence_ic(n, seed=10 + s, k0=2) for s in range(4)]
    g = O.rollout_loss_grad(u0, refs, h, nu, dt)
    for seed in (40, 41):
        v = S.random_field(n, seed)
        fd = (O.rollout_loss(u0 + 1e-5 * v, refs, h, nu, dt) - O.rollout_loss(u0 - 1e-5 * v, refs, h, nu, dt)) / 2e-5
        assert abs(fd - _dot(g, v)) < 1e-7 * np.abs(g * v).sum()
