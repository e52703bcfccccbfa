"""Pins of the oracle's Wray3 step (the low-storage three-stage Runge-Kutta
scheme named in Sec. 2.6.2 and Sec. 3.3) and of its pullback.

The oracle uses Wray's two-register recurrence; the pins use other routes:
* the coefficients satisfy the textbook order conditions of a third-order
  three-stage method (so its stability polynomial is 1 + z + z^2/2 + z^3/6);
* on Taylor-Green and shear-wave fields (which the projected stage map keeps
  in shape) the step multiplies by that polynomial exactly;
* a generic projected Butcher-tableau integrator in torch gives the same step
  and, through autograd, the same pullback;
* halving dt cuts the error of a nonlinear run by about 8;
* central differences of the step match the pullback.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import torch

import oracle as O
import synth as S


def _dot(a, b):
    return float(np.sum(a * b))


def _tableau():
    """Butcher tableau implied by the two-register coefficients, in exact fractions."""
    g = [Fraction(8, 15), Fraction(5, 12), Fraction(3, 4)]
    z = [Fraction(-17, 60), Fraction(-5, 12)]
    # u_1 = u0 + dt g1 F0 ; u_2 = u_1 + dt (g2 F1 + z1 F0) ; u_3 = u_2 + dt (g3 F2 + z2 F1)
    a21 = g[0]
    a31, a32 = g[0] + z[0], g[1]
    b = [g[0] + z[0], g[1] + z[1], g[2]]
    return [[Fraction(0)], [a21], [a31, a32]], b


def test_coefficients_are_the_oracle_constants():
    assert O.WRAY3_G == pytest.approx((8 / 15, 5 / 12, 3 / 4), abs=0)
    assert O.WRAY3_Z == pytest.approx((-17 / 60, -5 / 12), abs=0)


def test_third_order_conditions():
    A, b = _tableau()
    c = [sum(row) for row in A]
    assert sum(b) == 1
    assert sum(bi * ci for bi, ci in zip(b, c)) == Fraction(1, 2)
    assert sum(bi * ci * ci for bi, ci in zip(b, c)) == Fraction(1, 3)
    bac = sum(b[i] * sum(A[i][j] * c[j] for j in range(len(A[i]))) for i in range(3))
    assert bac == Fraction(1, 6)
    # the two-register form reaches the classical low-storage tableau
    assert b == [Fraction(1, 4), Fraction(0), Fraction(3, 4)]
    assert c == [0, Fraction(8, 15), Fraction(2, 3)]


def _r3(z):
    return 1 + z + z * z / 2 + z ** 3 / 6


def test_taylor_green_2d_wray3_closed_form():
    nn, nu, dt, steps = 64, 0.01, 1e-3, 100
    n = (nn, nn)
    h = S.spacing(n)
    u0 = S.taylor_green_2d(n)
    u = u0.copy()
    for _ in range(steps):
        u = O.step_wray3(u, h, nu, dt)
    lam = -2 * 4 * math.sin(h[0] / 2) ** 2 / h[0] ** 2
    exact = _r3(nu * lam * dt) ** steps * u0
    assert np.linalg.norm(u - exact) / np.linalg.norm(exact) < 1e-13


def test_shear_wave_3d_wray3_closed_form():
    n = (6, 12, 4)
    nu, dt, m = 0.1, 5e-3, 2
    h = S.spacing(n)
    u0 = S.shear_wave(n, m=m, amplitude=1.5)
    u = u0.copy()
    for _ in range(7):
        u = O.step_wray3(u, h, nu, dt)
    lam = -4 * math.sin(m * h[1] / 2) ** 2 / h[1] ** 2
    np.testing.assert_allclose(u, _r3(nu * lam * dt) ** 7 * u0, atol=1e-13)


def _torch_ops(h, d, nu, shape):
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

    n = tuple(reversed(shape))
    lam = torch.zeros(shape, dtype=torch.float64)
    for a in range(d):
        k = torch.arange(n[a], dtype=torch.float64)
        shp = [1] * d
        shp[d - 1 - a] = n[a]
        lam = lam - (4 * torch.sin(math.pi * k / n[a]) ** 2 / h[a] ** 2).reshape(shp)
    lam[(0,) * d] = 1.0

    def P(u):
        p = torch.real(torch.fft.ifftn(torch.fft.fftn(div(u)) / lam))
        return u - grad(p)

    return F, P


def _torch_tableau_step(u0, h, nu, dt):
    """Explicit projected Runge-Kutta in Butcher form: u_i = P(u0 + dt sum_j a_ij F_j)."""
    A, b = _tableau()
    F, P = _torch_ops(h, u0.shape[0], nu, u0.shape[1:])
    fs = []
    for i in range(3):
        if i == 0:
            ui = u0
        else:
            ui = P(u0 + dt * sum(float(A[i][j]) * fs[j] for j in range(i)))
        fs.append(F(ui))
    return P(u0 + dt * sum(float(b[j]) * fs[j] for j in range(3)))


@pytest.mark.parametrize("n", [(8, 6), (4, 6, 5)])
def test_step_and_vjp_against_tableau_autograd_and_fd(n):
    h = S.spacing(n)
    nu, dt = 0.05, 0.05
    u0 = S.turbulence_ic(n, seed=1, k0=2)
    ubar = S.random_field(n, 22)
    t = torch.tensor(u0, requires_grad=True)
    out = _torch_tableau_step(t, h, nu, dt)
    np.testing.assert_allclose(O.step_wray3(u0, h, nu, dt), out.detach().numpy(), atol=1e-13)
    (out * torch.tensor(ubar)).sum().backward()
    g = O.step_wray3_vjp(u0, ubar, h, nu, dt)
    np.testing.assert_allclose(g, t.grad.numpy(), atol=1e-12 * np.abs(g).max())
    for seed in (30, 31):
        v = S.random_field(n, seed)
        fd = _dot(ubar, (O.step_wray3(u0 + 1e-4 * v, h, nu, dt) - O.step_wray3(u0 - 1e-4 * v, h, nu, dt)) / 2e-4)
        assert abs(fd - _dot(g, v)) < 1e-7 * np.abs(g * v).sum()


def test_third_order_convergence_nonlinear():
    """Error at fixed time against a fine RK4 reference falls by ~2^3 per halving of dt."""
    n = (12, 10)
    h = S.spacing(n)
    nu, T = 0.01, 0.4
    u0 = S.turbulence_ic(n, seed=5, k0=2)
    ref = u0.copy()
    for _ in range(400):
        ref = O.step_rk4(ref, h, nu, T / 400)
    errs = []
    for m in (10, 20, 40):
        u = u0.copy()
        for _ in range(m):
            u = O.step_wray3(u, h, nu, T / m)
        errs.append(np.linalg.norm(u - ref))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 6.5 < r1 < 9.5 and 6.5 < r2 < 9.5, errs


def test_wray3_step_is_solenoidal_and_dissipative():
    n = (12, 10, 8)
    h = S.spacing(n)
    u = S.turbulence_ic(n, seed=4, k0=2)
    e0 = O.kinetic_energy(u)
    u1 = O.step_wray3(u, h, 0.01, 1e-2)
    assert np.abs(O.divergence(u1, h)).max() < 1e-12 / min(h)
    assert O.kinetic_energy(u1) < e0
