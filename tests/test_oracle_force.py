"""Pins of the channel oracle's body force (the forcing term collected in F, App. A
momentum equation; the constant driving force of the channel, Sec. 6), by
routes other than its own array code:

* exact solution: with nu = 0 a uniform streamwise/spanwise flow has no
  convection and no diffusion, so one RK4 or Wray3 step adds exactly dt f_x and
  dt f_z; a wall-normal force is balanced by the pressure (a uniform u^y is not
  solenoidal between the walls) and leaves no trace;
* steady state: the discrete Poiseuille profile, solved here from a 1D
  tridiagonal system assembled directly from the face coordinates (wall ghosts
  mirror the first row with the opposite sign), makes the right-hand side
  vanish, so it is a fixed point of both steps, uniform and stretched y;
* consistency: on a uniform y it approaches the continuous parabola
  f y (L - y) / (2 nu) at second order;
* the force has no Jacobian: the step pullbacks with and without it differ
  only through the forward stages, checked by central differences.
"""
import numpy as np
import pytest

import oracle.walls as W
import synth as S


def _box(n, gamma=0.0):
    lo, hi = S.channel_box(n)
    h = list(S.spacing(n, lo, hi))
    faces = None
    if gamma:
        faces = S.tanh_faces(n[1], lo[1], hi[1], gamma)
        h[1] = faces
    else:
        faces = lo[1] + np.arange(n[1] + 1) * h[1]
    return tuple(h), faces


def _poiseuille(faces, nu, fx):
    """nu (Lap_y u)_j + fx = 0 for the cell-centred tangential profile, rows 0..n-1:
    Lap_y u_j = ((u_{j+1} - u_j) / d_j - (u_j - u_{j-1}) / d_{j-1}) / w_j, with the
    ghost rows u_{-1} = -u_0, u_n = -u_{n-1} at the distances d_{-1} = w_0, d_{n-1} = w_{n-1}."""
    n = len(faces) - 1
    w = np.diff(faces)
    c = 0.5 * (faces[:-1] + faces[1:])
    d = np.empty(n + 1)
    d[0], d[n] = w[0], w[-1]
    d[1:n] = np.diff(c)
    A = np.zeros((n, n))
    for j in range(n):
        lo, hi = 1.0 / d[j], 1.0 / d[j + 1]  # d[j] is d_{j-1}
        A[j, j] -= (lo + hi) / w[j]
        if j > 0:
            A[j, j - 1] += lo / w[j]
        else:
            A[j, j] -= lo / w[j]  # ghost -u_0
        if j < n - 1:
            A[j, j + 1] += hi / w[j]
        else:
            A[j, j] -= hi / w[j]  # ghost -u_{n-1}
    return np.linalg.solve(nu * A, -fx * np.ones(n)), c


def _field(n, prof):
    d = len(n)
    u = np.zeros((d,) + tuple(reversed(n)))
    sh = [1] * d
    sh[d - 2] = n[1]
    u[0] = prof.reshape(sh) * np.ones(tuple(reversed(n)))
    return u


@pytest.mark.parametrize("n", [(8, 6), (6, 5, 4)])
@pytest.mark.parametrize("scheme", ["rk4", "wray3"])
def test_uniform_flow_gains_exactly_dt_f(n, scheme):
    h, _ = _box(n)
    d = len(n)
    f = (0.7, -1.3, 0.4)[:d]
    u0 = np.zeros((d,) + tuple(reversed(n)))
    u0[0] = 1.5
    if d == 3:
        u0[2] = -0.25
    dt = 0.01
    step = W.step_rk4 if scheme == "rk4" else W.step_wray3
    u1 = step(u0, h, 0.0, dt, force=f)
    expect = u0.copy()
    expect[0] += dt * f[0]
    if d == 3:
        expect[2] += dt * f[2]
    np.testing.assert_allclose(u1, expect, rtol=0, atol=1e-14)


@pytest.mark.parametrize("gamma", [0.0, 1.4])
@pytest.mark.parametrize("n", [(8, 10), (6, 9, 4)])
def test_poiseuille_is_a_fixed_point(n, gamma):
    nu, fx, dt = 0.05, 1.0, 0.02
    h, faces = _box(n, gamma)
    prof, _ = _poiseuille(faces, nu, fx)
    u = _field(n, prof)
    f = (fx, 0.0, 0.0)[: len(n)]
    scale = np.abs(u).max()
    assert np.abs(W.rhs(u, h, nu, force=f)).max() < 1e-12 * scale / dt
    for step in (W.step_rk4, W.step_wray3):
        np.testing.assert_allclose(step(u, h, nu, dt, force=f), u, rtol=0, atol=1e-12 * scale)
    # without the force the profile decays
    assert np.abs(W.step_rk4(u, h, nu, dt) - u).max() > 1e-3 * scale


def test_poiseuille_converges_to_the_parabola():
    nu, fx, L = 0.1, 2.0, 2.0
    errs = []
    for ny in (16, 32, 64):
        faces = np.linspace(0.0, L, ny + 1)
        prof, c = _poiseuille(faces, nu, fx)
        exact = fx * c * (L - c) / (2 * nu)
        errs.append(np.abs(prof - exact).max() / np.abs(exact).max())
    assert errs[0] > errs[1] > errs[2]
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


def test_force_has_no_jacobian_in_the_pullbacks():
    n = (6, 7, 4)
    h, _ = _box(n, 1.4)
    nu, dt = 0.03, 0.01
    f = (0.8, 0.0, -0.3)
    u0 = W.project(S.channel_ic(n, 3), h)[0]
    ubar = S.channel_random(n, 4)
    v = W.project(S.channel_random(n, 5), h)[0]
    g = W.step_rk4_vjp(u0, ubar, h, nu, dt, force=f)
    eps = 1e-5
    fd = (W.step_rk4(u0 + eps * v, h, nu, dt, force=f) - W.step_rk4(u0 - eps * v, h, nu, dt, force=f)) / (2 * eps)
    lhs, rhs = float(np.sum(ubar * fd)), float(np.sum(g * v))
    assert abs(lhs - rhs) < 1e-8 * abs(lhs)
    # the force changes the forward stages, hence the pullback
    g0 = W.step_rk4_vjp(u0, ubar, h, nu, dt)
    assert np.abs(g - g0).max() > 1e-9 * np.abs(g).max()
