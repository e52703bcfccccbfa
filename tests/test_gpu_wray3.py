"""Wray's low-storage three-stage Runge-Kutta step on the GPU (ins_step_wray3
and its pullback) against the float64 oracle.

Bar: float64 within 1e-12 element-wise (max |gpu - ref| / max |ref|); the FP32
mode within 1e-5 relative L2 of the float64 oracle after one step, as for RK4.
The grids are those of the RK4 parity tests (ragged tiles, mixed-radix and
840-long axes, 2D and 3D).
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
import oracle.cnn as OC
import synth as S
from tests.gpu_util import dev, f32, host, l2_rel, max_rel
from tests.test_gpu_parity import GRIDS, TOL64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _solver(n, nu=0.0, precision="fp64", batch=1):
    from paper_2604_18536_amd import Solver

    return Solver(n, nu=nu, precision=precision, batch=batch)


@pytest.mark.parametrize("n", GRIDS)
def test_wray3_step_fp64(n):
    nu, dt = 0.02, 5e-3
    s = _solver(n, nu)
    u0 = S.turbulence_ic(n, seed=40, k0=2)
    u1 = host(s.step(dev(u0), dt, scheme="wray3"))
    assert max_rel(u1, O.step_wray3(u0, S.spacing(n), nu, dt)) < TOL64


@pytest.mark.parametrize("n", GRIDS)
def test_wray3_step_vjp_fp64(n):
    nu, dt = 0.02, 5e-3
    s = _solver(n, nu)
    u0 = S.turbulence_ic(n, seed=41, k0=2)
    ubar = S.random_field(n, 42)
    g = host(s.step_vjp(dev(u0), dev(ubar), dt, scheme="wray3"))
    assert max_rel(g, O.step_wray3_vjp(u0, ubar, S.spacing(n), nu, dt)) < TOL64


def test_wray3_in_place_and_batch():
    n = (16, 12, 10)
    nu, dt = 0.03, 1e-2
    s = _solver(n, nu, batch=2)
    us = np.stack([S.turbulence_ic(n, seed=43 + b, k0=2) for b in range(2)])
    u = dev(us)
    out = s.step(u, dt, scheme="wray3")
    s.step(u, dt, out=u, scheme="wray3")
    assert torch.equal(out, u)
    for b in range(2):
        assert max_rel(host(out)[b], O.step_wray3(us[b], S.spacing(n), nu, dt)) < TOL64


def test_wray3_taylor_green_64_closed_form():
    nn, nu, dt, steps = 64, 0.01, 1e-3, 100
    s = _solver((nn, nn), nu)
    u0 = S.taylor_green_2d(nn)
    u = dev(u0)
    for _ in range(steps):
        s.step(u, dt, out=u, scheme="wray3")
    h = 2 * math.pi / nn
    z = nu * (-8 * math.sin(h / 2) ** 2 / h ** 2) * dt
    exact = (1 + z + z * z / 2 + z ** 3 / 6) ** steps * u0
    assert l2_rel(host(u), exact) < 1e-13


@pytest.mark.parametrize("n", [(16, 12, 20), (64, 64)])
def test_wray3_fp32_mode(n):
    nu, dt = 0.02, 5e-3
    s = _solver(n, nu, precision="fp32")
    u0 = f32(S.turbulence_ic(n, seed=44, k0=2))
    ubar = f32(S.random_field(n, 45))
    h = S.spacing(n)
    u1 = host(s.step(dev(u0, torch.float32), dt, scheme="wray3"))
    assert l2_rel(u1, O.step_wray3(u0, h, nu, dt)) < 1e-5
    g = host(s.step_vjp(dev(u0, torch.float32), dev(ubar, torch.float32), dt, scheme="wray3"))
    assert l2_rel(g, O.step_wray3_vjp(u0, ubar, h, nu, dt)) < 1e-5


def test_wray3_with_closure():
    """du/dt = P(F + m_theta): step and input gradient against the oracle (the
    closure's bfloat16 roundings make the bar that of the closure tests)."""
    n = (32, 8, 6)
    nu, dt = 0.02, 5e-3
    h = S.spacing(n)
    s = _solver(n, nu, precision="fp32")
    th = OC.init_params(8)
    s.set_closure(torch.tensor(th, dtype=torch.float32, device="cuda"))
    u0 = f32(S.turbulence_ic(n, seed=46, k0=2))
    ubar = f32(S.random_field(n, 47))
    u1 = host(s.step(dev(u0, torch.float32), dt, scheme="wray3"))

    def rhs_fn(v):
        return OC.rhs_with_closure(v, h, nu, th)

    ref = O.step_wray3(u0, h, nu, dt, rhs_fn=rhs_fn)
    err = np.abs(u1 - ref)
    assert err.mean() / np.abs(ref).max() < 1e-6 and err.max() / np.abs(ref).max() < 1e-4

    def rhs_vjp_fn(v, fb):
        return O.rhs_vjp(v, fb, h, nu) + OC.closure_vjp(v, th, fb)[0]

    s.closure_grad()
    g = host(s.step_vjp(dev(u0, torch.float32), dev(ubar, torch.float32), dt, scheme="wray3"))
    gref = O.step_wray3_vjp(u0, ubar, h, nu, dt, rhs_fn=rhs_fn, rhs_vjp_fn=rhs_vjp_fn)
    err = np.abs(g - gref)
    assert err.mean() / np.abs(gref).max() < 1e-5 and err.max() / np.abs(gref).max() < 1e-3
    assert np.abs(host(s.closure_grad())).sum() > 0


def test_wray3_rollout_gradient_matches_oracle():
    """Checkpointed autograd rollout with scheme="wray3" against reverse accumulation with the oracle."""
    from paper_2604_18536_amd import autograd as A

    n = (16, 12)
    nu, dt, steps = 0.02, 1e-2, 6
    h = S.spacing(n)
    s = _solver(n, nu)
    u0 = S.turbulence_ic(n, seed=48, k0=2)
    refs = [S.turbulence_ic(n, seed=60 + k, k0=2) * 0.5 for k in range(steps)]
    t = dev(u0).requires_grad_(True)
    loss = A.rollout_loss(s, t, dt, [dev(r) for r in refs], checkpoint_every=4, scheme="wray3")
    loss.backward()
    # oracle: forward states, then reverse accumulation of d loss / d u0
    us = [u0]
    for k in range(steps):
        us.append(O.step_wray3(us[-1], h, nu, dt))
    m = u0.size
    val = sum(np.sum((us[k + 1] - refs[k]) ** 2) / m / steps for k in range(steps))
    assert abs(float(loss) - val) < 1e-12 * abs(val)
    g = np.zeros_like(u0)
    for k in range(steps - 1, -1, -1):
        g = g + 2.0 * (us[k + 1] - refs[k]) / m / steps
        g = O.step_wray3_vjp(us[k], g, h, nu, dt)
    assert max_rel(host(t.grad), g) < 1e-11
