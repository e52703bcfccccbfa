"""Differentiation through the solver on the GPU: autograd wrappers over the
hand-written pullbacks, checkpointed unrolls, and the differentiable-rollout
workload (2D decaying turbulence 256^2, FP32, 50 steps, checkpoint every 10)
checked against float64 finite differences."""
import math

import numpy as np
import pytest
import torch

import oracle as O
import synth as S
from tests.gpu_util import dev, host, max_rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _solver(n, nu, precision="fp64"):
    from paper_2604_18536_amd import Solver

    return Solver(n, nu=nu, precision=precision)


def test_step_function_backward_is_the_library_pullback():
    from paper_2604_18536_amd import autograd as A

    n, nu, dt = (16, 12, 10), 0.02, 5e-3
    s = _solver(n, nu)
    u0 = dev(S.turbulence_ic(n, seed=1, k0=2)).requires_grad_(True)
    ubar = dev(S.random_field(n, 2))
    out = A.step(s, u0, dt)
    (out * ubar).sum().backward()
    ref = O.step_rk4_vjp(host(u0), host(ubar), S.spacing(n), nu, dt)
    assert max_rel(host(u0.grad), ref) < 1e-12


def test_rhs_and_project_functions():
    from paper_2604_18536_amd import autograd as A

    n, nu = (12, 10, 8), 0.03
    s = _solver(n, nu)
    u = dev(S.random_field(n, 3)).requires_grad_(True)
    fbar = dev(S.random_field(n, 4))
    (A.rhs(s, u) * fbar).sum().backward()
    assert max_rel(host(u.grad), O.rhs_vjp(host(u), host(fbar), S.spacing(n), nu)) < 1e-12
    v = dev(S.random_field(n, 5)).requires_grad_(True)
    (A.project(s, v) * fbar).sum().backward()
    assert max_rel(host(v.grad), O.project_vjp(host(fbar), S.spacing(n))) < 1e-12


@pytest.mark.parametrize("every", [1, 3, 5, 12])
def test_checkpointed_rollout_gradient_matches_oracle(every):
    from paper_2604_18536_amd import autograd as A

    n, nu, dt, steps = (32, 32), 5e-3, 2e-2, 12
    h = S.spacing(n)
    u0 = S.turbulence_ic(n, seed=5, k0=4)
    refs = [S.turbulence_ic(n, seed=100 + s, k0=4) * 0.9 for s in range(steps)]
    s = _solver(n, nu)
    x = dev(u0).requires_grad_(True)
    loss = A.rollout_loss(s, x, dt, [dev(r) for r in refs], checkpoint_every=every)
    loss.backward()
    lv = float(loss.detach())
    assert abs(lv - O.rollout_loss(u0, refs, h, nu, dt)) < 1e-12 * lv
    assert max_rel(host(x.grad), O.rollout_loss_grad(u0, refs, h, nu, dt)) < 1e-11


def _directions(s, n, seeds):
    out = []
    for sd in seeds:
        v = dev(S.random_field(n, sd))
        v = s.project(v)
        v = v / v.pow(2).mean().sqrt()
        out.append(v)
    return out


def test_differentiable_rollout_256_fp32_against_fp64_finite_differences():
    """2D decaying turbulence 256^2 (k0 = 4, nu = 5e-4), 50 RK4 steps of dt = 2e-3,
    loss = MSE to the trajectory from a seeded perturbed initial field, backward
    through the pullback kernels with a checkpoint every 10 steps; 16 directions."""
    from paper_2604_18536_amd import autograd as A

    n, nu, dt, steps = (256, 256), 5e-4, 2e-3, 50
    s64 = _solver(n, nu, "fp64")
    s32 = _solver(n, nu, "fp32")
    u0 = s64.project(dev(S.turbulence_ic(n, seed=1, k0=4)))
    xi = dev(S.random_field(n, 2))
    ur = s64.project(u0 + 1e-2 * xi)
    refs = []
    with torch.no_grad():
        for _ in range(steps):
            ur = s64.step(ur, dt)
            refs.append(ur.clone())

    def loss64(u):
        with torch.no_grad():
            return float(A.rollout_loss(s64, u, dt, refs, checkpoint_every=steps))

    x64 = u0.clone().requires_grad_(True)
    A.rollout_loss(s64, x64, dt, refs, checkpoint_every=10).backward()
    x32 = u0.float().clone().requires_grad_(True)
    A.rollout_loss(s32, x32, dt, [r.float() for r in refs], checkpoint_every=10).backward()
    eps = 1e-5
    fd, d64, d32 = [], [], []
    for v in _directions(s64, n, range(100, 116)):
        fd.append((loss64(u0 + eps * v) - loss64(u0 - eps * v)) / (2 * eps))
        d64.append(float((x64.grad * v).sum()))
        d32.append(float((x32.grad.double() * v).sum()))
    fd, d64, d32 = map(np.array, (fd, d64, d32))
    scale = np.sqrt(np.mean(fd ** 2))
    assert np.abs(d64 - fd).max() < 1e-7 * scale
    assert np.abs(d32 - fd).max() < 1e-3 * scale
