"""Channel body force on the GPU (the forcing term of F; the channel of Sec. 6 is
driven by f = (1, 0, 0)) against the channel oracle with the same force.

Bars as for the channel without force: the right-hand side 1e-12 element-wise,
steps and their pullbacks 1e-11 with the direct pressure solve (1e-10 with CG at
rtol 1e-14); the discrete Poiseuille profile (solved on the host from the 1D
tridiagonal system of the diffusion) is a fixed point of the GPU step to 1e-12
of its maximum, on uniform and tanh y.
"""
import numpy as np
import pytest
import torch

import oracle.walls as W
import synth as S
from tests.gpu_util import dev, host, max_rel
from tests.test_oracle_force import _box, _field, _poiseuille

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _solver(n, nu, faces=None, pressure="fft", force=None):
    from paper_2604_18536_amd import Solver

    lo, hi = S.channel_box(n)
    s = Solver(n, nu=nu, lo=lo, hi=hi, bc="walls", pressure=pressure)
    if faces is not None:
        s.set_y_faces(faces)
    s.cg_set(rtol=1e-14, maxiter=20000, check_every=16)
    if force is not None:
        s.set_body_force(force)
    return s


@pytest.mark.parametrize("gamma", [0.0, 1.4])
@pytest.mark.parametrize("n", [(70, 9), (24, 13, 6), (16, 12, 20)])
@pytest.mark.parametrize("pressure", ["fft", "cg"])
def test_rhs_steps_and_pullbacks_with_force(n, gamma, pressure):
    nu, dt = 0.02, 5e-3
    h, faces = _box(n, gamma)
    f = (1.0, -0.4, 0.3)[: len(n)]
    s = _solver(n, nu, faces if gamma else None, pressure, f)
    tol = 1e-11 if pressure == "fft" else 1e-10
    u = S.channel_random(n, 1)
    assert max_rel(host(s.rhs(dev(u))), W.rhs(u, h, nu, force=f)) < 1e-12
    u0 = W.project(S.channel_ic(n, 2), h)[0]
    ubar = S.channel_random(n, 3)
    for scheme, step, vjp in (("rk4", W.step_rk4, W.step_rk4_vjp), ("wray3", W.step_wray3, W.step_wray3_vjp)):
        u1 = host(s.step(dev(u0), dt, scheme=scheme))
        assert max_rel(u1, step(u0, h, nu, dt, force=f)) < tol
        g = host(s.step_vjp(dev(u0), dev(ubar), dt, scheme=scheme))
        assert max_rel(g, vjp(u0, ubar, h, nu, dt, force=f)) < tol


@pytest.mark.parametrize("gamma", [0.0, 1.4])
@pytest.mark.parametrize("n", [(8, 10), (6, 9, 4), (32, 48, 8)])
def test_poiseuille_fixed_point(n, gamma):
    nu, fx, dt = 0.05, 1.0, 2e-3
    h, faces = _box(n, gamma)
    prof, _ = _poiseuille(faces, nu, fx)
    u = _field(n, prof)
    s = _solver(n, nu, faces if gamma else None, "fft", (fx, 0.0, 0.0)[: len(n)])
    t = dev(u)
    for _ in range(5):
        s.step(t, dt, out=t)
    assert np.abs(host(t) - u).max() < 1e-12 * np.abs(u).max()


def test_force_setting():
    from paper_2604_18536_amd import Solver

    n = (16, 12, 8)
    s = _solver(n, 0.01)
    with pytest.raises(ValueError):
        s.set_body_force((1.0, 0.0))
    with pytest.raises(RuntimeError, match="INS_ERR_INVALID"):
        s.set_body_force((float("nan"), 0.0, 0.0))
    u = dev(S.channel_random(n, 5))
    f0 = s.rhs(u)
    s.set_body_force((0.5, 0.0, -2.0))
    f1 = s.rhs(u)
    d = host(f1 - f0)
    assert np.allclose(d[0], 0.5, rtol=0, atol=1e-12) and np.allclose(d[2], -2.0, rtol=0, atol=1e-12)
    assert np.abs(d[1]).max() == 0.0
    p = Solver(n, 0.01)
    with pytest.raises(RuntimeError, match="INS_ERR_UNSUPPORTED"):
        p.set_body_force((1.0, 0.0, 0.0))


def test_fp32_mode_with_force():
    from paper_2604_18536_amd import Solver

    n = (24, 13, 6)
    nu, dt = 0.02, 5e-3
    h, faces = _box(n, 1.4)
    f = (1.0, 0.0, -0.5)
    lo, hi = S.channel_box(n)
    s = Solver(n, nu=nu, precision="fp32", lo=lo, hi=hi, bc="walls")
    s.set_y_faces(faces)
    s.set_body_force(f)
    u0 = np.asarray(W.project(S.channel_ic(n, 6), h)[0], dtype=np.float32).astype(np.float64)
    u1 = host(s.step(dev(u0, torch.float32), dt))
    ref = W.step_rk4(u0, h, nu, dt, force=f)
    assert np.linalg.norm(u1 - ref) / np.linalg.norm(ref) < 1e-5


@pytest.mark.parametrize("pressure", ["fft", "cg"])
def test_forced_trajectory_on_a_tanh_grid(pressure):
    """20 RK4 steps of the forced channel (f = (1, 0, 0), tanh y) against the oracle's
    trajectory, compared every 5 steps: float64 rounding stays at the solve's level."""
    n = (16, 12, 8)
    nu, dt = 0.02, 5e-3
    h, faces = _box(n, 1.4)
    f = (1.0, 0.0, 0.0)
    s = _solver(n, nu, faces, pressure, f)
    u = W.project(S.channel_ic(n, 30, bulk=2.0, noise=0.3), h)[0]
    t = dev(u)
    for k in range(1, 21):
        u = W.step_rk4(u, h, nu, dt, force=f)
        s.step(t, dt, out=t)
        if k % 5 == 0:
            assert max_rel(host(t), u) < 1e-10, k
