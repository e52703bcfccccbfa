"""The Smagorinsky eddy-viscosity closure on the GPU (ins_eddy_*, and coupled
to the right-hand side, RK4 / Wray3 steps and their pullbacks) against the
float64 oracle: float64 within 1e-12 element-wise, the FP32 mode within 1e-5
relative L2 after one step."""
import math

import numpy as np
import pytest
import torch

import oracle as O
import oracle.eddy as E
import synth as S
from tests.gpu_util import dev, f32, host, l2_rel, max_rel

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
GRIDS = [(8, 6), (64, 10), (70, 9, 5), (16, 12, 20), (6, 840, 6), (140, 10, 9)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _lengths(n):
    return [2 * math.pi * (1.0, 1.3, 0.8)[a] for a in range(len(n))]


def _solver(n, nu=0.0, precision="fp64", lengths=None, cs=0.17, delta=None):
    from paper_2604_18536_amd import Solver

    hi = lengths if lengths is not None else [2 * math.pi] * len(n)
    s = Solver(n, nu=nu, precision=precision, hi=hi)
    s.set_eddy(cs, delta)
    return s


@pytest.mark.parametrize("n", GRIDS)
def test_eddy_forward_and_backward_fp64(n):
    L = _lengths(n)
    h = tuple(L[a] / n[a] for a in range(len(n)))
    s = _solver(n, lengths=L)
    u = S.random_field(n, 50)
    mbar = S.random_field(n, 51)
    assert max_rel(host(s.eddy_forward(dev(u))), E.smagorinsky(u, h)) < TOL64
    assert max_rel(host(s.eddy_backward(dev(u), dev(mbar))), E.smagorinsky_vjp(u, mbar, h)) < TOL64


def test_explicit_filter_width_and_energy_dissipation():
    n = (16, 12, 20)
    h = S.spacing(n)
    s = _solver(n, cs=0.3, delta=0.25)
    u = S.turbulence_ic(n, seed=52, k0=3)
    m = host(s.eddy_forward(dev(u)))
    assert max_rel(m, E.smagorinsky(u, h, 0.3, 0.25)) < TOL64
    assert float(np.sum(u * m)) < 0


@pytest.mark.parametrize("n", [(16, 12), (16, 12, 20)])
def test_rhs_step_and_pullbacks_with_eddy_fp64(n):
    nu, dt = 0.01, 5e-3
    h = S.spacing(n)
    s = _solver(n, nu)
    u0 = S.turbulence_ic(n, seed=53, k0=2)
    ubar = S.random_field(n, 54)

    def rhs_fn(v):
        return E.rhs_with_smagorinsky(v, h, nu)

    def rhs_vjp_fn(v, fb):
        return E.rhs_vjp_with_smagorinsky(v, fb, h, nu)

    assert max_rel(host(s.rhs(dev(u0))), rhs_fn(u0)) < TOL64
    assert max_rel(host(s.rhs_vjp(dev(u0), dev(ubar))), rhs_vjp_fn(u0, ubar)) < TOL64
    assert max_rel(host(s.step(dev(u0), dt)), O.step_rk4(u0, h, nu, dt, rhs_fn=rhs_fn)) < TOL64
    g = host(s.step_vjp(dev(u0), dev(ubar), dt))
    assert max_rel(g, O.step_rk4_vjp(u0, ubar, h, nu, dt, rhs_fn=rhs_fn, rhs_vjp_fn=rhs_vjp_fn)) < TOL64
    assert max_rel(host(s.step(dev(u0), dt, scheme="wray3")), O.step_wray3(u0, h, nu, dt, rhs_fn=rhs_fn)) < TOL64
    g3 = host(s.step_vjp(dev(u0), dev(ubar), dt, scheme="wray3"))
    assert max_rel(g3, O.step_wray3_vjp(u0, ubar, h, nu, dt, rhs_fn=rhs_fn, rhs_vjp_fn=rhs_vjp_fn)) < TOL64


def test_eddy_fp32_mode():
    n = (32, 16, 12)
    nu, dt = 0.01, 5e-3
    h = S.spacing(n)
    s = _solver(n, nu, precision="fp32")
    u0 = f32(S.turbulence_ic(n, seed=55, k0=2))
    ubar = f32(S.random_field(n, 56))

    def rhs_fn(v):
        return E.rhs_with_smagorinsky(v, h, nu)

    def rhs_vjp_fn(v, fb):
        return E.rhs_vjp_with_smagorinsky(v, fb, h, nu)

    u1 = host(s.step(dev(u0, torch.float32), dt))
    assert l2_rel(u1, O.step_rk4(u0, h, nu, dt, rhs_fn=rhs_fn)) < 1e-5
    g = host(s.step_vjp(dev(u0, torch.float32), dev(ubar, torch.float32), dt))
    assert l2_rel(g, O.step_rk4_vjp(u0, ubar, h, nu, dt, rhs_fn=rhs_fn, rhs_vjp_fn=rhs_vjp_fn)) < 1e-5


def test_set_and_clear():
    n = (16, 12, 20)
    nu = 0.02
    h = S.spacing(n)
    s = _solver(n, nu)
    u = S.turbulence_ic(n, seed=57, k0=2)
    f_eddy = host(s.rhs(dev(u)))
    s.set_closure(None)  # clears only a learned closure
    assert np.array_equal(host(s.rhs(dev(u))), f_eddy)
    s.set_eddy(0.0)
    assert max_rel(host(s.rhs(dev(u))), O.rhs(u, h, nu)) < TOL64
    from paper_2604_18536_amd import _lib

    with pytest.raises(RuntimeError):
        s.eddy_forward(dev(u))
    with pytest.raises(RuntimeError):
        s.set_eddy(-1.0)
    assert _lib is not None
