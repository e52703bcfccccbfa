"""The learned closure on the GPU (bfloat16 MFMA kernels) against the float64
closure oracle, alone and coupled to the right-hand side, the RK4 step and its
pullback.

Tolerance. Both sides round to bfloat16 at the same points, but the GPU forms
each pre-activation in float32 (a different summation order than the oracle's
float64), so a GELU output that lies within that float32 error of a bfloat16
rounding boundary can round the other way: a one-ulp (2^-8 relative) change of
one activation. Such flips are rare and propagate only through the following
layers' sums, so the comparison asks for a small mean error (1e-4 of the field
scale: flips, not systematic error) and bounds the worst entry at 2e-2 of the
scale.
"""
import numpy as np
import pytest
import torch

import oracle as O
import oracle.cnn as OC
import synth as S
from tests.gpu_util import dev, f32, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _solver(n, nu=0.01, precision="fp32", batch=1):
    from paper_2604_18536_amd import Solver

    return Solver(n, nu=nu, precision=precision, batch=batch)


def _close(got, ref, mean_tol=1e-4, max_tol=2e-2):
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    scale = np.abs(ref).max()
    err = np.abs(got - ref)
    return err.mean() / scale, err.max() / scale, (err.mean() / scale < mean_tol and err.max() / scale < max_tol)


def _theta(seed, scale=1.0):
    return OC.init_params(seed, scale)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("n,batch", [((32, 6, 5), 1), ((64, 8, 8), 2)])
def test_closure_forward(n, batch, precision):
    s = _solver(n, precision=precision, batch=batch)
    th = _theta(1)
    s.set_closure(torch.tensor(th, dtype=torch.float32, device="cuda"))
    dt = torch.float32 if precision == "fp32" else torch.float64
    u = np.stack([f32(S.turbulence_ic(n, seed=2 + b, k0=2)) for b in range(batch)])
    m = host(s.cnn_forward(dev(u, dt)))
    ref = OC.closure(u, th)
    mean_e, max_e, ok = _close(m, ref)
    assert ok, (mean_e, max_e)


def test_closure_backward():
    n = (32, 6, 5)
    s = _solver(n)
    th = _theta(3, 2.0)
    s.set_closure(torch.tensor(th, dtype=torch.float32, device="cuda"))
    u = f32(S.turbulence_ic(n, seed=4, k0=2))
    mbar = f32(S.random_field(n, 5))
    ub, tb = s.cnn_backward(dev(u, torch.float32), dev(mbar, torch.float32))
    ub_ref, tb_ref = OC.closure_vjp(u, th, mbar)
    e1 = _close(host(ub), ub_ref)
    assert e1[2], e1
    tb = host(tb)
    # per layer (each layer's gradient has its own scale)
    for lo, hi in [(0, 2592), (2592, 2624), (2624, 30272), (30272, 30304), (30304, 32896), (32896, 32899)]:
        e = _close(tb[lo:hi], tb_ref[lo:hi], 2e-3, 5e-2)
        assert e[2], (lo, hi, e)


def test_rhs_with_closure_and_detach():
    n = (32, 8, 6)
    nu = 0.02
    s = _solver(n, nu)
    th = _theta(6)
    u = f32(S.turbulence_ic(n, seed=7, k0=2))
    f0 = host(s.rhs(dev(u, torch.float32)))
    s.set_closure(torch.tensor(th, dtype=torch.float32, device="cuda"))
    f1 = host(s.rhs(dev(u, torch.float32)))
    ref = OC.rhs_with_closure(u, S.spacing(n), nu, th)
    e = _close(f1, ref, 1e-4, 5e-3)
    assert e[2], e
    s.set_closure(None)
    f2 = host(s.rhs(dev(u, torch.float32)))
    assert np.array_equal(f0, f2)


def test_step_with_closure_matches_oracle():
    n = (32, 8, 6)
    nu, dt = 0.02, 5e-3
    s = _solver(n, nu)
    th = _theta(8)
    s.set_closure(torch.tensor(th, dtype=torch.float32, device="cuda"))
    u0 = f32(S.turbulence_ic(n, seed=9, k0=2))
    u1 = host(s.step(dev(u0, torch.float32), dt))
    ref = OC.step_rk4_closure(u0, S.spacing(n), nu, dt, th)
    e = _close(u1, ref, 1e-6, 1e-4)
    assert e[2], e
    assert np.abs(O.divergence(u1, S.spacing(n))).max() < 1e-4


def test_step_vjp_with_closure_matches_oracle():
    n = (32, 8, 6)
    nu, dt = 0.02, 5e-3
    s = _solver(n, nu)
    th = _theta(10, 2.0)
    s.set_closure(torch.tensor(th, dtype=torch.float32, device="cuda"))
    u0 = f32(S.turbulence_ic(n, seed=11, k0=2))
    ubar = f32(S.random_field(n, 12))
    s.closure_grad()  # reset the accumulator
    g = host(s.step_vjp(dev(u0, torch.float32), dev(ubar, torch.float32), dt))
    tb = host(s.closure_grad())
    g_ref, tb_ref = OC.step_rk4_closure_vjp(u0, ubar, S.spacing(n), nu, dt, th)
    e = _close(g, g_ref, 1e-5, 1e-3)
    assert e[2], e
    for lo, hi in [(0, 2592), (2624, 30272), (30304, 32896)]:
        el = _close(tb[lo:hi], tb_ref[lo:hi], 5e-3, 1e-1)
        assert el[2], (lo, hi, el)
    # the accumulator was reset by the read
    assert not host(s.closure_grad()).any()
