"""Parity of the HIP path (through the C ABI) with the float64 oracle.

Bar: float64 results within 1e-12 of the oracle element-wise (max |gpu - ref| /
max |ref|); the FP32-stencil mode within the bounds stated per test. Grids span
several 64x4 tiles with ragged tails, odd and mixed-radix FFT lengths (radix
2, 3, 4, 5, 7, 8; 840 = 8*7*5*3), thin grids with one long axis, 2D and 3D,
and batches.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
import synth as S
from tests.gpu_util import dev, f32, host, l2_rel, max_rel

pytestmark = pytest.mark.gpu

TOL64 = 1e-12

GRIDS = [
    (8, 6),
    (10, 14),
    (64, 64),
    (6, 840),
    (8, 6, 10),
    (140, 10, 9),
    (70, 9, 5),
    (840, 6, 6),
    (6, 840, 6),
    (6, 6, 840),
    (16, 12, 20),
]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_18536_amd import _lib

    _lib.load()


def _solver(n, nu=0.0, precision="fp64", batch=1, lengths=None):
    from paper_2604_18536_amd import Solver

    hi = lengths if lengths is not None else [2 * math.pi] * len(n)
    return Solver(n, nu=nu, precision=precision, batch=batch, hi=hi)


def _lengths(n):
    return [2 * math.pi * (1.0, 1.3, 0.8)[a] for a in range(len(n))]


def _h(n):
    L = _lengths(n)
    return tuple(L[a] / n[a] for a in range(len(n)))


@pytest.mark.parametrize("n", GRIDS)
def test_rhs_fp64(n):
    nu = 0.07
    s = _solver(n, nu, lengths=_lengths(n))
    u = S.random_field(n, 1)
    f = host(s.rhs(dev(u)))
    assert max_rel(f, O.rhs(u, _h(n), nu)) < TOL64


@pytest.mark.parametrize("n", GRIDS)
def test_divergence_and_gradient_fp64(n):
    s = _solver(n, lengths=_lengths(n))
    u = S.random_field(n, 2)
    p = S.random_scalar(n, 3)
    assert max_rel(host(s.divergence(dev(u))), O.divergence(u, _h(n))) < TOL64
    assert max_rel(host(s.gradient(dev(p))), O.gradient(p, _h(n))) < TOL64


@pytest.mark.parametrize("n", GRIDS)
def test_poisson_fp64(n):
    s = _solver(n, lengths=_lengths(n))
    r = S.random_scalar(n, 4)
    p = host(s.poisson_solve(dev(r)))
    assert max_rel(p, O.poisson_solve(r, _h(n))) < TOL64


@pytest.mark.parametrize("n", GRIDS)
def test_project_fp64(n):
    s = _solver(n, lengths=_lengths(n))
    u = S.random_field(n, 5)
    pout = s.new_scalar()[0] if s.batch == 1 else s.new_scalar()
    pu = s.project(dev(u), p_out=pout)
    ref, pref = O.project(u, _h(n))
    assert max_rel(host(pu), ref) < TOL64
    assert max_rel(host(pout), pref) < TOL64
    _, _, maxdiv, finite = s.stats(pu)
    assert finite and maxdiv < 1e-11 * np.abs(u).max() / min(_h(n))


@pytest.mark.parametrize("n", GRIDS)
def test_step_fp64(n):
    nu, dt = 0.02, 5e-3
    s = _solver(n, nu)
    u0 = S.turbulence_ic(n, seed=6, k0=2)
    u1 = host(s.step(dev(u0), dt))
    assert max_rel(u1, O.step_rk4(u0, S.spacing(n), nu, dt)) < TOL64


def test_step_in_place_matches_out_of_place():
    n = (16, 12, 20)
    s = _solver(n, 0.01)
    u0 = dev(S.turbulence_ic(n, seed=7, k0=2))
    out = s.step(u0, 1e-2)
    u_in = u0.clone()
    s.step(u_in, 1e-2, out=u_in)
    assert torch.equal(out, u_in)


@pytest.mark.parametrize("n", GRIDS)
def test_pullbacks_fp64(n):
    nu = 0.05
    h = _h(n)
    s = _solver(n, nu, lengths=_lengths(n))
    u, fbar = S.random_field(n, 8), S.random_field(n, 9)
    rbar = S.random_scalar(n, 10)
    assert max_rel(host(s.rhs_vjp(dev(u), dev(fbar))), O.rhs_vjp(u, fbar, h, nu)) < TOL64
    assert max_rel(host(s.divergence_vjp(dev(rbar))), O.divergence_vjp(rbar, h)) < TOL64
    assert max_rel(host(s.gradient_vjp(dev(fbar))), O.gradient_vjp(fbar, h)) < TOL64
    assert max_rel(host(s.poisson_solve_vjp(dev(rbar))), O.poisson_solve_vjp(rbar, h)) < TOL64
    assert max_rel(host(s.project_vjp(dev(fbar))), O.project_vjp(fbar, h)) < TOL64


@pytest.mark.parametrize("n", GRIDS)
def test_step_vjp_fp64(n):
    nu, dt = 0.02, 5e-3
    s = _solver(n, nu)
    u0 = S.turbulence_ic(n, seed=11, k0=2)
    ubar = S.random_field(n, 12)
    g = host(s.step_vjp(dev(u0), dev(ubar), dt))
    assert max_rel(g, O.step_rk4_vjp(u0, ubar, S.spacing(n), nu, dt)) < TOL64


def test_batch_fields_are_independent():
    n = (16, 12, 10)
    nu, dt = 0.03, 1e-2
    s = _solver(n, nu, batch=3)
    us = np.stack([S.turbulence_ic(n, seed=20 + b, k0=2) for b in range(3)])
    out = host(s.step(dev(us), dt))
    rhs = host(s.rhs(dev(us)))
    ubar = np.stack([S.random_field(n, 30 + b) for b in range(3)])
    g = host(s.step_vjp(dev(us), dev(ubar), dt))
    for b in range(3):
        assert max_rel(out[b], O.step_rk4(us[b], S.spacing(n), nu, dt)) < TOL64
        assert max_rel(rhs[b], O.rhs(us[b], S.spacing(n), nu)) < TOL64
        assert max_rel(g[b], O.step_rk4_vjp(us[b], ubar[b], S.spacing(n), nu, dt)) < TOL64


def test_taylor_green_64_fp64_closed_form():
    """2D TG, 64^2, nu = 0.01, dt = 1e-3, 100 steps: discrete closed form and analytic decay."""
    nn, nu, dt, steps = 64, 0.01, 1e-3, 100
    s = _solver((nn, nn), nu)
    u0 = S.taylor_green_2d(nn)
    u = dev(u0)
    for _ in range(steps):
        s.step(u, dt, out=u)
    h = 2 * math.pi / nn
    z = nu * (-8 * math.sin(h / 2) ** 2 / h ** 2) * dt
    exact = (1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24) ** steps * u0
    assert l2_rel(host(u), exact) < 1e-13
    assert l2_rel(host(u), math.exp(-2 * nu * steps * dt) * u0) < 5e-6


# ------------------------------------------------------------------ FP32 mode
def _fp32_rhs_bound(u, h, nu):
    """Rounding bound of the float32 stencil: per direction b the diffusion difference
    carries ~4 |u| eps nu / h_b^2 and the flux difference ~4 |u|^2 eps / h_b (eps = 2^-24);
    a factor 4 covers the accumulation of the d terms."""
    eps = 2.0 ** -24
    U = np.abs(u).max()
    return 4 * eps * sum(4 * nu * U / hb ** 2 + 4 * U * U / hb for hb in h)


@pytest.mark.parametrize("n", [(16, 12, 20), (140, 10, 9), (64, 64)])
def test_rhs_fp32(n):
    nu = 0.05
    h = S.spacing(n)
    s = _solver(n, nu, precision="fp32")
    u = f32(S.turbulence_ic(n, seed=13, k0=2))
    f = host(s.rhs(dev(u, torch.float32)))
    ref = O.rhs(u, h, nu)
    assert np.abs(f - ref).max() < _fp32_rhs_bound(u, h, nu)
    assert max_rel(f, ref) < 1e-5


@pytest.mark.parametrize("n", [(16, 12, 20), (64, 64)])
def test_projection_fp32_mode_is_float64_inside(n):
    s = _solver(n, precision="fp32")
    u = f32(S.random_field(n, 14))
    pu = host(s.project(dev(u, torch.float32)))
    ref = O.project(u, S.spacing(n))[0]
    # only the final rounding to float32 separates the two
    assert max_rel(pu, ref) < 1.5e-7
    d = O.divergence(pu, S.spacing(n))
    assert np.abs(d).max() < 1e-5 * np.abs(u).max() / min(S.spacing(n))


@pytest.mark.parametrize("n", [(16, 12, 20), (64, 64)])
def test_step_fp32_within_1e5_of_fp64_oracle(n):
    nu, dt = 0.02, 5e-3
    s = _solver(n, nu, precision="fp32")
    u0 = f32(S.turbulence_ic(n, seed=15, k0=2))
    u1 = host(s.step(dev(u0, torch.float32), dt))
    assert l2_rel(u1, O.step_rk4(u0, S.spacing(n), nu, dt)) < 1e-5


@pytest.mark.parametrize("n", [(16, 12, 20), (64, 64)])
def test_step_vjp_fp32(n):
    nu, dt = 0.02, 5e-3
    s = _solver(n, nu, precision="fp32")
    u0 = f32(S.turbulence_ic(n, seed=16, k0=2))
    ubar = f32(S.random_field(n, 17))
    g = host(s.step_vjp(dev(u0, torch.float32), dev(ubar, torch.float32), dt))
    assert l2_rel(g, O.step_rk4_vjp(u0, ubar, S.spacing(n), nu, dt)) < 1e-5


def test_kernels_are_deterministic():
    n = (140, 10, 9)
    s = _solver(n, 0.01)
    u = dev(S.turbulence_ic(n, seed=18, k0=2))
    a = s.step(u, 1e-2).clone()
    b = s.step(u, 1e-2)
    assert torch.equal(a, b)
    ubar = dev(S.random_field(n, 19))
    assert torch.equal(s.step_vjp(u, ubar, 1e-2).clone(), s.step_vjp(u, ubar, 1e-2))


def test_abi_errors_on_gpu():
    from paper_2604_18536_amd import InsError

    s = _solver((8, 6, 10))
    with pytest.raises(InsError):
        s.step(dev(S.random_field((8, 6, 10), 1)), -1.0)
    u = dev(S.random_field((8, 6, 10), 1))
    with pytest.raises(InsError):
        s.step_vjp(u, u, 1e-3, out=u)
    with pytest.raises(ValueError):
        s.rhs(dev(S.random_field((8, 6, 12), 1)))
    with pytest.raises(TypeError):
        s.rhs(dev(S.random_field((8, 6, 10), 1), torch.float32))


# ------------------------------------------------- full size, bench launch shape
def test_full_size_256_step_fp64():
    """The benchmark workload itself: one float64 step of the 256^3 turbulence field vs the oracle."""
    n = (256, 256, 256)
    nu, dt = 1.0 / 1600.0, 1e-3
    u0 = S.turbulence_ic(n, seed=0, k0=4.0)
    s = _solver(n, nu)
    u1 = host(s.step(dev(u0), dt))
    s.close()
    assert max_rel(u1, O.step_rk4(u0, S.spacing(n), nu, dt)) < TOL64


def test_full_size_256_step_vjp_adjoint_identity():
    """<ubar, J v> = <J^T ubar, v> at 256^3, J v by central differences of GPU steps (float64)."""
    n = (256, 256, 256)
    nu, dt, eps = 1.0 / 1600.0, 1e-3, 1e-4
    s = _solver(n, nu)
    u0 = dev(S.turbulence_ic(n, seed=0, k0=4.0))
    v = dev(S.turbulence_ic(n, seed=1, k0=8.0))
    ubar = dev(S.random_field(n, 2))
    g = s.step_vjp(u0, ubar, dt)
    jv = (s.step(u0 + eps * v, dt) - s.step(u0 - eps * v, dt)) / (2 * eps)
    lhs = float((ubar * jv).sum())
    rhs = float((g * v).sum())
    s.close()
    assert abs(lhs - rhs) < 1e-9 * float((ubar.abs() * jv.abs()).sum())


def test_full_size_256_step_vjp_fp64():
    """The reverse z-march kernels in the benchmark's launch shape: the 256^3
    float64 step pullback against the oracle's, element by element."""
    n = (256, 256, 256)
    nu, dt = 1.0 / 1600.0, 1e-3
    u0 = S.turbulence_ic(n, seed=0, k0=4.0)
    ubar = S.random_field(n, 2)
    s = _solver(n, nu)
    g = host(s.step_vjp(dev(u0), dev(ubar), dt))
    s.close()
    assert max_rel(g, O.step_rk4_vjp(u0, ubar, S.spacing(n), nu, dt)) < TOL64
