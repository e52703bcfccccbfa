"""Channel on a stretched y grid (tanh faces, Sec. 2.5 non-uniform grids) on the
GPU against the channel oracle with the same face coordinates.

Bars as for the uniform channel: stencils and their pullbacks 1e-12
element-wise (max |gpu - ref| / max |ref|); anything with a pressure solve
1e-10 (CG stopped at rtol = 1e-14 against the oracle's exact sparse-LU
solution, error bounded by kappa(A) rtol with kappa < 1e3 here); CG iterates
after a fixed number of iterations 1e-11; FP32 mode 1e-5 relative L2.
"""
import numpy as np
import pytest
import torch

import oracle.walls as W
import synth as S
from tests.gpu_util import dev, f32, host, l2_rel, max_rel

pytestmark = pytest.mark.gpu

GRIDS = [(70, 9), (24, 13, 6), (16, 12, 20)]
TOL_OP = 1e-12
TOL_SOLVE = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _faces(n, gamma=1.4):
    lo, hi = S.channel_box(n)
    return S.tanh_faces(n[1], lo[1], hi[1], gamma)


def _h(n, gamma=1.4):
    lo, hi = S.channel_box(n)
    h = list(S.spacing(n, lo, hi))
    h[1] = _faces(n, gamma)
    return tuple(h)


def _solver(n, nu=0.0, precision="fp64", batch=1, rtol=1e-14, gamma=1.4):
    from paper_2604_18536_amd import Solver

    lo, hi = S.channel_box(n)
    s = Solver(n, nu=nu, precision=precision, batch=batch, lo=lo, hi=hi, bc="walls", pressure="cg")
    s.set_y_faces(_faces(n, gamma))
    s.cg_set(rtol=rtol, maxiter=20000, check_every=16)
    return s


def _wall_face(u, n):
    return u[1].take([n[1] - 1], axis=len(n) - 2)


@pytest.mark.parametrize("n", GRIDS)
def test_stencils(n):
    nu = 0.03
    s = _solver(n, nu)
    h = _h(n)
    u = S.channel_random(n, 1)
    p = S.random_scalar(n, 2)
    fbar = S.channel_random(n, 3)
    assert max_rel(host(s.rhs(dev(u))), W.rhs(u, h, nu)) < TOL_OP
    assert max_rel(host(s.divergence(dev(u))), W.divergence(u, h)) < TOL_OP
    assert max_rel(host(s.gradient(dev(p))), W.gradient(p, h)) < TOL_OP
    assert max_rel(host(s.rhs_vjp(dev(u), dev(fbar))), W.rhs_vjp(u, fbar, h, nu)) < TOL_OP
    assert max_rel(host(s.divergence_vjp(dev(p))), W.divergence_vjp(p, h)) < TOL_OP
    assert max_rel(host(s.gradient_vjp(dev(fbar))), W.gradient_vjp(fbar, h)) < TOL_OP


@pytest.mark.parametrize("n", GRIDS)
def test_solve_projection_and_their_pullbacks(n):
    s = _solver(n)
    h = _h(n)
    r = S.random_scalar(n, 4)
    p = host(s.poisson_solve(dev(r)))
    assert max_rel(p - p.mean(), W.poisson_solve(r, h)) < TOL_SOLVE
    assert max_rel(host(s.poisson_solve_vjp(dev(r))), W.poisson_solve_vjp(r, h)) < TOL_SOLVE
    u = S.channel_ic(n, 5) + 0.3 * S.channel_random(n, 6)
    Pu = host(s.project(dev(u)))
    assert max_rel(Pu, W.project(u, h)[0]) < TOL_SOLVE
    assert np.abs(_wall_face(Pu, n)).max() == 0.0
    g = host(s.project_vjp(dev(u)))
    assert max_rel(g, W.project_vjp(u, h)) < TOL_SOLVE
    assert np.abs(_wall_face(g, n)).max() == 0.0


@pytest.mark.parametrize("n", [(24, 13, 6), (70, 9)])
def test_cg_iterates_match_the_oracle_cg(n):
    s = _solver(n)
    h = _h(n)
    r = S.random_scalar(n, 7)
    for k in (1, 3, 7):
        s.cg_set(rtol=0.0, maxiter=k, check_every=0)
        x = host(s.poisson_solve(dev(r)))
        xo, ito, _ = W.cg_solve(r, h, rtol=0.0, maxiter=k)
        assert ito == k and s.cg_info()[0] == k
        assert max_rel(x, xo) < 1e-11
    s.cg_set(rtol=1e-8, maxiter=5000, check_every=16)
    s.poisson_solve(dev(r))
    it, rel = s.cg_info()
    assert abs(it - W.cg_solve(r, h, rtol=1e-8)[1]) <= 1 and rel <= 1e-8


@pytest.mark.parametrize("n", GRIDS)
@pytest.mark.parametrize("scheme", ["rk4", "wray3"])
def test_steps_and_pullbacks(n, scheme):
    nu, dt = 0.02, 5e-3
    h = _h(n)
    s = _solver(n, nu)
    u0 = W.project(S.channel_ic(n, 10), h)[0]
    ubar = S.channel_random(n, 11)
    step = W.step_rk4 if scheme == "rk4" else W.step_wray3
    vjp = W.step_rk4_vjp if scheme == "rk4" else W.step_wray3_vjp
    u1 = host(s.step(dev(u0), dt, scheme=scheme))
    assert max_rel(u1, step(u0, h, nu, dt)) < TOL_SOLVE
    assert np.abs(_wall_face(u1, n)).max() == 0.0
    g = host(s.step_vjp(dev(u0), dev(ubar), dt, scheme=scheme))
    assert max_rel(g, vjp(u0, ubar, h, nu, dt)) < TOL_SOLVE


def test_fp32_batch_and_kept_stages():
    n = (24, 13, 6)
    nu, dt = 0.02, 5e-3
    h = _h(n)
    us = np.stack([f32(W.project(S.channel_ic(n, 12 + b), h)[0]) for b in range(2)])
    s = _solver(n, nu, precision="fp32", batch=2, rtol=1e-12)
    u1 = host(s.step(dev(us, torch.float32), dt))
    for b in range(2):
        assert l2_rel(u1[b], W.step_rk4(us[b], h, nu, dt)) < 1e-5
    s64 = _solver(n, nu, rtol=1e-12)
    s64b = _solver(n, nu, batch=2, rtol=1e-12)
    ub = dev(np.stack([S.channel_random(n, 14), S.channel_random(n, 15)]))
    u0 = dev(us)
    gb = s64b.step_vjp(u0, ub, dt)
    kept = s64b.stage_buffers("rk4")
    assert torch.equal(s64b.step(u0, dt), s64b.step(u0, dt, keep=kept))
    assert torch.equal(gb, s64b.step_vjp(u0, ub, dt, kept=kept))
    for b in range(2):
        assert torch.equal(s64.step_vjp(u0[b].contiguous(), ub[b].contiguous(), dt), gb[b])


def test_face_checks():
    from paper_2604_18536_amd import Solver

    n = (16, 12, 20)
    s = _solver(n)
    bad = _faces(n).copy()
    bad[3] = bad[2]
    with pytest.raises(RuntimeError, match="INS_ERR_INVALID"):
        s.set_y_faces(bad)
    with pytest.raises(ValueError):
        s.set_y_faces(bad[:-1])
    p = Solver(n, 0.01)
    with pytest.raises(RuntimeError, match="INS_ERR_UNSUPPORTED"):
        p.set_y_faces(_faces(n))
