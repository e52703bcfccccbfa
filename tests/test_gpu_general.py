"""Grids stretched along every direction on the GPU (ins_set_faces; Sec. 2.5
non-uniform grids, App. B kernels with the widths of each direction) against
the stretched-grid oracle (oracle/stretched.py) with the same faces: periodic
in every direction (the setting of the paper's Taylor-Green convergence
study on a tanh grid, Sec. 7) and the channel with stretched x and z.

Bars: stencils and their pullbacks 1e-12 element-wise (max |gpu - ref| /
max |ref|); anything with a pressure solve 1e-10: the GPU runs CG to
rtol = 1e-14, the oracle solves exactly (sparse LU), and on these grids the
oracle's own CG at that rtol lands within 4e-14 of the exact solution (the
error is bounded by kappa(A) rtol); CG iterates after a fixed number of
iterations 1e-11; the FP32 mode 1e-5 relative L2 after one step. Grids
include ragged tiles (n_x = 70, 30; n_y = 9, 5) and a batch of two; x is
geometric (asymmetric: the periodic wrap joins the widest and the narrowest
cell), y and z tanh.
"""
import math

import numpy as np
import pytest
import torch

import synth as S
from oracle.stretched import StretchedGrid
from tests.gpu_util import dev, f32, host, l2_rel, max_rel

pytestmark = pytest.mark.gpu

GRIDS = [(70, 9), (24, 14, 6), (30, 5, 7)]
TOL_OP = 1e-12
TOL_SOLVE = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _geometric(n, s, lo, hi):
    i = np.arange(n + 1)
    return lo + (hi - lo) * (1.0 - s ** i) / (1.0 - s ** n)


def _box(n, walls):
    return S.channel_box(n) if walls else ([0.0] * len(n), [2 * math.pi] * len(n))


def _faces(n, walls):
    lo, hi = _box(n, walls)
    f = [_geometric(n[0], 1.04, lo[0], hi[0]), S.tanh_faces(n[1], lo[1], hi[1], 1.2)]
    if len(n) == 3:
        f.append(S.tanh_faces(n[2], lo[2], hi[2], 1.0))
    return f


def _solver(n, walls, nu=0.0, precision="fp64", batch=1, rtol=1e-14):
    from paper_2604_18536_amd import Solver

    lo, hi = _box(n, walls)
    s = Solver(n, nu=nu, precision=precision, batch=batch, lo=lo, hi=hi, bc="walls" if walls else "periodic")
    for a, f in enumerate(_faces(n, walls)):
        s.set_faces(a, f)
    s.cg_set(rtol=rtol, maxiter=20000, check_every=16)
    return s


def _field(n, walls, seed):
    return S.channel_random(n, seed) if walls else S.random_field(n, seed)


def _wall_face(u, n):
    return u[1].take([n[1] - 1], axis=len(n) - 2)


CASES = [(n, w) for w in (False, True) for n in GRIDS]


@pytest.mark.parametrize("n,walls", CASES)
def test_stencils_and_their_pullbacks(n, walls):
    nu = 0.03
    s = _solver(n, walls, nu)
    g = StretchedGrid(_faces(n, walls), walls)
    u, fb = _field(n, walls, 1), _field(n, walls, 3)
    p = S.random_scalar(n, 2)
    assert s.pressure == "cg"
    assert max_rel(host(s.rhs(dev(u))), g.rhs(u, nu)) < TOL_OP
    assert max_rel(host(s.divergence(dev(u))), g.divergence(u)) < TOL_OP
    assert max_rel(host(s.gradient(dev(p))), g.gradient(p)) < TOL_OP
    assert max_rel(host(s.rhs_vjp(dev(u), dev(fb))), g.rhs_vjp(u, fb, nu)) < TOL_OP
    assert max_rel(host(s.divergence_vjp(dev(p))), g.divergence_vjp(p)) < TOL_OP
    assert max_rel(host(s.gradient_vjp(dev(fb))), g.gradient_vjp(fb)) < TOL_OP
    if walls:
        assert np.abs(_wall_face(host(s.rhs(dev(u))), n)).max() == 0.0


@pytest.mark.parametrize("n,walls", CASES)
def test_poisson_projection_and_their_pullbacks(n, walls):
    s = _solver(n, walls)
    g = StretchedGrid(_faces(n, walls), walls)
    r = S.random_scalar(n, 4)
    p = host(s.poisson_solve(dev(r)))
    assert max_rel(p, g.poisson_solve(r)) < TOL_SOLVE
    it, rel = s.cg_info()
    assert 0 < it < 20000 and rel <= 1e-14
    u = _field(n, walls, 5)
    Pu = host(s.project(dev(u)))
    assert max_rel(Pu, g.project(u)[0]) < TOL_SOLVE
    assert np.abs(g.divergence(Pu)).max() < 1e-10 * np.abs(g.divergence(u)).max()
    assert max_rel(host(s.poisson_solve_vjp(dev(r))), g.poisson_solve_vjp(r)) < TOL_SOLVE
    assert max_rel(host(s.project_vjp(dev(u))), g.project_vjp(u)) < TOL_SOLVE


@pytest.mark.parametrize("n,walls", [((24, 14, 6), False), ((70, 9), True)])
def test_cg_iterates_match_the_oracle_cg(n, walls):
    s = _solver(n, walls)
    g = StretchedGrid(_faces(n, walls), walls)
    r = S.random_scalar(n, 7)
    for k in (1, 2, 7):
        s.cg_set(rtol=0.0, maxiter=k, check_every=0)
        x = host(s.poisson_solve(dev(r)))
        xo, ito, _ = g.cg_solve(r, rtol=0.0, maxiter=k)
        assert ito == k and s.cg_info()[0] == k
        assert max_rel(x, xo) < 1e-11


@pytest.mark.parametrize("n,walls", CASES)
@pytest.mark.parametrize("scheme", ["rk4", "wray3"])
def test_steps_and_pullbacks(n, walls, scheme):
    nu, dt = 0.02, 5e-3
    s = _solver(n, walls, nu)
    g = StretchedGrid(_faces(n, walls), walls)
    u0 = g.project(_field(n, walls, 10))[0]
    ubar = _field(n, walls, 11)
    step = g.step_rk4 if scheme == "rk4" else g.step_wray3
    vjp = g.step_rk4_vjp if scheme == "rk4" else g.step_wray3_vjp
    u1 = host(s.step(dev(u0), dt, scheme=scheme))
    assert max_rel(u1, step(u0, nu, dt)) < TOL_SOLVE
    gr = host(s.step_vjp(dev(u0), dev(ubar), dt, scheme=scheme))
    assert max_rel(gr, vjp(u0, ubar, nu, dt)) < TOL_SOLVE
    if walls:
        assert np.abs(_wall_face(u1, n)).max() == 0.0 and np.abs(_wall_face(gr, n)).max() == 0.0


def test_batch_in_place_and_fp32():
    n, walls = (24, 14, 6), False
    nu, dt = 0.02, 5e-3
    g = StretchedGrid(_faces(n, walls), walls)
    us = np.stack([g.project(_field(n, walls, 12 + b))[0] for b in range(2)])
    s2 = _solver(n, walls, nu, batch=2)
    u = dev(us)
    s2.step(u, dt, out=u)  # in place
    for b in range(2):
        assert max_rel(host(u[b]), g.step_rk4(us[b], nu, dt)) < TOL_SOLVE
    s32 = _solver(n, walls, nu, precision="fp32", rtol=1e-12)
    u32 = f32(us[0])
    assert l2_rel(host(s32.step(dev(u32, torch.float32), dt)), g.step_rk4(u32, nu, dt)) < 1e-5


def _tg(g, nu, t):
    fx, fy = g.faces
    cx, cy = 0.5 * (fx[:-1] + fx[1:]), 0.5 * (fy[:-1] + fy[1:])
    x1, y1 = np.meshgrid(fx[1:], cy)
    x2, y2 = np.meshgrid(cx, fy[1:])
    e = math.exp(-2 * nu * t)
    return np.stack([np.sin(x1) * np.cos(y1) * e, -np.cos(x2) * np.sin(y2) * e])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_taylor_green_converges_at_second_order_on_a_tanh_grid(precision):
    """The convergence study of Sec. 7 on the tanh grid: the 2D Taylor-Green
    vortex at t = 1 (nu = 0.01, RK4 with dt = 0.02) on N x N periodic tanh
    grids (gamma = 1.5), CG pressure solve; the velocity error against
    exp(-2 nu t) falls at second order in FP64 and FP32 (the FP32 plateau lies
    below these errors, as the paper observes on the non-uniform grid)."""
    from paper_2604_18536_amd import Solver

    nu, dt, T = 0.01, 0.02, 1.0
    dtype = torch.float64 if precision == "fp64" else torch.float32
    errs = []
    for N in (16, 32, 64):
        f = S.tanh_faces(N, 0.0, 2 * math.pi, 1.5)
        g = StretchedGrid([f, f])
        s = Solver((N, N), nu=nu, precision=precision)
        s.set_faces(0, f)
        s.set_faces(1, f)
        s.cg_set(rtol=1e-12, maxiter=20000, check_every=16)
        u = dev(g.project(_tg(g, nu, 0.0))[0], dtype)
        for _ in range(int(round(T / dt))):
            s.step(u, dt, out=u)
        ex = _tg(g, nu, T)
        om = g.volumes_u()
        errs.append(math.sqrt(np.sum(om * (host(u) - ex) ** 2) / np.sum(om * ex ** 2)))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) > 1.9, (errs, orders)


def test_errors_and_refusals():
    from paper_2604_18536_amd import Solver, _lib

    n = (16, 8)
    s = Solver(n)
    f = np.linspace(0.0, 2 * math.pi, n[0] + 1)
    with pytest.raises(ValueError):
        s.set_faces(2, f)
    bad = f.copy()
    bad[3] = bad[2]
    with pytest.raises(_lib.InsError) as e:
        s.set_faces(0, bad)
    assert e.value.status == _lib.INS_ERR_INVALID
    s.set_faces(0, S.tanh_faces(n[0], 0.0, 2 * math.pi, 1.0))
    assert s.pressure == "cg"
    with pytest.raises(_lib.InsError) as e:
        s.set_pressure("fft")
    assert e.value.status == _lib.INS_ERR_UNSUPPORTED
    with pytest.raises(_lib.InsError) as e:
        s.set_eddy(0.17)
    assert e.value.status == _lib.INS_ERR_UNSUPPORTED
    s.close()
