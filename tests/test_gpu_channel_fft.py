"""Direct (FFT in x and z, tridiagonal along y) pressure solve of the channel
on the GPU against the channel oracle's sparse-LU solve of the augmented
system (Sec. 2.6.1 direct solver), uniform and stretched y.

Both sides solve the same discrete system exactly, so the bar is rounding:
1e-11 element-wise (max |gpu - ref| / max |ref|) for solves, projections,
steps and pullbacks; the (0, 0) mode's Neumann operator has a condition number
growing as n_y^2 (about 5e5 at n_y = 1100), so kappa * eps stays below 1e-10
and well-conditioned modes are at 1e-16. FP32 mode: 1e-5 relative L2 after one
step. Grids cover one to 64 segments per line (n_y = 9 .. 1100), ragged k_x
chunks (n_x = 70),
2D and 3D, and a batch of two. At the 256^3 size the benchmark runs, the
checks are properties the exact solve has at any size: D P u = 0 to
rounding, P P u = P u, and D G p = r - mean_w(r).
"""
import numpy as np
import pytest
import torch

import oracle.walls as W
import synth as S
from tests.gpu_util import dev, f32, host, l2_rel, max_rel

pytestmark = pytest.mark.gpu

TOL = 1e-11
GRIDS = [(70, 9), (24, 13, 6), (16, 12, 20), (40, 36, 10), (8, 300, 4), (6, 1100)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _faces(n, gamma):
    lo, hi = S.channel_box(n)
    return S.tanh_faces(n[1], lo[1], hi[1], gamma)


def _h(n, gamma):
    lo, hi = S.channel_box(n)
    h = list(S.spacing(n, lo, hi))
    if gamma:
        h[1] = _faces(n, gamma)
    return tuple(h)


def _solver(n, nu=0.0, precision="fp64", batch=1, gamma=0.0):
    from paper_2604_18536_amd import Solver

    lo, hi = S.channel_box(n)
    s = Solver(n, nu=nu, precision=precision, batch=batch, lo=lo, hi=hi, bc="walls", pressure="fft")
    if gamma:
        s.set_y_faces(_faces(n, gamma))
    assert s.pressure == "fft"
    return s


def _wall_face(u, n):
    return u[1].take([n[1] - 1], axis=len(n) - 2)


@pytest.mark.parametrize("gamma", [0.0, 1.4])
@pytest.mark.parametrize("n", GRIDS)
def test_solve_projection_and_pullbacks(n, gamma):
    s = _solver(n, gamma=gamma)
    h = _h(n, gamma)
    r = S.random_scalar(n, 4)
    p = host(s.poisson_solve(dev(r)))
    pref = W.poisson_solve(r, h)
    assert max_rel(p, pref) < TOL
    assert abs(p.mean()) < 1e-12 * np.abs(pref).max()
    assert max_rel(host(s.poisson_solve_vjp(dev(r))), W.poisson_solve_vjp(r, h)) < TOL
    u = S.channel_ic(n, 5) + 0.3 * S.channel_random(n, 6)
    Pu = host(s.project(dev(u)))
    assert max_rel(Pu, W.project(u, h)[0]) < TOL
    assert np.abs(_wall_face(Pu, n)).max() == 0.0
    g = host(s.project_vjp(dev(u)))
    assert max_rel(g, W.project_vjp(u, h)) < TOL
    assert np.abs(_wall_face(g, n)).max() == 0.0


@pytest.mark.parametrize("gamma", [0.0, 1.4])
@pytest.mark.parametrize("n", [(70, 9), (24, 13, 6), (16, 12, 20)])
@pytest.mark.parametrize("scheme", ["rk4", "wray3"])
def test_steps_and_pullbacks(n, gamma, scheme):
    nu, dt = 0.02, 5e-3
    h = _h(n, gamma)
    s = _solver(n, nu, gamma=gamma)
    u0 = W.project(S.channel_ic(n, 10), h)[0]
    ubar = S.channel_random(n, 11)
    step = W.step_rk4 if scheme == "rk4" else W.step_wray3
    vjp = W.step_rk4_vjp if scheme == "rk4" else W.step_wray3_vjp
    u1 = host(s.step(dev(u0), dt, scheme=scheme))
    assert max_rel(u1, step(u0, h, nu, dt)) < TOL
    assert np.abs(_wall_face(u1, n)).max() == 0.0
    g = host(s.step_vjp(dev(u0), dev(ubar), dt, scheme=scheme))
    assert max_rel(g, vjp(u0, ubar, h, nu, dt)) < TOL


def test_batch_equals_single_and_fp32():
    n = (24, 13, 6)
    nu, dt = 0.02, 5e-3
    h = _h(n, 1.4)
    r = np.stack([S.random_scalar(n, 8), S.random_scalar(n, 9)])
    s2 = _solver(n, batch=2, gamma=1.4)
    a = s2.poisson_solve(dev(r))
    s1 = _solver(n, gamma=1.4)
    for i in range(2):
        assert torch.equal(s1.poisson_solve(dev(r[i])), a[i])
    us = np.stack([f32(W.project(S.channel_ic(n, 12 + b), h)[0]) for b in range(2)])
    s32 = _solver(n, nu, precision="fp32", batch=2, gamma=1.4)
    u1 = host(s32.step(dev(us, torch.float32), dt))
    for b in range(2):
        assert l2_rel(u1[b], W.step_rk4(us[b], h, nu, dt)) < 1e-5
    # FP32 pullback: float32 stencils, float64 transposed solves (scaled divergence in the x pass)
    ubar = np.stack([f32(S.channel_random(n, 40 + b)) for b in range(2)])
    g = host(s32.step_vjp(dev(us, torch.float32), dev(ubar, torch.float32), dt))
    for b in range(2):
        assert l2_rel(g[b], W.step_rk4_vjp(us[b], ubar[b], h, nu, dt)) < 1e-5


def test_kept_stages_and_agreement_with_cg():
    n = (24, 13, 6)
    nu, dt = 0.02, 5e-3
    s = _solver(n, nu, gamma=1.4)
    u0 = dev(S.channel_ic(n, 15))
    ubar = dev(S.channel_random(n, 16))
    kept = s.stage_buffers("rk4")
    assert torch.equal(s.step(u0, dt), s.step(u0, dt, keep=kept))
    assert torch.equal(s.step_vjp(u0, ubar, dt), s.step_vjp(u0, ubar, dt, kept=kept))
    # the CG solver converges to the same step
    s.set_pressure("cg")
    s.cg_set(rtol=1e-14, maxiter=20000, check_every=16)
    assert s.pressure == "cg"
    ucg = s.step(u0, dt)
    s.set_pressure("fft")
    assert max_rel(host(s.step(u0, dt)), host(ucg)) < 1e-10


@pytest.mark.parametrize("n", [(4, 2), (4, 3), (4, 2, 2), (6, 3, 4), (8, 160), (6, 200, 4), (4, 1000), (6, 700, 4),
                               (4, 2048)])
def test_smallest_and_largest_channels(n):
    """n_y = 2, 3 (one segment of two or three rows per line, n_x = 4: two complex
    points per x row); n_y = 700 and 1000 (64 segments of up to 16 rows, 512-thread
    workgroups, the shape of the paper's 1024-row channel); n_y = 2048, the largest
    the direct solve takes (64 segments of 32 rows). The (0, 0) mode's uniform
    Neumann operator has condition number 1 / sin^2(pi / (2 n_y)); the bar is
    20 eps kappa, at least 1e-11."""
    s = _solver(n, gamma=0.0)
    h = _h(n, 0.0)
    kappa = 1.0 / np.sin(np.pi / (2 * n[1])) ** 2
    tol = max(1e-11, 20 * np.finfo(float).eps * kappa)
    r = S.random_scalar(n, 21)
    assert max_rel(host(s.poisson_solve(dev(r))), W.poisson_solve(r, h)) < tol
    assert max_rel(host(s.poisson_solve_vjp(dev(r))), W.poisson_solve_vjp(r, h)) < tol
    u = S.channel_random(n, 22)
    assert max_rel(host(s.project(dev(u))), W.project(u, h)[0]) < tol


def test_solver_choice():
    from paper_2604_18536_amd import Solver

    lo, hi = S.channel_box((33, 5, 7))
    s = Solver((33, 5, 7), 0.01, lo=lo, hi=hi, bc="walls")  # odd n_x: no real-to-complex FFT
    assert s.pressure == "cg"
    with pytest.raises(RuntimeError, match="INS_ERR_UNSUPPORTED"):
        s.set_pressure("fft")
    lo, hi = S.channel_box((22, 8, 8))
    s = Solver((22, 8, 8), 0.01, lo=lo, hi=hi, bc="walls")  # n_x / 2 = 11
    assert s.pressure == "cg"
    lo, hi = S.channel_box((4, 2049))
    s = Solver((4, 2049), 0.01, lo=lo, hi=hi, bc="walls")  # n_y above the direct solve's 2048
    assert s.pressure == "cg"
    lo, hi = S.channel_box((16, 8, 8))
    s = Solver((16, 8, 8), 0.01, lo=lo, hi=hi, bc="walls")
    assert s.pressure == "fft"
    s.set_pressure("cg")
    assert s.pressure == "cg"
    s.set_pressure("auto")
    assert s.pressure == "fft"
    p = Solver((16, 8, 8), 0.01)
    assert p.pressure == "fft"
    with pytest.raises(RuntimeError, match="INS_ERR_UNSUPPORTED"):
        p.set_pressure("cg")
    with pytest.raises(ValueError):
        p.set_pressure("lu")
    # the C entry points themselves: an unknown solver value, a null output
    from paper_2604_18536_amd import _lib

    lib = _lib.load()
    assert lib.ins_set_pressure_solver(s._ctx, 7) == _lib.INS_ERR_INVALID
    assert lib.ins_get_pressure_solver(s._ctx, None) == _lib.INS_ERR_INVALID
    assert s.pressure == "fft"  # unchanged by the rejected calls


@pytest.mark.parametrize("gamma", [0.0, 1.5])
def test_full_size_properties(gamma):
    """256^3 FP64 channel (the benchmarked size): exact-solve properties."""
    n = (256, 256, 256)
    s = _solver(n, 1e-3, gamma=gamma)
    torch.manual_seed(0)
    u = torch.randn(s.vel_shape[1:], dtype=torch.float64, device="cuda")
    u[1, :, n[1] - 1, :] = 0.0
    r0 = s.divergence(u)
    Pu = s.project(u)
    r1 = s.divergence(Pu)
    assert float(r1.abs().max()) < 1e-12 * float(r0.abs().max())
    PPu = s.project(Pu)
    assert float((PPu - Pu).abs().max()) < 1e-12 * float(Pu.abs().max())
    assert float(Pu[1, :, n[1] - 1, :].abs().max()) == 0.0
    # D G p = r - mean_w(r) for a random r
    r = torch.randn(s.scal_shape[1:], dtype=torch.float64, device="cuda")
    p = s.poisson_solve(r)
    res = s.divergence(s.gradient(p))
    if gamma:
        w = torch.tensor(np.diff(_faces(n, gamma)), dtype=torch.float64, device="cuda")
    else:
        w = torch.full((n[1],), 2.0 / n[1], dtype=torch.float64, device="cuda")
    wr = w.view(1, -1, 1)
    mean_w = float((r * wr).sum() / (wr.expand_as(r)).sum())
    assert float((res - (r - mean_w)).abs().max()) < 1e-10 * float(r.abs().max())
    assert abs(float(p.mean())) < 1e-12 * float(p.abs().max())


def test_random_shapes_sweep():
    """Seeded random channels (n_x from the FFT's sizes, any n_y in 2..70, 2D or 3D,
    uniform or tanh y, batch 1 or 2): solve, its transpose and the projection against
    the oracle. Bar: 20 eps kappa with kappa = the (0, 0) mode's condition number,
    bounded by (max width / min width) / sin^2(pi / (2 n_y)), and at least 1e-11."""
    from paper_2604_18536_amd import Solver

    rng = np.random.default_rng(2026)
    for _ in range(10):
        nx = int(rng.choice([4, 6, 10, 14, 16, 20, 28, 30, 42, 56]))
        ny = int(rng.integers(2, 71))
        three = bool(rng.integers(0, 2))
        n = (nx, ny, int(rng.choice([2, 3, 5, 7, 8, 12]))) if three else (nx, ny)
        gamma = float(rng.choice([0.0, rng.uniform(0.5, 2.0)]))
        batch = int(rng.integers(1, 3))
        lo, hi = S.channel_box(n)
        s = Solver(n, nu=0.0, batch=batch, lo=lo, hi=hi, bc="walls", pressure="fft")
        h = list(S.spacing(n, lo, hi))
        if gamma:
            f = S.tanh_faces(ny, lo[1], hi[1], gamma)
            s.set_y_faces(f)
            h[1] = f
            ratio = np.diff(f).max() / np.diff(f).min()
        else:
            ratio = 1.0
        h = tuple(h)
        kappa = ratio / np.sin(np.pi / (2 * ny)) ** 2
        tol = max(1e-11, 20 * np.finfo(float).eps * kappa)
        r = np.stack([S.random_scalar(n, 100 + b) for b in range(batch)])
        u = np.stack([S.channel_random(n, 200 + b) for b in range(batch)])
        p = host(s.poisson_solve(dev(r)))
        q = host(s.poisson_solve_vjp(dev(r)))
        Pu = host(s.project(dev(u)))
        for b in range(batch):
            case = (n, gamma, batch, b)
            assert max_rel(p[b], W.poisson_solve(r[b], h)) < tol, case
            assert max_rel(q[b], W.poisson_solve_vjp(r[b], h)) < tol, case
            assert max_rel(Pu[b], W.project(u[b], h)[0]) < tol, case
        s.close()
