"""A-posteriori closure training on the GPU: the trajectory-loss gradient in the
closure parameters (autograd over the hand-written step pullback, checkpointed)
against the oracle, and a small end-to-end run (DNS 128^3 -> 4x face filter ->
LES 32^3) where the trained closure must beat the no-closure LES on a held-out
seed."""
import numpy as np
import pytest
import torch

import oracle.cnn as OC
import synth as S
from tests.gpu_util import dev, f32, host

pytestmark = pytest.mark.gpu

RANGES = [(0, 2592), (2592, 2624), (2624, 30272), (30272, 30304), (30304, 32896), (32896, 32899)]
FLIPS = 4.0


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_rollout_parameter_gradient_matches_oracle():
    """Checkpointed trajectory-loss gradient (float64 solver, bfloat16/float32
    closure): every parameter against the oracle within the closure's float32
    accumulation bounds summed over all its pullbacks (times 4 for flips, as in
    tests/test_gpu_closure.py); dL/du0 in the 2-norm chain of those bounds."""
    from paper_2604_18536_amd import Solver
    from paper_2604_18536_amd import autograd as A

    n, nu, dt, steps = (32, 8, 6), 0.02, 5e-3, 3
    h = S.spacing(n)
    th = OC.init_params(21, 2.0)
    th[2592:2624] = f32(0.05 * np.random.default_rng(1).standard_normal(32))
    u0 = f32(S.turbulence_ic(n, seed=22, k0=2))
    refs = [f32(S.turbulence_ic(n, seed=30 + s, k0=2)) for s in range(steps)]
    s = Solver(n, nu=nu, precision="fp64")
    theta = torch.tensor(th, dtype=torch.float32, device="cuda").requires_grad_(True)
    s.set_closure(theta.detach())
    x = dev(u0).requires_grad_(True)
    loss = A.rollout_loss(s, x, dt, [dev(r) for r in refs], checkpoint_every=2, theta=theta)
    loss.backward()
    pairs = []
    ub_ref, tb_ref = OC.rollout_loss_closure_grad(u0, refs, h, nu, dt, th, on_closure=lambda v, fb: pairs.append((v, fb)))
    assert len(pairs) == 4 * steps
    lref = OC.rollout_loss_closure(u0, refs, h, nu, dt, th)
    assert abs(float(loss.detach()) - lref) < 1e-6 * lref
    eth = np.zeros(OC.n_params())
    eub = 0.0
    for v, fb in pairs:
        b = OC.accumulation_bounds(v, th, fb)
        eth += b["theta"]
        eub += np.linalg.norm(b["ubar"])
    tb = host(theta.grad)
    eth = FLIPS * eth + 4 * steps * OC.U32 * np.abs(tb_ref) + 1e-12 * np.abs(tb_ref).max()
    for lo, hi in RANGES:
        err = np.abs(tb[lo:hi] - tb_ref[lo:hi])
        assert np.all(err <= eth[lo:hi]), (lo, hi, float(np.max(err / eth[lo:hi])))
    # each stage pullback grows a cotangent by at most 1 + dt |J| <= 1.2 (|J|_2 about 25 here)
    g = host(x.grad)
    bound = 1.2 ** (4 * steps) * FLIPS * eub + 1e-12 * np.abs(ub_ref).max()
    assert np.abs(g - ub_ref).max() <= bound, (np.abs(g - ub_ref).max(), bound)


def test_training_beats_no_closure_on_held_out_seed():
    from paper_2604_18536_amd import les

    nu, dt, every = 1.0 / 2000.0, 2.5e-3, 4
    data = [les.dns_snapshots(128, 4, sd, nu, dt, spinup=100, nsnap=40, every=every) for sd in (10, 11, 12)]
    dt_les = every * dt
    theta, hist = les.train(data[:2], nu, dt_les, iters=40, unroll=5, batch=2, lr=3e-3, seed=0, checkpoint_every=3)
    assert np.isfinite(hist).all()
    assert np.mean(hist[-8:]) < hist[0]
    windows = [(0, s0) for s0 in (0, 8, 16, 24, 32)]
    mse0 = les.rollout_mse(data[2:], None, nu, dt_les, windows, 5)
    mse1 = les.rollout_mse(data[2:], theta, nu, dt_les, windows, 5)
    assert mse1 < mse0, (mse1, mse0)
    e0, f0 = les.spectrum_error(data[2], None, nu, dt_les, 0, 30)
    e1, f1 = les.spectrum_error(data[2], theta, nu, dt_les, 0, 30)
    assert f0 and f1
    print(f"held-out MSE no closure {mse0:.4e} closure {mse1:.4e}; spectrum error {e0:.4f} -> {e1:.4f}")
