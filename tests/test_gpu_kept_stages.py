"""Steps that keep their stage inputs (ins_step_save) and the pullback that
uses them (ins_step_vjp_saved) run the same kernels as the plain step and the
recomputing pullback: results must be identical, bit for bit, for RK4 and
Wray3, both precisions, 2D and 3D, batches and the eddy-viscosity closure; and
checkpointed autograd rollouts give the same gradient either way."""
import numpy as np
import pytest
import torch

import synth as S
from tests.gpu_util import dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("scheme", ["rk4", "wray3"])
@pytest.mark.parametrize("n,precision,batch,eddy", [((24, 20, 14), "fp64", 1, False), ((40, 30), "fp32", 2, False),
                                                    ((32, 16, 12), "fp32", 1, True), ((70, 9, 5), "fp64", 2, True)])
def test_kept_stages_match_recompute(scheme, n, precision, batch, eddy):
    from paper_2604_18536_amd import Solver

    s = Solver(n, nu=0.02, precision=precision, batch=batch)
    if eddy:
        s.set_eddy(0.17)
    dtype = torch.float64 if precision == "fp64" else torch.float32
    u0 = dev(np.stack([S.turbulence_ic(n, seed=70 + b, k0=2) for b in range(batch)]), dtype)
    ubar = dev(np.stack([S.random_field(n, 80 + b) for b in range(batch)]), dtype)
    dt = 5e-3
    kept = s.stage_buffers(scheme)
    a = s.step(u0, dt, scheme=scheme)
    b = s.step(u0, dt, scheme=scheme, keep=kept)
    assert torch.equal(a, b)
    ga = s.step_vjp(u0, ubar, dt, scheme=scheme)
    gb = s.step_vjp(u0, ubar, dt, scheme=scheme, kept=kept)
    assert torch.equal(ga, gb)


def test_rollout_gradient_with_kept_stages():
    from paper_2604_18536_amd import Solver
    from paper_2604_18536_amd import autograd as A

    n = (32, 24)
    s = Solver(n, nu=0.01)
    u0 = dev(S.turbulence_ic(n, seed=90, k0=2))
    refs = [dev(S.turbulence_ic(n, seed=91 + k, k0=2)) * 0.5 for k in range(8)]
    grads = []
    for keep in (False, True):
        t = u0.clone().requires_grad_(True)
        A.rollout_loss(s, t, 1e-2, refs, checkpoint_every=3, keep_stages=keep).backward()
        grads.append(t.grad.clone())
    assert torch.equal(grads[0], grads[1])


def test_kept_stage_buffers_are_checked():
    from paper_2604_18536_amd import Solver

    s = Solver((16, 12, 10))
    u = dev(S.turbulence_ic((16, 12, 10), seed=1, k0=2))
    stages, pstages = s.stage_buffers("wray3")
    with pytest.raises(ValueError):
        s.step(u, 1e-3, scheme="rk4", keep=(stages, pstages))  # two stages, RK4 needs three
