"""Recorded HIP graphs of time steps replay exactly the eager steps: several
replays, with eager library work and host synchronisation between them, each
compared bit for bit with the same number of eager steps."""
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


@pytest.mark.parametrize("n,precision,scheme", [((64, 64), "fp64", "rk4"), ((48, 40), "fp32", "wray3"),
                                                ((32, 24, 20), "fp64", "rk4")])
def test_graph_replays_match_eager_steps(n, precision, scheme):
    from paper_2604_18536_amd import Solver
    from paper_2604_18536_amd.graphs import StepGraph

    dt, k = 2e-3, 7
    s = Solver(n, nu=0.01, precision=precision)
    dtype = torch.float64 if precision == "fp64" else torch.float32
    u0 = dev(S.turbulence_ic(n, seed=3, k0=2), dtype)
    ug = u0.clone()
    g = StepGraph(s, ug, dt, k, scheme=scheme)
    ue = u0.clone()
    for rep in range(3):
        g.replay()
        for _ in range(k):
            s.step(ue, dt, out=ue, scheme=scheme)
        torch.cuda.synchronize()
        assert torch.equal(ug, ue), rep
        s.stats(ue)  # eager work between replays
    assert np.isfinite(ug.double().cpu().numpy()).all()


@pytest.mark.parametrize("pressure", ["fft", "cg"])
def test_channel_graph_replays_match_eager_steps(pressure):
    """Forced channel on a tanh grid: the direct solve makes no host reads, and CG with
    check_every = 0 launches a fixed number of iterations, so both capture."""
    from paper_2604_18536_amd import Solver
    from paper_2604_18536_amd.graphs import StepGraph

    n, dt, k = (24, 20, 12), 2e-3, 3
    lo, hi = S.channel_box(n)
    s = Solver(n, nu=0.02, lo=lo, hi=hi, bc="walls", pressure=pressure)
    s.set_y_faces(S.tanh_faces(n[1], lo[1], hi[1], 1.4))
    s.set_body_force((1.0, 0.0, 0.0))
    s.cg_set(rtol=0.0, maxiter=40, check_every=0)
    u0 = dev(S.channel_ic(n, 4))
    s.project(u0, out=u0)
    ug = u0.clone()
    g = StepGraph(s, ug, dt, k)
    ue = u0.clone()
    for rep in range(3):
        g.replay()
        for _ in range(k):
            s.step(ue, dt, out=ue)
        torch.cuda.synchronize()
        assert torch.equal(ug, ue), rep
        s.stats(ue)
    assert np.isfinite(ug.double().cpu().numpy()).all()
