"""The learned closure on the GPU (bfloat16 MFMA kernels, float32 sums)
against the float64 closure oracle: layer by layer on the kernels' own
operands, and coupled to the right-hand side, the RK4 step and its pullback.

Standalone closure (``test_closure_layers``): the library exports every
intermediate tensor of a forward + backward pass (ins_cnn_saved), and each
layer is compared element by element with the oracle's layer on the same
bfloat16 operands, within the float32 summation bound gamma_K sum |w||x|;
every bfloat16 activation and cotangent must equal the oracle's rounding
except where a flip is possible, and flips are counted
(``tests/closure_check.py``).

Inside the solver (no intermediates): the solver runs in float64, so the
closure's float32 sums are the only rounding above 1e-12, and the bound is
the oracle's per-evaluation accumulation bound (``accumulation_bounds``)
summed over every closure evaluation, times 4 for the rare flips (a flip
moves one bfloat16 operand by one step, which the layer test shows and counts)
and, where a stage's error reaches the result through the projection and
later stages, in the 2-norm (the projection has norm 1 in it).
"""
import numpy as np
import pytest
import torch

import oracle as O
import oracle.cnn as OC
import synth as S
from tests.closure_check import check_closure_layers
from tests.gpu_util import dev, f32, host

pytestmark = pytest.mark.gpu

RANGES = [(0, 2592), (2592, 2624), (2624, 30272), (30272, 30304), (30304, 32896), (32896, 32899)]
FLIPS = 4.0


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _solver(n, nu=0.01, precision="fp32", batch=1):
    from paper_2604_18536_amd import Solver

    return Solver(n, nu=nu, precision=precision, batch=batch)


def _theta(seed, scale=1.0):
    th = OC.init_params(seed, scale)
    rng = np.random.default_rng(seed + 500)
    for lo, hi in RANGES[1::2]:
        th[lo:hi] = f32(0.05 * rng.standard_normal(hi - lo))
    return th


def _layout(t, batch, n):
    """[cells][C] (channels-last, cells in field order) -> [B][C][nz][ny][nx] float64."""
    a = t.double().cpu().numpy()
    return a.reshape((batch,) + tuple(n[::-1]) + (a.shape[1],)).transpose(0, 4, 1, 2, 3).copy()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("n,batch", [((32, 6, 5), 1), ((64, 8, 8), 2)])
def test_closure_layers(n, batch, precision):
    s = _solver(n, precision=precision, batch=batch)
    th = _theta(1, 2.0)
    s.set_closure(torch.tensor(th, dtype=torch.float32, device="cuda"))
    dt = torch.float32 if precision == "fp32" else torch.float64
    u = np.stack([f32(S.turbulence_ic(n, seed=2 + b, k0=2)) for b in range(batch)])
    mbar = np.stack([f32(S.random_field(n, 20 + b)) for b in range(batch)])
    m_fwd = host(s.cnn_forward(dev(u, dt)))
    ub, tb = s.cnn_backward(dev(u, dt), dev(mbar, dt))
    t = {k: _layout(s.cnn_saved(w), batch, n)
         for w, k in enumerate(("x0", "z1", "a1", "z2", "a2", "gm", "gz2", "gz1"))}
    t["m"] = host(s.cnn_saved(8))
    # the forward-only call (no float32 pre-activations kept) gives the same m
    assert np.array_equal(m_fwd, t["m"])
    ff, fb = check_closure_layers(u, th, mbar, t, host(ub), host(tb).astype(np.float64))
    hidden = u.size // 3 * 32 * 2
    print(f"bfloat16 flips: forward {ff}, backward {fb} of {hidden} each")
    assert ff < 1e-3 * hidden and fb < 1e-3 * hidden
    # end to end against the oracle's own network: within the accumulation bound up to the flips
    acc = OC.accumulation_bounds(u, th, mbar)
    assert np.all(np.abs(t["m"] - OC.closure(u, th)) <= FLIPS * acc["m"])
    s.close()


def test_rhs_with_closure_and_detach():
    n = (32, 8, 6)
    nu = 0.02
    s = _solver(n, nu, precision="fp64")
    th = _theta(6)
    u = f32(S.turbulence_ic(n, seed=7, k0=2))
    f0 = host(s.rhs(dev(u)))
    s.set_closure(torch.tensor(th, dtype=torch.float32, device="cuda"))
    f1 = host(s.rhs(dev(u)))
    ref = OC.rhs_with_closure(u, S.spacing(n), nu, th)
    mbar = np.ones_like(u)
    bound = FLIPS * OC.accumulation_bounds(u, th, mbar)["m"] + 1e-12 * np.abs(ref).max()
    assert np.all(np.abs(f1 - ref) <= bound), np.max(np.abs(f1 - ref) / bound)
    s.set_closure(None)
    f2 = host(s.rhs(dev(u)))
    assert np.array_equal(f0, f2)


def test_step_with_closure_matches_oracle():
    n = (32, 8, 6)
    nu, dt = 0.02, 5e-3
    h = S.spacing(n)
    s = _solver(n, nu, precision="fp64")
    th = _theta(8)
    s.set_closure(torch.tensor(th, dtype=torch.float32, device="cuda"))
    u0 = f32(S.turbulence_ic(n, seed=9, k0=2))
    u1 = host(s.step(dev(u0), dt))
    stages = []

    def rhs(v):
        stages.append(v)
        return OC.rhs_with_closure(v, h, nu, th)

    ref = O.step_rk4(u0, h, nu, dt, rhs_fn=rhs)
    # each stage's closure error reaches u1 through dt * (RK weight <= 1) and the projection (2-norm 1)
    e2 = sum(np.linalg.norm(OC.accumulation_bounds(v, th, np.ones_like(v))["m"]) for v in stages)
    bound = FLIPS * dt * e2 + 1e-12 * np.abs(ref).max()
    assert np.abs(u1 - ref).max() <= bound, (np.abs(u1 - ref).max(), bound)
    assert np.abs(O.divergence(u1, h)).max() < 1e-12 * np.abs(u1).max() / min(h)


def _closure_pairs_bounds(pairs, th):
    """Sum of the accumulation bounds over the (stage velocity, cotangent) pairs at
    which the oracle pulled the closure back: theta element-wise, ubar in the 2-norm."""
    eth = np.zeros(OC.n_params())
    eub = 0.0
    for v, fb in pairs:
        b = OC.accumulation_bounds(v, th, fb)
        eth += b["theta"]
        eub += np.linalg.norm(b["ubar"])
    return eth, eub


def test_step_vjp_with_closure_matches_oracle():
    n = (32, 8, 6)
    nu, dt = 0.02, 5e-3
    h = S.spacing(n)
    s = _solver(n, nu, precision="fp64")
    th = _theta(10, 2.0)
    s.set_closure(torch.tensor(th, dtype=torch.float32, device="cuda"))
    u0 = f32(S.turbulence_ic(n, seed=11, k0=2))
    ubar = f32(S.random_field(n, 12))
    s.closure_grad()  # reset the accumulator
    g = host(s.step_vjp(dev(u0), dev(ubar), dt))
    tb = host(s.closure_grad())
    pairs = []
    g_ref, tb_ref = OC.step_rk4_closure_vjp(u0, ubar, h, nu, dt, th, on_closure=lambda v, fb: pairs.append((v, fb)))
    assert len(pairs) == 4
    eth, eub = _closure_pairs_bounds(pairs, th)
    # float32 accumulation of theta_bar over the four stages: one rounding per add
    eth = FLIPS * eth + 4 * OC.U32 * np.abs(tb_ref) + 1e-12 * np.abs(tb_ref).max()
    for lo, hi in RANGES:
        err = np.abs(tb[lo:hi] - tb_ref[lo:hi])
        assert np.all(err <= eth[lo:hi]), (lo, hi, float(np.max(err / eth[lo:hi])))
    # ubar: the closure's input-gradient errors travel back through the earlier
    # stages (each a contraction up to 1 + dt |J| <= 1.2 here) in the 2-norm
    bound = 1.2 ** 4 * FLIPS * eub + 1e-12 * np.abs(g_ref).max()
    assert np.abs(g - g_ref).max() <= bound, (np.abs(g - g_ref).max(), bound)
    # the accumulator was reset by the read
    assert not host(s.closure_grad()).any()
