"""Accuracy of the FP32-stencil mode (float32 fields and stencils, float64
divergence/Poisson/projection) over long runs, against float64.

* 64^3 decaying turbulence (k0 = 4, nu = 1/1600, dt = 1e-3), 100 steps: GPU
  FP64 and GPU FP32 mode against the float64 CPU oracle run for the same steps.
* The benchmark trajectory, 256^3, 200 steps: FP32 mode against GPU FP64 (which
  matches the oracle step by step to 1e-12). Velocity error (relative L2) and
  kinetic-energy error are printed and bounded.
"""
import numpy as np
import pytest
import torch

import oracle as O
import synth as S
from tests.gpu_util import dev, f32, host, l2_rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _solver(n, nu, precision):
    from paper_2604_18536_amd import Solver

    return Solver(n, nu=nu, precision=precision)


def test_long_run_64_against_oracle():
    n, nu, dt, steps = (64, 64, 64), 1.0 / 1600.0, 1e-3, 100
    h = S.spacing(n)
    u0 = f32(S.turbulence_ic(n, seed=0, k0=4.0))
    ref = u0.copy()
    for _ in range(steps):
        ref = O.step_rk4(ref, h, nu, dt)
    s64, s32 = _solver(n, nu, "fp64"), _solver(n, nu, "fp32")
    a, b = dev(u0), dev(u0, torch.float32)
    for _ in range(steps):
        s64.step(a, dt, out=a)
        s32.step(b, dt, out=b)
    e64 = l2_rel(host(a), ref)
    e32 = l2_rel(host(b), ref)
    ke_ref = O.kinetic_energy(ref)
    dke32 = abs(O.kinetic_energy(host(b)) - ke_ref) / ke_ref
    print(f"64^3 x {steps}: FP64 rel L2 {e64:.2e}; FP32 mode rel L2 {e32:.2e}, KE rel {dke32:.2e}")
    assert e64 < 1e-11
    assert e32 < 1e-5 and dke32 < 1e-5


def test_benchmark_trajectory_256_fp32_vs_fp64():
    n, nu, dt, steps = (256, 256, 256), 1.0 / 1600.0, 1e-3, 200
    u0 = f32(S.turbulence_ic(n, seed=0, k0=4.0))
    s64, s32 = _solver(n, nu, "fp64"), _solver(n, nu, "fp32")
    a, b = dev(u0), dev(u0, torch.float32)
    errs = []
    for k in range(1, steps + 1):
        s64.step(a, dt, out=a)
        s32.step(b, dt, out=b)
        if k in (1, 10, 50, 100, 200):
            d = (b.double() - a)
            e = float(d.norm() / a.norm())
            ke64, ke32 = 0.5 * float((a * a).sum(0).mean()), 0.5 * float((b.double() ** 2).sum(0).mean())
            errs.append((k, e, abs(ke32 - ke64) / ke64))
    for k, e, dk in errs:
        print(f"256^3 step {k}: FP32 mode vs FP64 rel L2 {e:.2e}, KE rel {dk:.2e}")
    assert errs[0][1] < 1e-6  # one step
    assert errs[-1][1] < 1e-5 and errs[-1][2] < 1e-5  # 200 steps
    assert s64.stats(a)[3] and s32.stats(b)[3]
