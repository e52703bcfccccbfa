"""LES data helpers on the GPU vs the oracle: face filter and energy spectrum."""
import numpy as np
import pytest
import torch

import oracle as O
import synth as S
from tests.gpu_util import dev, f32, host, max_rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _solver(n, precision="fp64", batch=1):
    from paper_2604_18536_amd import Solver

    return Solver(n, nu=0.01, precision=precision, batch=batch)


@pytest.mark.parametrize("n,f", [((16, 8), 4), ((8, 12, 16), 4), ((24, 12, 6), 2), ((64, 64, 64), 4)])
def test_face_filter(n, f):
    s = _solver(n)
    u = S.random_field(n, 3)
    uc = host(s.face_filter(dev(u), f))
    assert max_rel(uc, O.face_filter(u, f)) < 1e-14


def test_face_filter_keeps_solenoidal_fp32():
    n = (64, 32, 48)
    s = _solver(n, "fp32")
    u = f32(S.turbulence_ic(n, seed=4, k0=3))
    uc = host(s.face_filter(dev(u, torch.float32), 4))
    assert max_rel(uc, O.face_filter(u, 4)) < 2e-7
    nc = tuple(v // 4 for v in n)
    assert np.abs(O.divergence(uc, S.spacing(nc))).max() < 1e-5 * np.abs(uc).max() * max(nc)


@pytest.mark.parametrize("n", [(16, 16), (32, 24), (8, 12, 10), (24, 20, 14), (64, 64, 64)])
def test_energy_spectrum(n):
    s = _solver(n)
    u = S.turbulence_ic(n, seed=5, k0=3)
    e = host(s.energy_spectrum(dev(u)))
    ref = O.energy_spectrum(u)
    # the library sizes the shells for the longest axis; shells past the largest |k| stay empty
    assert len(e) >= len(ref) and not e[len(ref):].any()
    assert max_rel(e[:len(ref)], ref) < 1e-12
    assert abs(e.sum() - O.kinetic_energy(u)) < 1e-12


def test_energy_spectrum_batch_and_fp32():
    n = (16, 12, 10)
    s = _solver(n, "fp32", batch=2)
    us = np.stack([f32(S.turbulence_ic(n, seed=6 + b, k0=2)) for b in range(2)])
    e = host(s.energy_spectrum(dev(us, torch.float32)))
    for b in range(2):
        ref = O.energy_spectrum(us[b])
        assert max_rel(e[b][:len(ref)], ref) < 1e-12 and not e[b][len(ref):].any()
