"""The allocation-free statistics entry point (ins_stats_noalloc) against
ins_stats, through the C ABI, on the same fields.

Bars: max |u|, max |D u| and the finiteness flag are the same per-cell values
reduced with max, so they must agree exactly. The kinetic energy is a sum of
non-negative terms reduced in a different order: ins_stats adds its per-tile
partials one after another on the host (error at most about n_tiles ulps), the
allocation-free call reduces in trees on the device (a few tens of ulps), so
the bar is (n_tiles + 64) * 2^-52 relative.

Consecutive calls share the device's fixed scratch: a large field (more tiles
than the capped workgroup count, so workgroups walk several tiles) is
followed by a smaller one on another context, whose result must not see the
stale partials of the first.
"""
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


def _tiles(n, batch):
    nz = n[2] if len(n) == 3 else 1
    return -(-n[0] // 64) * -(-n[1] // 4) * nz * batch


def _compare(s, u, n, batch):
    out = torch.full((4,), -7.0, dtype=torch.float64, device=s.device)
    s.stats_noalloc(u, out)
    got = out.cpu().numpy()
    ref = s.stats(u)
    tol = (_tiles(n, batch) + 64) * 2.0 ** -52
    if np.isnan(ref[0]):  # a non-finite entry: both energies are NaN
        assert np.isnan(got[0])
    else:
        assert abs(got[0] - ref[0]) <= tol * abs(ref[0]), (got[0], ref[0])
    assert got[1] == ref[1] and got[2] == ref[2], (got[1:3], ref[1:3])
    assert got[3] == (1.0 if ref[3] else 0.0)
    return got


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_two_calls_large_then_small(precision):
    from paper_2604_18536_amd import Solver

    dt = torch.float64 if precision == "fp64" else torch.float32
    big, small = (256, 64, 64), (40, 18, 6)
    assert _tiles(big, 1) > 2048  # workgroups walk several tiles
    sb = Solver(big, precision=precision)
    ub = dev(S.random_field(big, 5), dt)
    g1 = _compare(sb, ub, big, 1)
    ss = Solver(small, precision=precision, batch=2)
    us = dev(np.stack([S.random_field(small, 6), 3.0 * S.random_field(small, 7)]), dt)
    g2 = _compare(ss, us, small, 2)
    assert g2[0] < g1[0] * 20  # a sum over the small field only
    sb.close()
    ss.close()


def test_channel_and_nonfinite():
    from paper_2604_18536_amd import Solver

    n = (33, 9, 7)
    lo, hi = S.channel_box(n)
    s = Solver(n, lo=lo, hi=hi, bc="walls", pressure="cg")
    s.set_y_faces(S.tanh_faces(n[1], lo[1], hi[1], 1.4))
    u = S.channel_random(n, 3)
    _compare(s, dev(u), n, 1)
    u[0, 2, 3, 4] = np.nan
    got = _compare(s, dev(u), n, 1)
    assert got[3] == 0.0
    s.close()


def test_rejects_null_output():
    import ctypes as C

    from paper_2604_18536_amd import Solver, _lib

    s = Solver((16, 8))
    u = s.new_velocity()
    st = _lib.load().ins_stats_noalloc(s._ctx, C.c_void_p(u.data_ptr()), None)
    assert st == _lib.INS_ERR_INVALID
    s.close()
