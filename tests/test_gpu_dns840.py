"""Full-size 840^3 runs (840 = 2^3 * 3 * 5 * 7, mixed-radix FFT): the z-extruded
Taylor-Green field is an exact discrete solution of the projected RK4 scheme at
any grid size (convection is a gradient there and the Laplacian scales it), so
after k steps u = R(z)^k u_TG with R the RK4 stability polynomial and
z = nu * (-8 sin^2(h/2) / h^2) * dt. Checked element-wise on the GPU in FP64
and in the FP32-stencil mode, in the launch configuration the benchmark uses."""
import math

import pytest
import torch

import synth as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _tg840(dtype, amplitude=2.0):
    n = 840
    u2 = torch.tensor(S.taylor_green_2d((n, n), amplitude), device="cuda", dtype=torch.float64)
    u = torch.zeros((3, n, n, n), dtype=dtype, device="cuda")
    u[0] = u2[0][None].to(dtype)
    u[1] = u2[1][None].to(dtype)
    return u


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 2e-6)])
def test_extruded_taylor_green_840_closed_form(precision, tol):
    from paper_2604_18536_amd import Solver

    n, nu, dt, steps = 840, 1.0 / 5000.0, 1e-3, 2
    s = Solver((n, n, n), nu=nu, precision=precision)
    u = _tg840(s.dtype)
    u0 = u.clone()
    for _ in range(steps):
        s.step(u, dt, out=u)
    h = 2 * math.pi / n
    z = nu * (-8 * math.sin(h / 2) ** 2 / h ** 2) * dt
    r = (1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24) ** steps
    err = float((u.double() - r * u0.double()).abs().max())
    scale = float(u0.abs().max())
    ke, umax, maxdiv, finite = s.stats(u)
    s.close()
    assert finite and err < tol * scale, err / scale
    assert maxdiv < (1e-9 if precision == "fp64" else 1e-2)
