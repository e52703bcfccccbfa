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


# Discrete Fourier modes with every wavenumber component nonzero (Nyquist in x
# included): eigenvectors of D G with eigenvalue -sum_a 4 sin^2(pi k_a / N) / h^2.
MODES = [((1, 2, 3), 1.0, 0.3), ((5, 7, 11), -0.7, 1.1), ((301, 419, 139), 0.4, -0.6), ((420, 35, 833), 0.25, 2.0),
         ((16, 840 - 3, 210), -0.5, 0.0)]


def _mode_sum(n, coef):
    """sum_m coef(k_m) A_m cos(2 pi (k_m . I) / n + phi_m) on the pressure points (float64, on the GPU);
    the angle is reduced exactly in integers before the cosine."""
    i = torch.arange(n, device="cuda", dtype=torch.int64)
    out = torch.zeros((n, n, n), dtype=torch.float64, device="cuda")
    for (kx, ky, kz), amp, phi in MODES:
        idx = (kz * i[:, None, None] + ky * i[None, :, None]) % n
        for z0 in range(0, n, 105):  # planes in chunks (bounded temporaries)
            ang = (idx[z0:z0 + 105] + kx * i[None, None, :]) % n
            out[z0:z0 + 105] += coef((kx, ky, kz)) * amp * torch.cos(2 * math.pi * ang.double() / n + phi)
    return out


def test_poisson_840_fourier_modes_closed_form():
    from paper_2604_18536_amd import Solver

    n = 840
    h = 2 * math.pi / n
    lam = lambda k: -sum(4 * math.sin(math.pi * ka / n) ** 2 for ka in k) / h ** 2  # noqa: E731
    r = _mode_sum(n, lambda k: 1.0)
    s = Solver((n, n, n), nu=0.0, precision="fp64")
    p = s.poisson_solve(r)
    del r
    ref = _mode_sum(n, lambda k: 1.0 / lam(k))
    err = float((p - ref).abs().max()) / float(ref.abs().max())
    s.close()
    assert err < 1e-12, err


def test_projection_840_random_field_invariants():
    from paper_2604_18536_amd import Solver

    n = 840
    s = Solver((n, n, n), nu=0.0, precision="fp64")
    g = torch.Generator(device="cuda").manual_seed(7)
    u = torch.randn((3, n, n, n), dtype=torch.float64, device="cuda", generator=g)
    pu = s.project(u)
    del u
    h = 2 * math.pi / n
    div = float(s.divergence(pu).abs().max())
    scale = float(pu.abs().max())
    assert div < 1e-12 * scale / h, div * h / scale
    ppu = s.project(pu)
    err = float((ppu - pu).abs().max())
    s.close()
    assert err < 1e-12 * scale, err / scale
