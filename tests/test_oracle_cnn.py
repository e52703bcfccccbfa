"""Pins of the closure oracle: bfloat16 rounding against torch's cast, the
circular convolution's tap orientation (delta and shift kernels, brute-force
loops), the 1x1x1 special case as a channel GEMM, GELU against torch's, and the
pullback against float64 central differences with the rounding removed."""
import numpy as np
import pytest
import torch
import torch.nn.functional as Fn

import oracle as O
import oracle.cnn as C
import synth as S


def test_bf16_round_matches_torch_cast_of_float32_values():
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(20000) * np.exp(rng.uniform(-20, 20, 20000))).astype(np.float32)
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(C.bf16_round(x.astype(np.float64)), ref)


def test_bf16_round_ties_to_even():
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: ties to the even significand (1.0)
    assert C.bf16_round(1.0 + 2.0 ** -8) == 1.0
    assert C.bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6


def test_conv_delta_and_shift_kernels():
    x = torch.tensor(S.random_field((6, 5, 4), 1))[None]
    w = torch.zeros(3, 3, 3, 3, 3, dtype=torch.float64)
    for c in range(3):
        w[c, c, 1, 1, 1] = 1.0
    assert torch.equal(C.conv3d_circular(x, w, None), x)
    # tap (kz, ky, kx) = (1, 1, 2) reads x[p + e_x]: a periodic shift by one cell
    w2 = torch.zeros(3, 3, 3, 3, 3, dtype=torch.float64)
    for c in range(3):
        w2[c, c, 1, 1, 2] = 1.0
    assert torch.equal(C.conv3d_circular(x, w2, None), torch.roll(x, -1, dims=-1))
    w3 = torch.zeros(3, 3, 3, 3, 3, dtype=torch.float64)
    for c in range(3):
        w3[c, c, 0, 1, 1] = 1.0  # kz = 0 reads x[p - e_z]
    assert torch.equal(C.conv3d_circular(x, w3, None), torch.roll(x, 1, dims=-3))


def test_conv_one_by_one_is_a_channel_gemm():
    rng = np.random.default_rng(1)
    x = torch.tensor(rng.standard_normal((2, 5, 3, 4, 6)))
    w = torch.zeros(7, 5, 3, 3, 3, dtype=torch.float64)
    w[:, :, 1, 1, 1] = torch.tensor(rng.standard_normal((7, 5)))
    b = torch.tensor(rng.standard_normal(7))
    ref = torch.einsum("oi,bizyx->bozyx", w[:, :, 1, 1, 1], x) + b[None, :, None, None, None]
    assert torch.allclose(C.conv3d_circular(x, w, b), ref, atol=1e-13)


def test_conv_brute_force_loops():
    rng = np.random.default_rng(2)
    nz, ny, nx, ci, co = 3, 4, 5, 2, 3
    x = rng.standard_normal((ci, nz, ny, nx))
    w = rng.standard_normal((co, ci, 3, 3, 3))
    b = rng.standard_normal(co)
    got = C.conv3d_circular(torch.tensor(x)[None], torch.tensor(w), torch.tensor(b))[0].numpy()
    for o in range(co):
        for z in range(nz):
            for y in range(ny):
                for xx in range(nx):
                    acc = b[o]
                    for i in range(ci):
                        for kz in range(3):
                            for ky in range(3):
                                for kx in range(3):
                                    acc += w[o, i, kz, ky, kx] * x[i, (z + kz - 1) % nz, (y + ky - 1) % ny, (xx + kx - 1) % nx]
                    assert abs(got[o, z, y, xx] - acc) < 1e-12


def test_gelu_matches_torch():
    x = torch.linspace(-8, 8, 1001, dtype=torch.float64)
    assert torch.allclose(C.gelu(x), Fn.gelu(x), atol=1e-15)


def test_parameter_count_and_init():
    assert C.n_params() == 32899
    th = C.init_params(0)
    assert th.shape == (32899,)
    assert np.array_equal(th, th.astype(np.float32).astype(np.float64))


def _smooth_closure(u, theta):
    params = C.unpack(theta)
    x = torch.tensor(u)[None]
    for li, (w, b) in enumerate(params):
        x = C.conv3d_circular(x, w, b)
        if li < 2:
            x = C.gelu(x)
    return x[0]


def test_closure_without_rounding_gradients_match_central_differences():
    n = (4, 5, 3)
    u = S.random_field(n, 3)
    th = C.init_params(4, scale=2.0)
    mbar = S.random_field(n, 5)
    # pullback of the smooth network via autograd (no rounding nodes)
    ut = torch.tensor(u, requires_grad=True)
    tt = torch.tensor(th, requires_grad=True)
    off, x = 0, ut[None]
    for li, (ci, co) in enumerate(C.LAYERS):
        nw = co * ci * 27
        w = tt[off:off + nw].reshape(co, ci, 3, 3, 3)
        b = tt[off + nw:off + nw + co]
        off += nw + co
        x = C.conv3d_circular(x, w, b)
        if li < 2:
            x = C.gelu(x)
    (x[0] * torch.tensor(mbar)).sum().backward()
    rng = np.random.default_rng(6)
    for _ in range(3):
        v = rng.standard_normal(u.shape)
        fd = float(((_smooth_closure(u + 1e-6 * v, th) - _smooth_closure(u - 1e-6 * v, th)) * torch.tensor(mbar)).sum()) / 2e-6
        assert abs(fd - float((ut.grad.numpy() * v).sum())) < 1e-7 * (1 + abs(fd))
        vt = rng.standard_normal(th.shape)
        fd = float(((_smooth_closure(u, th + 1e-6 * vt) - _smooth_closure(u, th - 1e-6 * vt)) * torch.tensor(mbar)).sum()) / 2e-6
        assert abs(fd - float((tt.grad.numpy() * vt).sum())) < 1e-7 * (1 + abs(fd))


def test_rounded_closure_is_close_to_smooth_and_pullback_rounds_only_where_stated():
    n = (4, 5, 3)
    u = S.random_field(n, 7)
    th = C.init_params(8)
    m = C.closure(u, th)
    assert np.abs(m - _smooth_closure(u, th).numpy()).max() < 0.05 * np.abs(m).max()
    # with bfloat16-representable inputs, weights and an exactly representable
    # cotangent of zero, the pullback is exactly zero
    ub, tb = C.closure_vjp(u, th, np.zeros_like(u))
    assert not ub.any() and not tb.any()


def test_closure_step_vjp_consistent_with_central_difference():
    n = (6, 4, 4)
    h = S.spacing(n)
    nu, dt = 0.02, 1e-2
    th = C.init_params(9, scale=0.5)
    u0 = S.turbulence_ic(n, seed=1, k0=2)
    ubar = S.random_field(n, 2)
    g, tb = C.step_rk4_closure_vjp(u0, ubar, h, nu, dt, th)
    assert g.shape == u0.shape and tb.shape == th.shape and np.isfinite(tb).all()
    # the pullback is the exact transpose of the linearisation with straight-through
    # rounding; with nu-only dynamics (closure zeroed) it reduces to the plain step pullback
    g0, tb0 = C.step_rk4_closure_vjp(u0, ubar, h, nu, dt, np.zeros_like(th))
    assert np.abs(g0 - O.step_rk4_vjp(u0, ubar, h, nu, dt)).max() < 1e-12 * np.abs(g0).max()
