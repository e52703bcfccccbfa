"""Pins of the closure oracle: bfloat16 rounding against torch's cast, the
circular convolution's tap orientation (delta and shift kernels, brute-force
loops), the 1x1x1 special case as a channel GEMM, GELU against torch's; with
the rounding switched off, the pullbacks of the closure, of the closure-coupled
RK4 step and of the trajectory loss against float64 central differences (every
parameter range on its own); with the rounding on, the rounding points against
a centre-tap network written as per-cell matrix products; the float32 error
bound against an independent float32 evaluation. Planted mistakes (taps of the
input gradient not flipped, bias gradient dropped, cotangent rounded after
instead of before the GELU derivative) each fail one of these pins."""
import numpy as np
import pytest
import scipy.special
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


def test_closure_without_rounding_is_the_smooth_network():
    n = (4, 5, 3)
    u = S.random_field(n, 3)
    th = C.init_params(4, scale=2.0)
    with C.bf16_rounding(False):
        m = C.closure(u, th)
    assert np.abs(m - _smooth_closure(u, th).numpy()).max() < 1e-14 * np.abs(m).max()


RANGES = [(0, 2592), (2592, 2624), (2624, 30272), (30272, 30304), (30304, 32896), (32896, 32899)]


def _theta_with_bias(seed, scale=2.0):
    th = C.init_params(seed, scale)
    rng = np.random.default_rng(seed + 1000)
    for lo, hi in RANGES[1::2]:
        th[lo:hi] = 0.1 * rng.standard_normal(hi - lo)
    return th


def _closure_fd_errors(n=(4, 5, 3), batch=2):
    """Relative errors of the closure pullback (rounding off) against central
    differences: u directions, a full theta direction, one direction per range."""
    rng = np.random.default_rng(11)
    u = rng.standard_normal((batch, 3) + n[::-1])
    th = _theta_with_bias(12)
    mbar = rng.standard_normal(u.shape)
    errs = []
    with C.bf16_rounding(False):
        ub, tb = C.closure_vjp(u, th, mbar)
        eps = 1e-6
        f = lambda uu, tt: float((C.closure(uu, tt) * mbar).sum())  # noqa: E731
        for _ in range(2):
            v = rng.standard_normal(u.shape)
            fd = (f(u + eps * v, th) - f(u - eps * v, th)) / (2 * eps)
            errs.append(abs(fd - float((ub * v).sum())) / (abs(fd) + 1e-12))
        for lo, hi in [(0, th.size)] + RANGES:
            vt = np.zeros_like(th)
            vt[lo:hi] = rng.standard_normal(hi - lo)
            fd = (f(u, th + eps * vt) - f(u, th - eps * vt)) / (2 * eps)
            errs.append(abs(fd - float((tb * vt).sum())) / (abs(fd) + 1e-12))
    return errs


def test_closure_vjp_matches_central_differences_without_rounding():
    errs = _closure_fd_errors()
    assert max(errs) < 1e-7, errs


def _step_fd_errors():
    n = (6, 4, 4)
    h = S.spacing(n)
    nu, dt = 0.02, 1e-2
    th = _theta_with_bias(9, 1.0)
    u0 = S.turbulence_ic(n, seed=1, k0=2)
    ubar = S.random_field(n, 2)
    rng = np.random.default_rng(3)
    errs = []
    with C.bf16_rounding(False):
        g, tb = C.step_rk4_closure_vjp(u0, ubar, h, nu, dt, th)
        f = lambda uu, tt: float((C.step_rk4_closure(uu, h, nu, dt, tt) * ubar).sum())  # noqa: E731
        eps = 1e-6
        v = O.project(rng.standard_normal(u0.shape), h)[0]
        fd = (f(u0 + eps * v, th) - f(u0 - eps * v, th)) / (2 * eps)
        errs.append(abs(fd - float((g * v).sum())) / abs(fd))
        for lo, hi in [(0, th.size)] + RANGES:
            vt = np.zeros_like(th)
            vt[lo:hi] = rng.standard_normal(hi - lo)
            fd = (f(u0, th + eps * vt) - f(u0, th - eps * vt)) / (2 * eps)
            errs.append(abs(fd - float((tb * vt).sum())) / abs(fd))
    return errs


def test_closure_step_vjp_matches_central_differences_without_rounding():
    errs = _step_fd_errors()
    assert max(errs) < 1e-7, errs


def test_closure_step_vjp_with_zero_closure_is_the_plain_step_pullback():
    n = (6, 4, 4)
    h = S.spacing(n)
    u0 = S.turbulence_ic(n, seed=1, k0=2)
    ubar = S.random_field(n, 2)
    g0, tb0 = C.step_rk4_closure_vjp(u0, ubar, h, 0.02, 1e-2, np.zeros(C.n_params()))
    assert np.abs(g0 - O.step_rk4_vjp(u0, ubar, h, 0.02, 1e-2)).max() < 1e-12 * np.abs(g0).max()


def test_rollout_closure_gradient_matches_central_differences_without_rounding():
    n = (6, 4, 4)
    h = S.spacing(n)
    nu, dt, steps = 0.02, 1e-2, 3
    th = _theta_with_bias(21, 1.0)
    u0 = S.turbulence_ic(n, seed=22, k0=2)
    refs = [S.turbulence_ic(n, seed=30 + s, k0=2) for s in range(steps)]
    rng = np.random.default_rng(4)
    with C.bf16_rounding(False):
        g, tb = C.rollout_loss_closure_grad(u0, refs, h, nu, dt, th)
        f = lambda uu, tt: C.rollout_loss_closure(uu, refs, h, nu, dt, tt)  # noqa: E731
        eps = 1e-6
        v = rng.standard_normal(u0.shape)
        # tolerance: 1e-7 relative plus the central difference's own rounding, eps_64 |L| / eps
        fl = 20 * np.finfo(float).eps * f(u0, th) / eps
        fd = (f(u0 + eps * v, th) - f(u0 - eps * v, th)) / (2 * eps)
        assert abs(fd - float((g * v).sum())) < 1e-7 * abs(fd) + fl
        for lo, hi in [(0, th.size)] + RANGES:
            vt = np.zeros_like(th)
            vt[lo:hi] = rng.standard_normal(hi - lo)
            fd = (f(u0, th + eps * vt) - f(u0, th - eps * vt)) / (2 * eps)
            assert abs(fd - float((tb * vt).sum())) < 1e-7 * abs(fd) + fl, (lo, hi)


# --- rounding points: a network whose only nonzero tap is the centre one is a per-cell MLP

def _centre_tap_theta(seed):
    th = _theta_with_bias(seed, 2.0)
    for (cin, cout), (lo, _) in zip(C.LAYERS, RANGES[0::2]):
        w = th[lo:lo + cout * cin * 27].reshape(cout, cin, 3, 3, 3)
        keep = w[:, :, 1, 1, 1].copy()
        w[:] = 0.0
        w[:, :, 1, 1, 1] = keep
    return th


def _bf(x):
    return C.bf16_round(x)


def _gelu_np(z):
    return 0.5 * z * (1.0 + scipy.special.erf(z / np.sqrt(2.0)))


def _gelu_grad_np(z):
    return 0.5 * (1.0 + scipy.special.erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2 * np.pi)


def _mlp_reference(u, th, mbar):
    """The stated rounding points, written out for a centre-tap network: each
    cell is a 3 -> 32 -> 32 -> 3 perceptron; the weight gradient of tap t sums
    over cells p the cotangent at p times the input at p + offset(t)."""
    shape = u.shape[1:]
    cells = lambda a: a.reshape(a.shape[0], -1).T  # noqa: E731  [channels][...] -> [cell][channels]
    Ws, bs = [], []
    for (cin, cout), (lo, _), (blo, bhi) in zip(C.LAYERS, RANGES[0::2], RANGES[1::2]):
        Ws.append(_bf(th[lo:lo + cout * cin * 27].reshape(cout, cin, 3, 3, 3)[:, :, 1, 1, 1]))
        bs.append(th[blo:bhi])
    X0 = _bf(cells(u))
    Z1 = X0 @ Ws[0].T + bs[0]
    X1 = _bf(_gelu_np(Z1))
    Z2 = X1 @ Ws[1].T + bs[1]
    X2 = _bf(_gelu_np(Z2))
    M = X2 @ Ws[2].T + bs[2]
    G3 = _bf(cells(mbar))
    GZ2 = _bf((G3 @ Ws[2]) * _gelu_grad_np(Z2))
    GZ1 = _bf((GZ2 @ Ws[1]) * _gelu_grad_np(Z1))
    UB = GZ1 @ Ws[0]
    parts = []
    for G, X in ((GZ1, X0), (GZ2, X1), (G3, X2)):
        Xg = X.T.reshape((X.shape[1],) + shape)
        wg = np.zeros((G.shape[1], X.shape[1], 3, 3, 3))
        for kz in range(3):
            for ky in range(3):
                for kx in range(3):
                    Xs = np.roll(Xg, (1 - kz, 1 - ky, 1 - kx), axis=(1, 2, 3)).reshape(X.shape[1], -1)
                    wg[:, :, kz, ky, kx] = G.T @ Xs.T
        parts += [wg.reshape(-1), G.sum(axis=0)]
    back = lambda a: a.T.reshape((a.shape[1],) + shape)  # noqa: E731
    return back(M), back(UB), np.concatenate(parts)


def _centre_tap_errors():
    n = (5, 4, 3)
    rng = np.random.default_rng(5)
    u = f32(rng.standard_normal((3,) + n[::-1]))
    mbar = f32(rng.standard_normal(u.shape))
    th = _centre_tap_theta(6)
    m_ref, ub_ref, tb_ref = _mlp_reference(u, th, mbar)
    m = C.closure(u, th)
    ub, tb = C.closure_vjp(u, th, mbar)
    rel = lambda a, b: float(np.abs(a - b).max() / np.abs(b).max())  # noqa: E731
    return rel(m, m_ref), rel(ub, ub_ref), max(rel(tb[lo:hi], tb_ref[lo:hi]) for lo, hi in RANGES)


def f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def test_rounding_points_on_a_centre_tap_network():
    errs = _centre_tap_errors()
    assert max(errs) < 1e-13, errs


def test_rounded_network_stays_near_the_smooth_one():
    n = (4, 5, 3)
    u = S.random_field(n, 7)
    th = _theta_with_bias(8, 1.0)
    mbar = S.random_field(n, 9)
    m = C.closure(u, th)
    ub, tb = C.closure_vjp(u, th, mbar)
    with C.bf16_rounding(False):
        m0 = C.closure(u, th)
        ub0, tb0 = C.closure_vjp(u, th, mbar)
    # a few bfloat16 units (2^-8 relative) per rounding point, and rounding does matter
    for a, b in ((m, m0), (ub, ub0), (tb, tb0)):
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        assert 1e-4 < rel < 0.03, rel
    ubz, tbz = C.closure_vjp(u, th, np.zeros_like(u))
    assert not ubz.any() and not tbz.any()


# --- the float32 error bound against an independent float32 evaluation

def _float32_closure(u, th, mbar):
    """The network and its pullback in float32, layer by layer (torch's float32
    convolutions and their autograd transposes, float32 GELU and GELU',
    bfloat16 casts at the stated points): an arithmetic of the kind the bounds
    describe, written without the oracle. Returns its tensors (as the GPU
    library exports them, in the oracle layout), ubar and thetabar."""
    f = lambda a: torch.tensor(a, dtype=torch.float32)  # noqa: E731
    bf = lambda a: a.to(torch.bfloat16).to(torch.float32)  # noqa: E731
    pad = lambda a: Fn.pad(a, (1, 1) * 3, mode="circular")  # noqa: E731
    g32 = lambda z: 0.5 * z * (1.0 + torch.erf(z * 0.70710678118654752))  # noqa: E731
    dg32 = lambda z: 0.5 * (1.0 + torch.erf(z * 0.70710678118654752)) + z * 0.3989422804014327 * torch.exp(-0.5 * z * z)  # noqa: E731
    params = [(bf(w.float()), b.float()) for w, b in C.unpack(f(th).double().numpy())]
    x0 = bf(f(u))
    ins, t = [x0], {}
    for li, (w, b) in enumerate(params):
        z = Fn.conv3d(pad(ins[-1]), w, b)
        if li < 2:
            t[f"z{li + 1}"] = z
            ins.append(bf(g32(z)))
            t[f"a{li + 1}"] = ins[-1]
        else:
            t["m"] = z
    cot = [None, None, bf(f(mbar))]
    grads = [None] * 3
    for li in (2, 1, 0):
        w, _ = params[li]
        xi = ins[li].clone().requires_grad_(True)
        wi = w.clone().requires_grad_(True)
        gx, gw = torch.autograd.grad(Fn.conv3d(pad(xi), wi), (xi, wi), cot[li])
        grads[li] = torch.cat([gw.reshape(-1), cot[li].sum(dim=(0, 2, 3, 4))])
        if li > 0:
            cot[li - 1] = bf(gx * dg32(t[f"z{li}"]))
            t[f"gz{li}"] = cot[li - 1]
        else:
            ub = gx
    zeros5 = torch.zeros((u.shape[0], 5) + u.shape[2:])
    t["x0"] = torch.cat([x0, zeros5], dim=1)
    t["gm"] = torch.cat([cot[2], zeros5], dim=1)
    t = {k: v.double().numpy() for k, v in t.items()}
    return t, ub.double().numpy(), torch.cat(grads).double().numpy()


def test_layer_bounds_cover_a_float32_evaluation_and_are_tight():
    from tests.closure_check import check_closure_layers

    n = (8, 6, 4)
    rng = np.random.default_rng(13)
    u = f32(rng.standard_normal((2, 3) + n[::-1]))
    mbar = f32(rng.standard_normal(u.shape))
    th = f32(_theta_with_bias(14, 2.0))
    t, ub, tb = _float32_closure(u, th, mbar)
    ff, fb = check_closure_layers(u, th, mbar, t, ub, tb)
    assert ff < 1e-3 * u.size * 32 and fb < 1e-3 * u.size * 32, (ff, fb)
    # not vacuous: each layer's bound lies far below 1% of almost every entry
    ub_ref, e = C.layer_dgrad(t["gz1"], th, 0)
    big = np.abs(ub_ref) > 1e-3 * np.abs(ub_ref).max()
    assert np.mean(e[big] < 1e-2 * np.abs(ub_ref[big])) > 0.9
    for li, (g, x) in enumerate(((t["gz1"], t["x0"][:, :3]), (t["gz2"], t["a1"]), (t["gm"][:, :3], t["a2"]))):
        val, bound = C.layer_wgrad(g, x, li)
        big = np.abs(val) > 1e-3 * np.abs(val).max()
        assert np.mean(bound[big] < 1e-2 * np.abs(val[big])) > 0.9, li
    # and the whole network stays within the accumulation bounds, up to the few flips
    m_ref = C.closure(u, th)
    acc = C.accumulation_bounds(u, th, mbar)
    assert np.mean(np.abs(t["m"] - m_ref) <= acc["m"]) > 0.99


# --- planted mistakes: each fails a pin above

_CONV = C.conv3d_circular


class _ConvPlant(torch.autograd.Function):
    """The convolution with a planted mistake in its backward."""
    mode = "unflipped"

    @staticmethod
    def forward(ctx, x, w, b):
        ctx.save_for_backward(x, w)
        return _CONV(x, w, b)

    @staticmethod
    def backward(ctx, g):
        x, w = ctx.saved_tensors
        with torch.enable_grad():
            xx, ww = x.detach().requires_grad_(True), w.detach().requires_grad_(True)
            gx, gw = torch.autograd.grad(_CONV(xx, ww, None), (xx, ww), g)
        gb = g.sum(dim=(0, 2, 3, 4))
        if _ConvPlant.mode == "unflipped":
            gx = _CONV(g, w.transpose(0, 1).contiguous(), None)
        else:
            gb = torch.zeros_like(gb)
        return gx, gw, gb


@pytest.mark.parametrize("mode", ["unflipped", "no_bias_grad"])
def test_planted_backward_mistakes_fail_the_central_difference_pins(monkeypatch, mode):
    monkeypatch.setattr(_ConvPlant, "mode", mode)
    monkeypatch.setattr(C, "conv3d_circular", lambda x, w, b: _ConvPlant.apply(x, w, b))
    assert max(_closure_fd_errors()) > 1e-3
    assert max(_step_fd_errors()) > 1e-3


def test_planted_cotangent_rounding_point_fails_the_centre_tap_pin(monkeypatch):
    def moved(u, flat, record=None):
        h = C._RoundFwd.apply(u)
        layers = C._layer_params(flat)
        for li, (w, b) in enumerate(layers):
            z = C.conv3d_circular(h, C._RoundFwd.apply(w), b)
            if li < len(layers) - 1:
                # mistake: the cotangent is rounded before, not after, the GELU derivative
                h = C._RoundGrad.apply(C._RoundFwd.apply(C.gelu(z)))
            else:
                h = C._RoundGrad.apply(z)
        return h

    monkeypatch.setattr(C, "_network", moved)
    assert max(_centre_tap_errors()) > 1e-6
