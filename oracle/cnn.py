"""Float64 oracle of the learned closure m_theta(u) (Sec. 4) and of the LES right-hand side with it.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper embeds a neural closure in the solver and trains it a-posteriori by
differentiating through the time integration (Sec. 4), but does not fix an
architecture. The closure here is a 3D CNN 3 -> 32 -> 32 -> 3 channels with
3x3x3 kernels, circular padding (the grid is periodic), biases, and the exact
(erf) GELU between layers; no output activation. The three staggered velocity
components are fed as three channels on the cell grid, and output channel a is
added to the a-velocity right-hand side: du/dt = P(F(u) + m_theta(u)).

Parameters (float32 master copy, float64 here): for each layer in order,
W[out][in][kz][ky][kx] then b[out]; 32,899 values in all.

Rounding points (the arithmetic the GPU kernels perform, reproduced here in
float64 on the rounded values): the input u, every weight, and every GELU
output are rounded to bfloat16 (round to nearest even) before entering a
convolution; pre-activations and the output are not rounded. In the backward
pass the cotangent entering each convolution's backward (of m, of each
pre-activation) is rounded to bfloat16; bias gradients use that rounded
cotangent too; the rounding of u and of weights passes gradients through
unchanged.
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as Fn

LAYERS = ((3, 32), (32, 32), (32, 3))
KS = 3


def n_params():
    return sum(o * i * KS ** 3 + o for i, o in LAYERS)


def unpack(theta):
    """Flat parameter vector -> [(W, b)] as float64 torch tensors."""
    t = torch.as_tensor(np.asarray(theta, dtype=np.float64))
    out, off = [], 0
    for cin, cout in LAYERS:
        nw = cout * cin * KS ** 3
        w = t[off:off + nw].reshape(cout, cin, KS, KS, KS)
        off += nw
        b = t[off:off + cout]
        off += cout
        out.append((w, b))
    assert off == t.numel()
    return out


def bf16_round(x):
    """Round float64 values to the nearest bfloat16 (ties to even), returned as float64."""
    a = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(a)  # a = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.rint(m * 256.0) / 256.0, e)


def _bf16_t(x):
    return torch.as_tensor(bf16_round(x.detach().numpy()))


class _RoundFwd(torch.autograd.Function):
    """bfloat16 rounding of a value; the gradient passes through."""

    @staticmethod
    def forward(ctx, x):
        return _bf16_t(x)

    @staticmethod
    def backward(ctx, g):
        return g


class _RoundGrad(torch.autograd.Function):
    """Identity on the value; its incoming cotangent is rounded to bfloat16."""

    @staticmethod
    def forward(ctx, x):
        return x.clone()

    @staticmethod
    def backward(ctx, g):
        return _bf16_t(g)


def gelu(x):
    """Exact GELU x * Phi(x) (erf form)."""
    return 0.5 * x * (1.0 + torch.erf(x / np.sqrt(2.0)))


def conv3d_circular(x, w, b):
    """Cross-correlation with circular padding: out[o,p] = b[o] + sum_{i,t} w[o,i,t] x[i, p + t - 1]."""
    xp = Fn.pad(x, (1, 1, 1, 1, 1, 1), mode="circular")
    return Fn.conv3d(xp, w, b)


def _forward_graph(u, theta):
    """Batched u [B][3][nz][ny][nx] (torch float64) -> m, with rounding nodes."""
    params = unpack(theta)
    x = _RoundFwd.apply(u)
    for li, (w, b) in enumerate(params):
        wr = _RoundFwd.apply(w)
        z = conv3d_circular(x, wr, b)
        z = _RoundGrad.apply(z)
        if li < len(params) - 1:
            x = _RoundFwd.apply(gelu(z))
        else:
            x = z
    return x


def _as_batch(u):
    u = np.asarray(u, dtype=np.float64)
    return (u[None] if u.ndim == 4 else u), u.ndim == 4


def closure(u, theta):
    """m_theta(u) for u of shape [3][nz][ny][nx] or [B][3][nz][ny][nx]."""
    ub, single = _as_batch(u)
    with torch.no_grad():
        m = _forward_graph(torch.as_tensor(ub), theta).numpy()
    return m[0] if single else m


def closure_vjp(u, theta, mbar):
    """(ubar, thetabar) = pullback of m_theta at u applied to mbar."""
    ub, single = _as_batch(u)
    mb, _ = _as_batch(mbar)
    params = unpack(theta)
    flat = torch.as_tensor(np.asarray(theta, dtype=np.float64)).clone().requires_grad_(True)
    x = torch.as_tensor(ub).clone().requires_grad_(True)
    # rebuild the graph on the flat tensor so theta gets a gradient
    off = 0
    h = _RoundFwd.apply(x)
    for li, (cin, cout) in enumerate(LAYERS):
        nw = cout * cin * KS ** 3
        w = flat[off:off + nw].reshape(cout, cin, KS, KS, KS)
        off += nw
        b = flat[off:off + cout]
        off += cout
        z = _RoundGrad.apply(conv3d_circular(h, _RoundFwd.apply(w), b))
        h = _RoundFwd.apply(gelu(z)) if li < len(LAYERS) - 1 else z
    (h * torch.as_tensor(mb)).sum().backward()
    ubar = x.grad.numpy()
    del params
    return (ubar[0] if single else ubar), flat.grad.numpy()


def init_params(seed, scale=1.0):
    """Glorot-uniform weights (fan_in = in*27, fan_out = out*27), zero biases, as float32 values."""
    rng = np.random.default_rng(seed)
    parts = []
    for cin, cout in LAYERS:
        fan_in, fan_out = cin * KS ** 3, cout * KS ** 3
        lim = scale * np.sqrt(6.0 / (fan_in + fan_out))
        parts.append(rng.uniform(-lim, lim, size=cout * cin * KS ** 3))
        parts.append(np.zeros(cout))
    return np.concatenate(parts).astype(np.float32).astype(np.float64)


# ----------------------------------------------------------------------------
# LES right-hand side and RK4 step with the closure (Sec. 4, a-posteriori setting)
# ----------------------------------------------------------------------------

def rhs_with_closure(u, h, nu, theta):
    from . import ins

    return ins.rhs(u, h, nu) + closure(u, theta)


def step_rk4_closure(u0, h, nu, dt, theta):
    from . import ins

    return ins.step_rk4(u0, h, nu, dt, rhs_fn=lambda v: rhs_with_closure(v, h, nu, theta))


def step_rk4_closure_vjp(u0, u1bar, h, nu, dt, theta):
    """(u0bar, thetabar) of one closure-coupled RK4 step."""
    from . import ins

    tbar = np.zeros(n_params())

    def gv(v, fb):
        ub_c, tb = closure_vjp(v, theta, fb)
        tbar[:] += tb
        return ins.rhs_vjp(v, fb, h, nu) + ub_c

    u0bar = ins.step_rk4_vjp(u0, u1bar, h, nu, dt, rhs_fn=lambda v: rhs_with_closure(v, h, nu, theta), rhs_vjp_fn=gv)
    return u0bar, tbar


def rollout_loss_closure(u0, refs, h, nu, dt, theta):
    """(1/S) sum_s mean((u_s - refs[s-1])^2) for the closure-coupled step."""
    S = len(refs)
    u = np.array(u0, dtype=np.float64)
    total = 0.0
    for s in range(S):
        u = step_rk4_closure(u, h, nu, dt, theta)
        total += float(np.mean((u - refs[s]) ** 2)) / S
    return total


def rollout_loss_closure_grad(u0, refs, h, nu, dt, theta):
    """(dL/du0, dL/dtheta) by reverse accumulation over the steps (Sec. 3.4 back-propagation)."""
    S = len(refs)
    states = [np.array(u0, dtype=np.float64)]
    for s in range(S):
        states.append(step_rk4_closure(states[-1], h, nu, dt, theta))
    m = states[0].size
    ubar = np.zeros_like(states[0])
    tbar = np.zeros(n_params())
    for s in range(S, 0, -1):
        ubar = ubar + 2.0 * (states[s] - refs[s - 1]) / (m * S)
        ubar, tb = step_rk4_closure_vjp(states[s - 1], ubar, h, nu, dt, theta)
        tbar += tb
    return ubar, tbar
