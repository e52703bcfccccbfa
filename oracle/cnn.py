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

``bf16_rounding(False)`` turns every rounding point into the identity, so the
network becomes a smooth function of u and theta that central differences can
check. ``layer_forward``, ``layer_dgrad`` and ``layer_wgrad`` evaluate one
layer on given operands with the bound gamma_K sum |w||x| that a float32 sum of
the same terms obeys (the GPU kernels sum in float32), so the GPU can be
checked layer by layer on its own operands.
"""
from __future__ import annotations

import contextlib

import numpy as np
import torch
import torch.nn.functional as Fn

LAYERS = ((3, 32), (32, 32), (32, 3))
KS = 3


def n_params():
    return sum(o * i * KS ** 3 + o for i, o in LAYERS)


def unpack(theta):
    """Flat parameter vector -> [(W, b)] as float64 torch tensors."""
    return _layer_params(torch.as_tensor(np.asarray(theta, dtype=np.float64)))


def _layer_params(flat):
    """Views (W, b) of each layer inside a flat parameter tensor."""
    out, off = [], 0
    for cin, cout in LAYERS:
        nw = cout * cin * KS ** 3
        out.append((flat[off:off + nw].reshape(cout, cin, KS, KS, KS), flat[off + nw:off + nw + cout]))
        off += nw + cout
    assert off == flat.numel()
    return out


def bf16_round(x):
    """Round float64 values to the nearest bfloat16 (ties to even), returned as float64."""
    a = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(a)  # a = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.rint(m * 256.0) / 256.0, e)


_ROUND = [True]


@contextlib.contextmanager
def bf16_rounding(on):
    """Within the block every bfloat16 rounding point is on (True) or the identity (False)."""
    old = _ROUND[0]
    _ROUND[0] = bool(on)
    try:
        yield
    finally:
        _ROUND[0] = old


def _bf16_t(x):
    x = x.detach()
    if not _ROUND[0]:
        return x.clone()
    return torch.as_tensor(bf16_round(x.numpy()))


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


def _network(u, flat, record=None):
    """m = m_theta(u) for batched u [B][3][nz][ny][nx] (float64 tensors) and a
    flat parameter tensor, with the rounding nodes at the stated points.

    With ``record`` (a list) every layer appends a dict of its tensors: ``c``
    the convolution output (before the cotangent rounding), ``z`` the
    pre-activation, ``a`` the GELU output before rounding (None for the last
    layer), ``h`` the layer's output, ``w``/``b`` its parameters. Gradients of
    c, z and h are retained, so a backward pass leaves in ``.grad``: of z the
    cotangent before rounding, of c the rounded one, of h the cotangent of the
    layer's (rounded) output."""
    h = _RoundFwd.apply(u)
    layers = _layer_params(flat)
    for li, (w, b) in enumerate(layers):
        c = conv3d_circular(h, _RoundFwd.apply(w), b)
        z = _RoundGrad.apply(c)
        a = gelu(z) if li < len(layers) - 1 else None
        h = _RoundFwd.apply(a) if a is not None else z
        if record is not None:
            if c.requires_grad:
                for t in (c, z, h):
                    t.retain_grad()
            record.append({"c": c, "z": z, "a": a, "h": h, "w": w, "b": b})
    return h


def _as_batch(u):
    u = np.asarray(u, dtype=np.float64)
    return (u[None] if u.ndim == 4 else u), u.ndim == 4


def closure(u, theta):
    """m_theta(u) for u of shape [3][nz][ny][nx] or [B][3][nz][ny][nx]."""
    ub, single = _as_batch(u)
    with torch.no_grad():
        m = _network(torch.as_tensor(ub), torch.as_tensor(np.asarray(theta, dtype=np.float64))).numpy()
    return m[0] if single else m


def closure_vjp(u, theta, mbar):
    """(ubar, thetabar) = pullback of m_theta at u applied to mbar."""
    ub, single = _as_batch(u)
    mb, _ = _as_batch(mbar)
    flat = torch.as_tensor(np.asarray(theta, dtype=np.float64)).clone().requires_grad_(True)
    x = torch.as_tensor(ub).clone().requires_grad_(True)
    (_network(x, flat) * torch.as_tensor(mb)).sum().backward()
    ubar = x.grad.numpy()
    return (ubar[0] if single else ubar), flat.grad.numpy()


# ----------------------------------------------------------------------------
# Single layers on given operands, and the error bounds of float32 sums
# ----------------------------------------------------------------------------

U32 = 2.0 ** -24   # unit roundoff of float32
GELU_D1 = 1.1290   # max |GELU'(x)| (at x = sqrt 2: Phi(sqrt 2) + sqrt 2 phi(sqrt 2) = 1.12897)
GELU_D2 = 0.7979   # max |GELU''(x)| = 2 phi(0) (GELU'' = phi(x)(2 - x^2))


def gamma(k):
    """gamma_k = k u / (1 - k u): a k-term float32 sum, in any order, errs by at
    most gamma_k times the sum of the absolute terms (Higham, Accuracy and
    Stability of Numerical Algorithms, Sec. 3.1)."""
    k = float(k)
    return k * U32 / (1.0 - k * U32)


def gelu_grad(z):
    """GELU'(z) = Phi(z) + z phi(z) (float64 tensor or array)."""
    z = torch.as_tensor(z)
    return 0.5 * (1.0 + torch.erf(z / np.sqrt(2.0))) + z * torch.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def gelu_f32_error(z):
    """Bound on |GELU(z) evaluated in float32 - GELU(z)|: the erf argument is
    off by 2u|z|, erf by 4u (2 ulp) plus that argument error times 2/sqrt(pi);
    the sum 1 + erf and the two products add 3u relative."""
    z = np.abs(np.asarray(z))
    return U32 * z * (6.0 + 0.5 * z)


def gelu_grad_f32_error(z):
    """Bound on |GELU'(z) evaluated in float32 - GELU'(z)| (same float32 error
    model: erf and exp to 2 ulp, every other operation rounded once)."""
    z = np.abs(np.asarray(z))
    return U32 * (16.0 + 2.0 * z)


def flip_allowance(v, e):
    """Largest change of the bfloat16 rounding of v when v moves by at most e:
    0 where no rounding boundary lies within e of v (rounding is monotone)."""
    r = bf16_round(v)
    return np.maximum(np.abs(bf16_round(v + e) - r), np.abs(bf16_round(v - e) - r))


def _layer_wb(theta, li):
    w, b = unpack(theta)[li]
    return bf16_round(w.numpy()), b.numpy()


def _conv_sums(x, w, g=None):
    """conv(x, w) and, with a cotangent g, conv^T(g, w) and corr(g, x): the
    forward, input-gradient and weight-gradient sums of a circular
    convolution without bias (float64)."""
    xt = torch.as_tensor(np.asarray(x, dtype=np.float64)).requires_grad_(g is not None)
    wt = torch.as_tensor(np.asarray(w, dtype=np.float64)).requires_grad_(g is not None)
    y = conv3d_circular(xt, wt, None)
    if g is None:
        return y.detach().numpy()
    dx, dw = torch.autograd.grad(y, (xt, wt), torch.as_tensor(np.asarray(g, dtype=np.float64)))
    return y.detach().numpy(), dx.numpy(), dw.numpy()


def layer_forward(x, theta, li):
    """Layer li (0, 1, 2) on a given (bfloat16-valued) input x [B][C_in][nz][ny][nx]:
    (z, bound) with z = conv(x, bf16(W)) + b in float64 and bound =
    gamma_{K+1} (conv(|x|, |W|) + |b|), K = 27 C_in: how far a float32 sum of
    the same terms may lie from z."""
    w, b = _layer_wb(theta, li)
    bb = b[None, :, None, None, None]
    z = _conv_sums(x, w) + bb
    k = LAYERS[li][0] * KS ** 3
    return z, gamma(k + 1) * (_conv_sums(np.abs(x), np.abs(w)) + np.abs(bb))


def layer_dgrad(g, theta, li):
    """Input gradient of layer li for a given (bfloat16-valued) cotangent g of its
    output: (conv^T(g, bf16(W)), gamma_K conv^T(|g|, |W|)), K = 27 C_out."""
    w, _ = _layer_wb(theta, li)
    shape = (g.shape[0], LAYERS[li][0]) + g.shape[2:]
    _, dx, _ = _conv_sums(np.zeros(shape), w, g)
    _, da, _ = _conv_sums(np.zeros(shape), np.abs(w), np.abs(g))
    return dx, gamma(LAYERS[li][1] * KS ** 3) * da


def layer_wgrad(g, x, li):
    """Weight and bias gradient of layer li from its cotangent g and input x:
    (flat [W_bar, b_bar], bound) with W_bar[o,i,t] = sum_p g[p,o] x[p+t,i],
    b_bar[o] = sum_p g[p,o]; bound = gamma_K of the absolute sums with K = the
    number of cells (no split of the cells into float32 partial sums has more
    terms), plus the float32 store of each result."""
    cin, cout = LAYERS[li]
    w0 = np.zeros((cout, cin, KS, KS, KS))
    _, _, dw = _conv_sums(x, w0, g)
    _, _, da = _conv_sums(np.abs(x), w0, np.abs(g))
    kc = g.shape[0] * int(np.prod(g.shape[2:]))
    val = np.concatenate([dw.reshape(-1), g.sum(axis=(0, 2, 3, 4))])
    absum = np.concatenate([da.reshape(-1), np.abs(g).sum(axis=(0, 2, 3, 4))])
    bound = gamma(kc) * absum
    return val, bound + U32 * (np.abs(val) + bound)


def accumulation_bounds(u, theta, mbar):
    """The float32 summation bounds of the last sum behind each output, at this
    oracle's own operands: m from layer 3's forward sum, ubar from layer 1's
    input-gradient sum, thetabar from each layer's weight-gradient sums. Where
    no bfloat16 rounding flips (a float32 value landing on the other side of a
    rounding boundary), every earlier operand is the same on both sides and
    these are the whole bound; flips are rare and are checked layer by layer
    where the operands are available. Returns a dict m, ubar, theta."""
    ub, single = _as_batch(u)
    mb, _ = _as_batch(mbar)
    rec = []
    flat = torch.as_tensor(np.asarray(theta, dtype=np.float64)).clone().requires_grad_(True)
    x = torch.as_tensor(ub).clone().requires_grad_(True)
    m = _network(x, flat, rec)
    (m * torch.as_tensor(mb)).sum().backward()
    ops = [bf16_round(ub)] + [L["h"].detach().numpy() for L in rec[:-1]]
    grads = [L["c"].grad.numpy() for L in rec]
    em = layer_forward(ops[2], theta, 2)[1]
    eu = layer_dgrad(grads[0], theta, 0)[1]
    eth = np.concatenate([layer_wgrad(grads[li], ops[li], li)[1] for li in range(3)])
    return {"m": em[0] if single else em, "ubar": eu[0] if single else eu, "theta": eth}


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


def step_rk4_closure_vjp(u0, u1bar, h, nu, dt, theta, on_closure=None):
    """(u0bar, thetabar) of one closure-coupled RK4 step. ``on_closure(v, fbar)``,
    if given, sees every (stage velocity, cotangent of its right-hand side)
    pair at which the closure is pulled back."""
    from . import ins

    tbar = np.zeros(n_params())

    def gv(v, fb):
        if on_closure is not None:
            on_closure(v, fb)
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


def rollout_loss_closure_grad(u0, refs, h, nu, dt, theta, on_closure=None):
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
        ubar, tb = step_rk4_closure_vjp(states[s - 1], ubar, h, nu, dt, theta, on_closure)
        tbar += tb
    return ubar, tbar
