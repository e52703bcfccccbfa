"""Layer-by-layer parity of a float32-accumulating closure implementation
against the oracle's layers evaluated on that implementation's own operands.

Every layer's sum is compared element by element with the oracle's float64
sum of the same bfloat16 operands, within gamma_K sum |w||x| (K = the number
of terms: 81 for the 3-channel input, 864 for 32 channels, the number of cells
for weight gradients). Every bfloat16 activation and cotangent is compared
with the oracle's rounding of the float64 value computed from the same
operands: they may differ only where that value lies within its float32 error
bound of a rounding boundary (a flip), and then by at most one bfloat16 step;
the flips are counted. Used with the GPU kernels' exported tensors and, on the
CPU, with a float32 evaluation in torch.
"""
import numpy as np
import torch

import oracle.cnn as C


def check_closure_layers(u, th, mbar, t, ubar, thbar):
    """u, mbar: [B][3][nz][ny][nx]; t: dict of the implementation's tensors in the
    same layout (x0 [B][8], z1, a1, z2, a2 [B][32], gm [B][8], gz2, gz1 [B][32],
    m [B][3]); ubar, thbar: its pullback. Returns (forward flips, backward flips);
    raises AssertionError naming the first tensor outside its bound."""
    def within(name, got, ref, bound):
        err = np.abs(got - ref)
        bad = err > bound
        assert not bad.any(), (name, int(bad.sum()), float(np.max(err / np.maximum(bound, 1e-300))))

    x0 = t["x0"]
    assert np.array_equal(x0[:, :3], C.bf16_round(u)) and not x0[:, 3:].any(), "x0"
    acts = [x0[:, :3]]
    flips_fwd = 0
    for li, (zn, an) in enumerate((("z1", "a1"), ("z2", "a2"))):
        z, e = C.layer_forward(acts[-1], th, li)
        within(zn, t[zn], z, e)
        v = C.gelu(torch.as_tensor(t[zn])).numpy()
        allow = C.flip_allowance(v, C.gelu_f32_error(t[zn]))
        d = np.abs(t[an] - C.bf16_round(v))
        within(an, d, 0.0, allow)
        flips_fwd += int(np.count_nonzero(d))
        acts.append(t[an])
    m, e = C.layer_forward(acts[2], th, 2)
    within("m", t["m"], m, e)

    gm = t["gm"]
    assert np.array_equal(gm[:, :3], C.bf16_round(mbar)) and not gm[:, 3:].any(), "gm"
    cots = [None, None, gm[:, :3]]
    flips_bwd = 0
    for li, (zn, gn) in ((2, ("z2", "gz2")), (1, ("z1", "gz1"))):
        gx, e = C.layer_dgrad(cots[li], th, li)
        d1 = np.abs(C.gelu_grad(t[zn]).numpy())
        e1 = C.gelu_grad_f32_error(t[zn])
        v = gx * C.gelu_grad(t[zn]).numpy()
        ev = e * (d1 + e1) + np.abs(gx) * e1 + C.U32 * (np.abs(gx) + e) * (d1 + e1)
        allow = C.flip_allowance(v, ev)
        d = np.abs(t[gn] - C.bf16_round(v))
        within(gn, d, 0.0, allow)
        flips_bwd += int(np.count_nonzero(d))
        cots[li - 1] = t[gn]
    ub, e = C.layer_dgrad(cots[0], th, 0)
    within("ubar", ubar, ub, e)
    off = 0
    for li in range(3):
        val, bound = C.layer_wgrad(cots[li], acts[li], li)
        within(f"theta layer {li + 1}", thbar[off:off + val.size], val, bound)
        off += val.size
    assert off == thbar.size
    return flips_fwd, flips_bwd
