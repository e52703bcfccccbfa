"""Large-eddy simulation with the learned closure, trained a-posteriori (Sec. 4).

The pipeline the paper describes — DNS data generation, filtering, closure
training by differentiating through the LES time integration, LES evaluation —
on the GPU path of this library:

1. ``dns_snapshots``: decaying-turbulence DNS from a seeded solenoidal field,
   face-filtered to the LES grid every ``every`` steps (``ins_face_filter``).
2. ``train``: Adam on the closure parameters; each iteration unrolls
   ``unroll`` LES steps from filtered-DNS windows of a batch of seeds and
   back-propagates the trajectory MSE through the hand-written step pullback
   (which also returns the closure's parameter gradient), checkpointing inside
   the unroll.
3. ``spectrum_error`` / ``rollout_mse``: LES with no model, with the
   Smagorinsky eddy viscosity (the classical baseline of the paper's appendix)
   and with the trained closure against the filtered DNS, compared by
   mean_k |log E_LES(k) - log E_fDNS(k)| and by the trajectory MSE.

``python -m paper_2604_18536_amd.les`` runs the full-size workload (DNS 512^3
FP32, nu = 1/2000, k0 = 4, dt = 1e-3, 4x face filter to 128^3, LES dt = 4e-3,
unroll 10, batch 4, seeds 10-13 for training and 14 held out).
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import torch

from . import autograd as A
from .solver import Solver

LAYERS = ((3, 32), (32, 32), (32, 3))


def init_params(seed, device="cuda"):
    """Glorot-uniform hidden layers, zero output layer (so the closure starts as m = 0,
    i.e. as the no-closure LES), zero biases; float32, flat parameter layout."""
    g = torch.Generator(device="cpu")
    g.manual_seed(int(seed))
    parts = []
    for li, (ci, co) in enumerate(LAYERS):
        fi, fo = ci * 27, co * 27
        lim = math.sqrt(6.0 / (fi + fo))
        w = (torch.rand(co * ci * 27, generator=g, dtype=torch.float64) * 2 - 1) * lim
        if li == len(LAYERS) - 1:
            w.zero_()
        parts += [w, torch.zeros(co, dtype=torch.float64)]
    return torch.cat(parts).to(torch.float32).to(device)


def dns_snapshots(n_dns, factor, seed, nu, dt, spinup, nsnap, every, k0=4.0, precision="fp32"):
    """Filtered snapshots [nsnap][3][n/f][n/f][n/f] of a DNS started from a seeded field."""
    from synth import turbulence_ic_torch

    s = Solver((n_dns,) * 3, nu=nu, precision=precision)
    u = turbulence_ic_torch((n_dns,) * 3, seed, k0=k0, device=s.device).to(s.dtype).contiguous()
    s.project(u, out=u)
    for _ in range(spinup):
        s.step(u, dt, out=u)
    snaps = []
    for i in range(nsnap):
        snaps.append(s.face_filter(u, factor).clone())
        if i < nsnap - 1:
            for _ in range(every):
                s.step(u, dt, out=u)
    s.close()
    return torch.stack(snaps)


def les_loss(les, theta, data, windows, unroll, dt, checkpoint_every):
    """Trajectory MSE of the closure LES against the filtered DNS over `unroll` steps."""
    u0 = torch.stack([data[b][s0] for b, s0 in windows]).contiguous()
    refs = [torch.stack([data[b][s0 + k] for b, s0 in windows]).contiguous() for k in range(1, unroll + 1)]
    return A.rollout_loss(les, u0, dt, refs, checkpoint_every=checkpoint_every, theta=theta)


def train(data, nu, dt, iters, unroll=10, batch=4, lr=1e-3, seed=0, checkpoint_every=5, log=None):
    """Adam on the closure parameters. data: list (per seed) of snapshot tensors."""
    nc = data[0].shape[-1]
    les = Solver((nc,) * 3, nu=nu, precision="fp32" if data[0].dtype == torch.float32 else "fp64", batch=batch)
    theta = init_params(seed, device=les.device).requires_grad_(True)
    opt = torch.optim.Adam([theta], lr=lr)
    g = torch.Generator(device="cpu")
    g.manual_seed(int(seed) + 1)
    history = []
    for it in range(iters):
        les.set_closure(theta.detach())
        windows = []
        for b in range(batch):
            sd = int(torch.randint(len(data), (1,), generator=g))
            s0 = int(torch.randint(data[sd].shape[0] - unroll, (1,), generator=g))
            windows.append((sd, s0))
        loss = les_loss(les, theta, data, windows, unroll, dt, checkpoint_every)
        opt.zero_grad()
        loss.backward()
        opt.step()
        history.append(float(loss.detach()))
        if log is not None:
            log(it, history[-1])
    les.close()
    return theta.detach(), history


SMAGORINSKY = "smagorinsky"


def _attach(les, closure):
    """closure: None (no model), SMAGORINSKY (eddy viscosity, C_s = 0.17) or CNN parameters."""
    if closure is None:
        return
    if isinstance(closure, str):
        if closure != SMAGORINSKY:
            raise ValueError(f"unknown closure {closure!r}")
        les.set_eddy(0.17)
    else:
        les.set_closure(closure)


def rollout_mse(data, theta, nu, dt, windows, unroll):
    """Trajectory MSE of the LES (closure per _attach) on given windows, no gradient."""
    nc = data[0].shape[-1]
    les = Solver((nc,) * 3, nu=nu, precision="fp32" if data[0].dtype == torch.float32 else "fp64", batch=len(windows))
    _attach(les, theta)
    with torch.no_grad():
        loss = les_loss(les, None, data, windows, unroll, dt, unroll)
    les.close()
    return float(loss)


def spectrum_error(snaps, theta, nu, dt, start, nsteps):
    """LES from snaps[start] for nsteps against snaps[start + nsteps]:
    mean over k = 1..n/2 of |log E_LES(k) - log E_ref(k)|."""
    nc = snaps.shape[-1]
    les = Solver((nc,) * 3, nu=nu, precision="fp32" if snaps.dtype == torch.float32 else "fp64")
    _attach(les, theta)
    u = snaps[start].clone()
    for _ in range(nsteps):
        les.step(u, dt, out=u)
    e = les.energy_spectrum(u)[1:nc // 2 + 1]
    r = les.energy_spectrum(snaps[start + nsteps].contiguous())[1:nc // 2 + 1]
    finite = les.stats(u)[3]
    les.close()
    return float((torch.log(e) - torch.log(r)).abs().mean()), bool(finite)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-dns", type=int, default=512)
    ap.add_argument("--factor", type=int, default=4)
    ap.add_argument("--nu", type=float, default=1.0 / 2000.0)
    ap.add_argument("--dt", type=float, default=1e-3)
    ap.add_argument("--spinup", type=int, default=1000)
    ap.add_argument("--nsnap", type=int, default=251)
    ap.add_argument("--iters", type=int, default=100)
    ap.add_argument("--unroll", type=int, default=10)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--eval-steps", type=int, default=100)
    args = ap.parse_args()
    every = args.factor
    dt_les = every * args.dt
    t0 = time.time()
    train_seeds, test_seed = [10, 11, 12, 13], 14
    data = []
    for sd in train_seeds + [test_seed]:
        data.append(dns_snapshots(args.n_dns, args.factor, sd, args.nu, args.dt, args.spinup, args.nsnap, every))
        print(f"[les] DNS seed {sd} done {time.time() - t0:.0f}s", file=sys.stderr, flush=True)
    t_dns = time.time() - t0
    theta, hist = train(data[:4], args.nu, dt_les, args.iters, args.unroll, args.batch, args.lr,
                        log=lambda i, l: print(f"[les] iter {i} loss {l:.4e}", file=sys.stderr, flush=True) if i % 10 == 0 else None)
    t_train = time.time() - t0 - t_dns
    test = data[4]
    windows = [(0, s0) for s0 in range(0, test.shape[0] - args.unroll, max(1, (test.shape[0] - args.unroll) // 8))][:8]
    res = {
        "train_loss_first": hist[0], "train_loss_last": hist[-1],
        "heldout_mse_no_closure": rollout_mse([test], None, args.nu, dt_les, windows, args.unroll),
        "heldout_mse_closure": rollout_mse([test], theta, args.nu, dt_les, windows, args.unroll),
        "heldout_mse_smagorinsky": rollout_mse([test], SMAGORINSKY, args.nu, dt_les, windows, args.unroll),
    }
    ns = min(args.eval_steps, test.shape[0] - 1)
    res["spectrum_err_no_closure"], f0 = spectrum_error(test, None, args.nu, dt_les, 0, ns)
    res["spectrum_err_closure"], f1 = spectrum_error(test, theta, args.nu, dt_les, 0, ns)
    res["spectrum_err_smagorinsky"], f2 = spectrum_error(test, SMAGORINSKY, args.nu, dt_les, 0, ns)
    res.update({"finite": f0 and f1 and f2, "dns_seconds": round(t_dns, 1), "train_seconds": round(t_train, 1)})
    print(json.dumps(res))


if __name__ == "__main__":
    main()
