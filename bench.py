"""Throughput of the RK4 step of the staggered periodic Navier-Stokes solver on one MI355X.

Workload: 3D periodic decaying turbulence on [0, 2 pi]^3, 256^3 staggered grid,
nu = 1/1600, dt = 1e-3, seeded solenoidal initial field with
E(k) ~ k^4 exp(-2 (k/4)^2) and unit kinetic energy.

`value` is the float64 forward step rate in Mcell-updates/s (one cell update =
one full RK4 step of one cell; inputs resident in HBM). The same line reports
the float64 forward+adjoint rate, the FP32-stencil mode (float32 fields,
float64 divergence/Poisson/projection), Wray's low-storage RK3 step (modes
*_wray3: three stages and solves per step), forward+adjoint with the stage
inputs kept from the forward instead of recomputed (modes *_adj_kept), the
HBM-roofline fraction of each
step and of the dominant kernel (per-kernel durations from HIP events recorded
on the library's stream), and the float64 CPU oracle timed on a bounded
sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 256] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure

CONFIGS = {
    # the benchmark workload: 3D decaying turbulence at 256^3
    "turb256": {"n": 256, "nu": 1.0 / 1600.0, "dt": 1e-3, "k0": 4.0, "seed": 0,
                "modes": "fp64,fp64_adj,fp32,fp32_adj,fp64_adj_kept,fp32_adj_kept,fp64_wray3,fp32_wray3,fp32_all"},
    # the largest single-GPU DNS: 840^3 = 2^3*3*5*7 (mixed-radix FFT), FP64 and FP32 mode
    "dns840": {"n": 840, "nu": 1.0 / 5000.0, "dt": 1e-3, "k0": 8.0, "seed": 3, "modes": "fp64,fp32"},
}
METRIC = "Mcell-updates/s per RK4 step (fwd, fwd+adjoint), FP32 vs FP64, % HBM peak"


def kernel_bytes(name, n, elem, batch=1, scal=8):
    """Algorithmic HBM bytes of one launch: each input read once, each output written once.

    n = (nx, ny, nz); elem = bytes of a velocity value (8 or 4). Pressure-point
    fields are float64 (8 B); the half spectrum holds (nx/2+1) ny nz complex
    float64 values (16 B). With scal = 4 (the all-float32 mode) pressure-point
    values take 4 B and complex values 8 B.
    """
    nx, ny, nz = n
    N = nx * ny * nz * batch
    Ns = (nx // 2 + 1) * ny * nz * batch
    E, S, C = elem, scal, 2 * scal
    v = 3 * E  # one velocity field per cell
    table = {
        "stage_first": 3 * v * N,                 # read u0; write y, w
        "stage_first_rec": 2 * v * N,             # read u0; write w
        "stage": (5 * v + S) * N,                 # read w, p, u0, y; write y, w
        "stage_yw": (5 * v + S) * N,              # read w, p, u0, W2 (y formed from them); write y, w
        "stage_last": (3 * v + S) * N,            # read w, p, y; write y
        "stage_rec": (3 * v + S) * N,             # read w, p, u0; write w
        "wray_stage1": 3 * v * N,                 # read u0; write yacc, w
        "wray_stage2": (3 * v + S) * N,           # read w, p, yacc; write w
        "wray_stage3": (3 * v + S) * N,
        "fft_x_fwd_div": v * N + C * Ns,          # read w; write spectrum
        "fft_x_fwd": S * N + C * Ns,
        "fft_y_fwd": 2 * C * Ns,
        "fft_y_inv": 2 * C * Ns,
        "fft_z_solve": 2 * C * Ns,
        "fft_y_solve": 2 * C * Ns,
        "fft_x_inv": C * Ns + S * N,              # read spectrum; write p
        "apply_projection": (2 * v + S) * N,      # read w, p; write u
        "stage_vjp_first": (4 * v + S) * N,       # read w, p, ybar; write u0bar, ubar
        "stage_vjp": (6 * v + 2 * S) * N,         # read w, p, ybar, ubar', q, u0bar; write u0bar, ubar
        "stage_vjp_last": (5 * v + S) * N,        # read u0, ybar, ubar', q, u0bar; write u0bar
        "rhs": 2 * v * N,
        "rhs_vjp": 3 * v * N,
        # channel grid: conjugate-gradient pressure solve (float64 pressure-point fields)
        "cg_div": (v + S) * N,                    # read w; write r
        "cg_copy": 2 * S * N,
        "cg_init": 3 * S * N,                     # read r; write r, x
        "cg_apply": 5 * S * N,                    # read r, p_old, x; write p, x
        "cg_update": 3 * S * N,                   # read r, p; write r (A p recomputed)
        "wall_projection": (2 * v + S) * N,       # read w, p; write u
        # channel grid: direct solve (x, z FFTs, tridiagonal solves along y)
        "fft_z_fwd": 2 * C * Ns,
        "fft_z_inv": 2 * C * Ns,
        "channel_ysolve": 2 * C * Ns,             # read and write the half spectrum once
    }
    return table.get(name)


def _source_hash(names):
    h = hashlib.sha256()
    for f in names:
        with open(os.path.join(ROOT, "paper_2604_18536_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic_record(kernel, cells):
    """HBM bytes per launch measured with rocprofv3 counters, if still valid for the current source
    and measured on a field of the same number of cells."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        recs = json.load(fh).get(kernel)
    if not recs:
        return None
    for rec in recs if isinstance(recs, list) else [recs]:  # one record per profiled field size
        if rec.get("cells") == cells and rec.get("source_hash") == _source_hash(rec.get("sources", [])):
            return rec.get("bytes_per_launch")
    return None


def time_steps(fn, steps, warmup, solver=None):
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    if solver is not None:
        solver.profile_reset()
        solver.profile(True)
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    torch.cuda.synchronize()
    prof = None
    if solver is not None:
        prof = solver.profile_read()
        solver.profile(False)
    return a.elapsed_time(b) / steps, prof


def run_mode(n, nu, dt, precision, steps, warmup, u0_np, adjoint, scheme="rk4", keep=False, channel=None):
    import torch

    from paper_2604_18536_amd import Solver

    if channel is None:
        s = Solver(n, nu=nu, precision=precision)
    else:
        s = Solver(n, nu=nu, precision=precision, lo=channel["lo"], hi=channel["hi"], bc="walls",
                   pressure=channel["pressure"])
        if channel.get("faces") is not None:
            s.set_y_faces(channel["faces"])
        if channel.get("force") is not None:
            s.set_body_force(channel["force"])
        s.cg_set(rtol=channel["rtol"], maxiter=20000, check_every=channel["check"])
    u0 = torch.as_tensor(u0_np).to(device="cuda", dtype=s.dtype).contiguous()
    s.project(u0, out=u0)
    u1 = torch.empty_like(u0)
    ubar = torch.empty_like(u0)
    gbar = torch.empty_like(u0)
    if adjoint:
        torch.manual_seed(0)
        ubar.copy_(torch.randn_like(u0))
        kept = s.stage_buffers(scheme) if keep else None

        def fn():
            s.step(u0, dt, out=u1, scheme=scheme, keep=kept)
            s.step_vjp(u0, ubar, dt, out=gbar, scheme=scheme, kept=kept)
    else:

        def fn():
            s.step(u0, dt, out=u1, scheme=scheme)
    ms, _ = time_steps(fn, steps, warmup)
    ms_p, prof = time_steps(fn, steps, 1, solver=s)
    if channel is not None and channel["pressure"] == "cg":
        channel["iterations_last_solve"] = s.cg_info()[0]
    ok = s.stats(u1)[3]
    ws = s.workspace_bytes()
    if adjoint and keep:  # the caller-owned stage buffers count as workspace too
        ws += sum(t.numel() * t.element_size() for t in kept)
    s.close()
    return ms, ms_p, prof, ok, ws


CHANNEL = {"n": (256, 256, 256), "nu": 1.0 / 1000.0, "dt": 1e-3, "seed": 5, "rtol": 1e-8, "check": 16,
           "gamma": 1.5, "modes": "fp64,fp64_adj,fp64_adj_kept,fp32,fp64_tanh,fp64_tanh_adj,fp64_cg,fp64_tanh_cg"}
# the paper's turbulent channel (Sec. 6): Re_tau = 180, box 4pi x 2 x 4pi/3, nu = 1/180, driven by
# f = (1, 0, 0), its uniform DNS grid 512 x 1024 x 256; dt from the CFL of the initial field
CHANNEL_DNS = {"n": (512, 1024, 256), "nu": 1.0 / 180.0, "dt": 2e-4, "seed": 7, "rtol": 1e-8, "check": 16,
               "gamma": 1.5, "box": ((0.0, 0.0, 0.0), (4 * math.pi, 2.0, 4 * math.pi / 3)),
               "force": (1.0, 0.0, 0.0), "bulk": 15.6, "noise": 0.1, "modes": "fp64,fp32,fp64_adj_kept"}
# the same channel at the reference DNS resolution 512 x 256 x 256 with tanh stretching in y, first
# cell Delta y+ = 0.49 (Sec. 6): the run the paper's sparse LDL^T factorisation had no memory for
CHANNEL_VK = dict(CHANNEL_DNS, n=(512, 256, 256), seed=8, first_width_plus=0.49)


def channel_timing(steps, warmup, modes=None, cfg=None):
    """Channel flow (no-slip walls at both y ends, x and z periodic) on a 256^3
    grid over [0, 2pi] x [0, 2] x [0, pi]: laminar profile of bulk velocity 1
    plus a 20% solenoidal perturbation, nu = 1/1000, dt = 1e-3. Pressure by the
    direct solve (FFTs along x and z, tridiagonal solves along y); modes *_cg
    by matrix-free CG stopped at a relative residual of 1e-8 (timed over at
    most 2 steps after 1 warmup step). Modes *_tanh: the tanh-stretched y grid
    (gamma = 1.5, cells 3x finer at the walls than in the centre)."""
    import synth as S

    cfg = dict(CHANNEL if cfg is None else cfg)
    n = cfg["n"]
    lo, hi = S.channel_box(n) if "box" not in cfg else (list(cfg["box"][0]), list(cfg["box"][1]))
    u0 = S.channel_ic(n, cfg["seed"], bulk=cfg.get("bulk", 1.0), noise=cfg.get("noise", 0.2), box=(lo, hi))
    print(f"[bench] channel initial field ready {n}", file=sys.stderr, flush=True)
    ncell = n[0] * n[1] * n[2]
    box = "x".join(f"{v:.4g}" for v in hi)
    force = f", body force {tuple(cfg['force'])}" if cfg.get("force") else ""
    out = {"workload": f"channel {n[0]}x{n[1]}x{n[2]}, box {box}, walls at y=0,{hi[1]:g}, "
                       f"nu=1/{round(1 / cfg['nu'])}, dt={cfg['dt']}{force}, direct pressure solve "
                       f"(CG rtol={cfg['rtol']:g} in *_cg modes)",
           "modes": {}, "kernels": {}}
    for mode in (modes or cfg["modes"]).split(","):
        precision = "fp64" if mode.startswith("fp64") else "fp32"
        adjoint = "_adj" in mode
        cg = mode.endswith("_cg")
        ch = {"lo": lo, "hi": hi, "rtol": cfg["rtol"], "check": cfg["check"], "pressure": "cg" if cg else "fft",
              "force": cfg.get("force")}
        if "_tanh" in mode:
            ch["faces"] = S.tanh_faces(n[1], lo[1], hi[1], cfg["gamma"])
        if cfg.get("first_width_plus"):  # stretched in every mode, first cell in wall units (u_tau = 1)
            gam = S.tanh_gamma(n[1], hi[1] - lo[1], cfg["first_width_plus"] * cfg["nu"])
            ch["faces"] = S.tanh_faces(n[1], lo[1], hi[1], gam)
            out["tanh_gamma"] = round(gam, 6)
        k_steps, k_warm = (min(steps, 2), min(warmup, 1)) if cg else (steps, warmup)
        print(f"[bench] channel {mode} starts", file=sys.stderr, flush=True)
        ms, ms_p, prof, ok, ws = run_mode(n, cfg["nu"], cfg["dt"], precision, k_steps, k_warm, u0, adjoint, "rk4",
                                          mode.endswith("_kept"), ch)
        elem = 8 if precision == "fp64" else 4
        alg = sum(kernel_bytes(k, n, elem) * c for k, (c, t) in prof.items() if kernel_bytes(k, n, elem))
        rec = {
            "mcell_per_s": round(ncell / (ms * 1e-3) / 1e6, 3),
            "ms_per_step": round(ms, 3),
            "steps": k_steps,
            "pressure": ch["pressure"],
            "alg_bytes_per_cell": round(alg / k_steps / ncell, 1),
            "hbm_frac": round(alg / k_steps / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
            "finite": bool(ok),
            "workspace_gb": round(ws / 1e9, 3),
        }
        if cg:
            applies = prof.get("cg_apply", (0, 0.0))[0] / k_steps
            solves = prof.get("cg_init", (0, 0.0))[0] / k_steps
            rec["cg_solves_per_step"] = solves
            rec["cg_iterations_per_solve"] = round(applies / solves, 1) if solves else None
            rec["cg_iterations_last_solve"] = ch["iterations_last_solve"]
        out["modes"][mode] = rec
        out["kernels"][mode] = {
            k: {"launches_per_step": c / k_steps, "avg_ms": round(t / c, 5),
                "gbs": round(kernel_bytes(k, n, elem) / (t / c * 1e-3) / 1e9, 1) if kernel_bytes(k, n, elem) else None}
            for k, (c, t) in prof.items()
        }
        print(f"[bench] channel {mode}: {out['modes'][mode]}", file=sys.stderr, flush=True)
    kp = out["kernels"]["fp64"] if "fp64" in out["kernels"] else next(iter(out["kernels"].values()))
    dom = max(kp, key=lambda k: kp[k]["avg_ms"] * kp[k]["launches_per_step"])
    b = kernel_bytes(dom, n, 8)
    achieved = b / (kp[dom]["avg_ms"] * 1e-3) / 1e9
    out["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                       "traffic": _traffic_record("channel:" + dom, ncell),
                       "alg_bytes_per_launch": b, "avg_ms": kp[dom]["avg_ms"]}
    return out


def stream_copy_gbs(nbytes=2 << 30, reps=10):
    """Bandwidth of the library's plain copy kernel (read + write bytes / time)."""
    import torch

    from paper_2604_18536_amd import Solver

    s = Solver((8, 8, 8))
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    s.stream_copy(a, b)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        s.stream_copy(a, b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    s.close()
    del a, b
    return 2 * nbytes / (ms * 1e-3) / 1e9


def les_closure_timing(steps, warmup):
    """LES with the learned closure (128^3, batch 4, FP32, nu = 1/2000, dt = 4e-3)
    next to the 512^3 FP32 DNS step it stands in for (4 DNS steps of dt = 1e-3
    per LES step, per field)."""
    import torch

    import synth as S
    from paper_2604_18536_amd import Solver
    from paper_2604_18536_amd.les import init_params

    nu = 1.0 / 2000.0
    les = Solver((128, 128, 128), nu=nu, precision="fp32", batch=4)
    th = init_params(0)
    th[30304:30304 + 2592].uniform_(-0.02, 0.02)  # a non-zero output layer so the closure does work
    les.set_closure(th)
    u = torch.stack([S.turbulence_ic_torch((128,) * 3, seed=10 + b, k0=4.0).float() for b in range(4)]).contiguous()
    les.project(u, out=u)
    u1 = torch.empty_like(u)
    ubar = torch.randn_like(u)
    g = torch.empty_like(u)
    ms_fwd, prof_fwd = time_steps(lambda: les.step(u, 4e-3, out=u1), steps, warmup, solver=les)
    nadj = max(2, steps // 4)
    ms_adj, prof_adj = time_steps(lambda: (les.step(u, 4e-3, out=u1), les.step_vjp(u, ubar, 4e-3, out=g)), nadj, 1,
                                  solver=les)
    # the classical baseline closure on the same LES: Smagorinsky eddy viscosity (C_s = 0.17)
    les.set_closure(None)
    les.set_eddy(0.17)
    ms_smag, _ = time_steps(lambda: les.step(u, 4e-3, out=u1), steps, warmup)
    ms_smag_adj, _ = time_steps(lambda: (les.step(u, 4e-3, out=u1), les.step_vjp(u, ubar, 4e-3, out=g)), nadj, 1)
    les.close()
    ncl = 4 * 128 ** 3
    conv2 = prof_fwd.get("cnn_conv2")
    conv2_ms = conv2[1] / conv2[0] if conv2 else None
    cnn_kernels = {k: {"avg_ms": round(t / c, 4), "per_step": round(c / nadj, 2)}
                   for k, (c, t) in prof_adj.items() if k.startswith("cnn_")}
    dns = Solver((512, 512, 512), nu=nu, precision="fp32")
    v = S.turbulence_ic_torch((512,) * 3, seed=10, k0=4.0).float().contiguous()
    dns.project(v, out=v)
    ms_dns, _ = time_steps(lambda: dns.step(v, 1e-3, out=v), max(2, steps // 4), 1)
    dns.close()
    cnn_ms = sum(t for k, (c, t) in prof_fwd.items() if k.startswith("cnn_")) / steps
    return {
        "workload": "LES 128^3 x batch 4, FP32, CNN closure 3-32-32-3 (bf16 MFMA), dt=4e-3; vs DNS 512^3 FP32 dt=1e-3",
        "les_step_ms": round(ms_fwd, 3),
        "les_closure_ms_per_step": round(cnn_ms, 3),
        "les_step_plus_vjp_ms": round(ms_adj, 3),
        "dns512_step_ms": round(ms_dns, 3),
        "les_smagorinsky_step_ms": round(ms_smag, 3),
        "les_smagorinsky_step_plus_vjp_ms": round(ms_smag_adj, 3),
        "speedup_vs_dns_same_time_span": round(4 * 4 * ms_dns / ms_fwd, 1),
        # layer 2 (32 -> 32, 3x3x3) is the MFMA-bound contraction: 2 * 864 * 32 flop per cell
        "conv2_mfma": None if conv2_ms is None else {
            "bound": "mfma", "achieved": round(2 * 864 * 32 * ncl / (conv2_ms * 1e-3) / 1e12, 1),
            "peak": 2500.0, "unit": "TFLOP/s", "avg_ms": round(conv2_ms, 4)},
        "cnn_kernels_fwd_and_vjp": cnn_kernels,
    }


def small_grid_timing(steps):
    """2D grids that live in the last-level cache (launch-bound): eager steps
    against the same steps replayed from a recorded HIP graph, and the
    checkpointed 50-step trajectory-loss gradient on 256^2."""
    import torch

    import synth as S
    from paper_2604_18536_amd import Solver
    from paper_2604_18536_amd import autograd as A
    from paper_2604_18536_amd.graphs import StepGraph

    out = {}
    cases = {"taylor_green_64x64_fp64": ((64, 64), "fp64", 0.01, 1e-3, S.taylor_green_2d(64)),
             "turbulence_256x256_fp32": ((256, 256), "fp32", 5e-4, 2e-3, S.turbulence_ic((256, 256), seed=1, k0=4.0))}
    for name, (n, prec, nu, dt, u0) in cases.items():
        s = Solver(n, nu=nu, precision=prec)
        u = torch.as_tensor(u0).to(device="cuda", dtype=s.dtype).contiguous()
        ms_eager, _ = time_steps(lambda: s.step(u, dt, out=u), steps, 3)
        g = StepGraph(s, u, dt, steps)
        ms_graph, _ = time_steps(g.replay, 3, 1)
        ms_graph /= steps
        out[name] = {"eager_ms_per_step": round(ms_eager, 4), "graph_ms_per_step": round(ms_graph, 4),
                     "graph_mcell_per_s": round(n[0] * n[1] / (ms_graph * 1e-3) / 1e6, 1)}
        s.close()
    # 50-step trajectory loss and its gradient (checkpoint every 10), 256^2 FP32
    n = (256, 256)
    s = Solver(n, nu=5e-4, precision="fp32")
    u0 = torch.as_tensor(S.turbulence_ic(n, seed=1, k0=4.0)).to(device="cuda", dtype=torch.float32).contiguous()
    refs = [torch.zeros_like(u0) for _ in range(50)]

    def grad():
        t = u0.clone().requires_grad_(True)
        A.rollout_loss(s, t, 2e-3, refs, checkpoint_every=10).backward()
    ms_grad, _ = time_steps(grad, 3, 1)
    out["loss_gradient_50_steps_256x256_fp32_ms"] = round(ms_grad, 3)
    s.close()
    return out


def kernel_table(prof, n, elem, steps, scal=8):
    """Per-kernel launches per step, average duration, algorithmic GB/s and its fraction of the HBM peak."""
    out = {}
    for k, (c, t) in prof.items():
        b = kernel_bytes(k, n, elem, scal=scal)
        gbs = b / (t / c * 1e-3) / 1e9 if b else None
        out[k] = {"launches_per_step": c / steps, "avg_ms": round(t / c, 5),
                  "gbs": None if gbs is None else round(gbs, 1),
                  "frac": None if gbs is None else round(gbs / HBM_PEAK_GBS, 4)}
    return out


def size_sweep(sizes, steps, warmup):
    """The RK4 step of 3D decaying turbulence at larger grids, FP64 and FP32 mode, with
    per-kernel algorithmic GB/s against the 8 TB/s HBM peak: 512^3 (nu = 1/2000, k0 = 4,
    the DNS of the closure's training data) and 840^3 (nu = 1/5000, k0 = 8, the paper's
    largest single-GPU DNS size). Initial fields are built on the GPU."""
    import torch

    import synth as S

    out = {}
    for n1 in sizes:
        cfg = CONFIGS["dns840"] if n1 == 840 else {"nu": 1.0 / 2000.0, "dt": 1e-3, "k0": 4.0, "seed": 10}
        n = (n1,) * 3
        ncell = n1 ** 3
        u0 = S.turbulence_ic_torch(n, seed=cfg["seed"], k0=cfg["k0"], device="cuda")
        print(f"[bench] size {n1}^3 initial field ready", file=sys.stderr, flush=True)
        rec = {"nu": cfg["nu"], "dt": cfg["dt"], "k0": cfg["k0"], "modes": {}}
        for precision in ("fp64", "fp32"):
            ms, ms_p, prof, ok, ws = run_mode(n, cfg["nu"], cfg["dt"], precision, steps, warmup, u0, False)
            elem = 8 if precision == "fp64" else 4
            kt = kernel_table(prof, n, elem, steps)
            alg = sum(kernel_bytes(k, n, elem) * c for k, (c, t) in prof.items() if kernel_bytes(k, n, elem))
            dom = max(kt, key=lambda k: kt[k]["avg_ms"] * kt[k]["launches_per_step"])
            rec["modes"][precision] = {
                "mcell_per_s": round(ncell / (ms * 1e-3) / 1e6, 2),
                "ms_per_step": round(ms, 3),
                "alg_bytes_per_cell": round(alg / steps / ncell, 1),
                "hbm_frac": round(alg / steps / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
                "finite": bool(ok),
                "workspace_gb": round(ws / 1e9, 3),
                "dominant": {"kernel": dom, "frac": kt[dom]["frac"],
                             "traffic": _traffic_record(dom, ncell) if precision == "fp64" else None},
                "kernels": kt,
            }
            print(f"[bench] size {n1}^3 {precision}: {rec['modes'][precision]['mcell_per_s']} Mcell/s",
                  file=sys.stderr, flush=True)
        out[f"{n1}^3"] = rec
        del u0
        torch.cuda.empty_cache()
    return out


def precision_study(steps=200):
    """FP32 mode and the all-float32 comparison mode against FP64 on the benchmark
    trajectory (256^3 decaying turbulence, nu = 1/1600, dt = 1e-3, from the same
    float32-rounded field): relative L2 velocity error, kinetic-energy error and the
    largest discrete divergence (in float64) of each stored field."""
    import torch

    import synth as S
    from paper_2604_18536_amd import Solver

    n, nu, dt = (256, 256, 256), 1.0 / 1600.0, 1e-3
    u0 = S.turbulence_ic(n, seed=0, k0=4.0).astype("float32")
    s64, s32, s32a = Solver(n, nu=nu), Solver(n, nu=nu, precision="fp32"), Solver(n, nu=nu, precision="fp32_all")
    a = torch.as_tensor(u0).cuda().double()
    b = torch.as_tensor(u0).cuda()
    c = b.clone()
    rows = {}
    for k in range(1, steps + 1):
        s64.step(a, dt, out=a)
        s32.step(b, dt, out=b)
        s32a.step(c, dt, out=c)
        if k in (1, 10, 50, 100, 200):
            ke64 = 0.5 * float((a * a).sum(0).mean())
            row = {"fp64_max_div": float(s64.divergence(a).abs().max())}
            for name, v in (("fp32", b), ("fp32_all", c)):
                vd = v.double()
                row[name] = {"rel_l2": float((vd - a).norm() / a.norm()),
                             "ke_rel": abs(0.5 * float((vd * vd).sum(0).mean()) - ke64) / ke64,
                             "max_div": float(s64.divergence(vd).abs().max())}
            rows[str(k)] = row
    for s_ in (s64, s32, s32a):
        s_.close()
    return {"workload": "256^3 decaying turbulence, nu=1/1600, dt=1e-3, 200 RK4 steps from the same float32 field",
            "max_u0": float(abs(u0).max()), "steps": rows}


def cpu_baseline(n, nu, dt, u0_np, budget_s=30.0):
    """The float64 numpy oracle, as written, on the host: RK4 steps of the same field."""
    import oracle as O
    import synth as S

    h = S.spacing(n)
    ncell = n[0] * n[1] * n[2]
    t0 = time.perf_counter()
    u = O.step_rk4(u0_np, h, nu, dt)
    t1 = time.perf_counter()
    steps = 1
    if (t1 - t0) * 2 < budget_s:
        u = O.step_rk4(u, h, nu, dt)
        steps = 2
    t = time.perf_counter() - t0
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), None)
    except OSError:
        pass
    return {
        "value": round(ncell * steps / t / 1e6, 4),
        "unit": "Mcell/s",
        "cores": 1,
        "kind": "oracle",
        "host_cpu": model,
        "host_nproc": os.cpu_count(),
        "sample": f"{steps} float64 RK4 step(s) of the {n[0]}x{n[1]}x{n[2]} field (numpy, single-threaded "
                  f"elementwise and FFT), {t:.1f} s",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="turb256",
                    choices=sorted(CONFIGS) + ["channel256", "channel_dns", "channel_vk"])
    ap.add_argument("--n", type=int, default=None, help="override the grid size of the config")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-les", action="store_true", help="skip the closure-LES and small-grid timings")
    ap.add_argument("--no-channel", action="store_true", help="skip the channel (wall-bounded) timing")
    ap.add_argument("--modes", default=None)
    ap.add_argument("--sizes", default="512,840", help="larger grids for the per-kernel table ('' to skip)")
    ap.add_argument("--no-precision", action="store_true", help="skip the 256^3 precision study")
    args = ap.parse_args()
    if args.config in ("channel256", "channel_dns", "channel_vk"):
        return channel_main(args)
    cfg = dict(CONFIGS[args.config])
    if args.n is not None:
        cfg["n"] = args.n
    if args.modes is None:
        args.modes = cfg["modes"]
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested); multi-GPU runs are not part "
              "of this build.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth as S

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    n = (cfg["n"],) * 3
    nu, dt = cfg["nu"], cfg["dt"]
    ncell = n[0] * n[1] * n[2]
    if cfg["n"] <= 256:
        u0 = S.turbulence_ic(n, seed=cfg["seed"], k0=cfg["k0"])
    else:  # too large for numpy in reasonable time: same construction on the GPU
        u0 = S.turbulence_ic_torch(n, seed=cfg["seed"], k0=cfg["k0"], device="cuda")
        args.no_cpu = True
    print(f"[bench] initial field ready {n}", file=sys.stderr, flush=True)

    copy_gbs = stream_copy_gbs()
    print(f"[bench] streaming copy {copy_gbs:.0f} GB/s", file=sys.stderr, flush=True)
    modes = {}
    kernels = {}
    for mode in args.modes.split(","):
        precision = "fp64" if mode.startswith("fp64") else ("fp32_all" if mode.startswith("fp32_all") else "fp32")
        scal = 4 if precision == "fp32_all" else 8
        adjoint = mode.endswith("_adj") or mode.endswith("_adj_kept")
        keep = mode.endswith("_adj_kept")
        scheme = "wray3" if "_wray3" in mode else "rk4"
        ms, ms_p, prof, ok, ws = run_mode(n, nu, dt, precision, args.steps, args.warmup, u0, adjoint, scheme, keep)
        elem = 8 if precision == "fp64" else 4
        alg = 0
        for name, (cnt, tot) in prof.items():
            b = kernel_bytes(name, n, elem, scal=scal)
            if b is not None:
                alg += b * cnt
        alg_per_step = alg / args.steps
        modes[mode] = {
            "mcell_per_s": round(ncell / (ms * 1e-3) / 1e6, 2),
            "ms_per_step": round(ms, 4),
            "ms_per_step_with_kernel_events": round(ms_p, 4),
            "alg_bytes_per_cell": round(alg_per_step / ncell, 1),
            "hbm_frac": round(alg_per_step / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
            "finite": bool(ok),
            "workspace_gb": round(ws / 1e9, 3),
        }
        kernels[mode] = {
            name: {
                "launches_per_step": cnt / args.steps,
                "avg_ms": round(tot / cnt, 5),
                "gbs": (round(kernel_bytes(name, n, elem, scal=scal) / (tot / cnt * 1e-3) / 1e9, 1)
                        if kernel_bytes(name, n, elem, scal=scal) else None),
            }
            for name, (cnt, tot) in prof.items()
        }
        print(f"[bench] {mode}: {modes[mode]}", file=sys.stderr, flush=True)

    main_mode = "fp64" if "fp64" in modes else next(iter(modes))
    kprof = kernels[main_mode]
    dom = max(kprof, key=lambda k: kprof[k]["avg_ms"] * kprof[k]["launches_per_step"])
    elem = 8 if main_mode.startswith("fp64") else 4
    dom_bytes = kernel_bytes(dom, n, elem)
    achieved = dom_bytes / (kprof[dom]["avg_ms"] * 1e-3) / 1e9
    roofline = {
        "bound": "hbm",
        "kernel": dom,
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": _traffic_record(dom, ncell),
        "alg_bytes_per_launch": dom_bytes,
        "avg_ms": kprof[dom]["avg_ms"],
        "frac_of_copy": round(achieved / copy_gbs, 4),  # against the measured streaming-copy rate
    }
    cpu = None if args.no_cpu else cpu_baseline(n, nu, dt, u0)
    les = None if args.no_les or args.config != "turb256" else les_closure_timing(args.steps, args.warmup)
    small = None if args.no_les or args.config != "turb256" else small_grid_timing(50)
    channel = None if args.no_channel or args.config != "turb256" else channel_timing(args.steps, args.warmup)
    precision = None if args.no_precision or args.config != "turb256" else precision_study()
    sizes = None
    if args.sizes and args.config == "turb256":
        sizes = size_sweep([int(v) for v in args.sizes.split(",")], min(args.steps, 10), min(args.warmup, 2))
    ms = modes[main_mode]["ms_per_step"]
    line = {
        "metric": METRIC,
        "value": modes[main_mode]["mcell_per_s"],
        "unit": "Mcell/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"3D periodic decaying turbulence {n[0]}^3 staggered grid, nu=1/{round(1 / nu)}, dt={dt}, "
                        f"E(k)~k^4 exp(-2(k/{cfg['k0']:g})^2), unit KE; {main_mode} RK4 step",
            "grid": list(n),
            "nu": nu,
            "dt": dt,
        },
        "roofline": roofline,
        "stream_copy_gbs": round(copy_gbs, 1),
        "les_closure": les,
        "small_grids": small,
        "channel": channel,
        "precision_256": precision,
        "sizes": sizes,
        "cpu_baseline": cpu,
        "modes": modes,
        "kernels": kernels,
    }
    print(json.dumps(line))


def channel_main(args):
    """Bench line of the channel workload alone (for its profiles)."""
    import torch

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested)", file=sys.stderr)
        sys.exit(2)
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    copy_gbs = stream_copy_gbs()
    presets = {"channel256": None, "channel_dns": CHANNEL_DNS, "channel_vk": CHANNEL_VK}
    ch = channel_timing(args.steps, args.warmup, args.modes, presets[args.config])
    ch["roofline"]["frac_of_copy"] = round(ch["roofline"]["achieved"] / copy_gbs, 4)
    main_mode = "fp64" if "fp64" in ch["modes"] else next(iter(ch["modes"]))
    line = {
        "metric": METRIC,
        "value": ch["modes"][main_mode]["mcell_per_s"],
        "unit": "Mcell/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ch["modes"][main_mode]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_mode.startswith("fp64") else "f32",
        "data": "synthetic",
        "config": {"workload": ch["workload"] + f"; {main_mode} RK4 step"},
        "roofline": ch["roofline"],
        "stream_copy_gbs": round(copy_gbs, 1),
        "cpu_baseline": None,
        "modes": ch["modes"],
        "kernels": ch["kernels"],
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
