#!/usr/bin/env python
"""Benchmark of the lensless RF volumetric rendering hot path on one MI355X.

A step is one full training step of the 2^20-point MLP workload: lensless
samples, the 8 x 256 FP32 SDF network with its reflectiveness head (and the
detached origin occupancies), signal tracing with lensless alpha blending,
the matched filter, the L2 heatmap loss, all adjoints (matched filter,
signal tracing, transmittance scan, network double backward) and AdamW.

The metric counts render terms: one (point, measurement, frequency) triple
per pass, four passes per step (signal tracing forward and adjoint, matched
filter forward and adjoint), 2^20 x 1024 x 128 terms each.

Prints one JSON line (rank 0).  Only --gpus 1 is supported: the path runs on
one GPU (sharding the points across GPUs would all-reduce the signal, its
gradient and the network gradient each step; that is not built).
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3         # MI355X FP32 MFMA peak (dense)
# FP32 vector issue rate this build can reach: 256 CU x 4 SIMD x 16 lanes x 2
# FLOP per FMA x 2.4 GHz.  The 157.3 TFLOP/s vector figure counts packed FP32
# instructions, which every kernel here is compiled without.
PEAK_FP32_VALU_TFLOPS = 78.6


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "mlp_backward_train_mlp_box_hbm_counters.md")
# the network kernels' source: the counters stand while it is unchanged (the
# shared header holds no network kernel code)
NETWORK_SOURCES = [os.path.join(ROOT, "paper_2605_29097_amd", "csrc", "mlp.hip")]


def network_digest() -> str:
    """sha256 over the code of the network kernels' sources: comments and
    blank lines left out, so a change of wording keeps the counters, a change
    of code drops them."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in NETWORK_SOURCES:
        with open(f) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        code = "\n".join(line.rstrip() for line in src.splitlines() if line.strip())
        h.update(code.encode())
    return h.hexdigest()


def mlp_backward_flop(cfg) -> int:
    """Algorithmic FLOP per point of the training backward of the network
    (2 per multiply-add, unpadded shapes): per trunk layer the tangent product
    and two weight-gradient products, per layer above the first the adjoint
    product H_bar = Z_bar W (the tangent's adjoint comes from the forward's
    gradient sweep); the head's forward recompute, adjoint and weight
    gradients; the scalar output layers are not counted."""
    W, L, HW, HL = cfg.width, cfg.n_layers, cfg.head_width, cfg.head_layers
    fin = [3 + 6 * cfg.pe_octaves] + [W] * (L - 1)
    trunk = sum(2 * f * W for f in fin)                 # tangent
    trunk += sum(2 * 2 * f * W for f in fin)            # W_bar = Z_bar^T H + Zdot_bar^T Hdot
    trunk += sum(2 * W * W for _ in fin[1:])            # H_bar of the layer below
    hin = [W] + [HW] * (HL - 1)
    head = sum(2 * f * HW for f in hin)                 # forward recompute
    head += sum(2 * f * HW for f in hin)                # weight gradients
    head += sum(2 * f * HW for f in hin)                # adjoints of the head inputs (into the trunk)
    return trunk + head


def moment_flop_per_pair(K: int) -> int:
    """FLOP per (measurement, point) pair of the moment kernel: per order one
    recurrence FMA and one complex-by-real multiply-add (2 FMA)."""
    return 6 * K


def measured_traffic():
    """HBM bytes per call of the network training backward from the committed
    counter summary (FETCH_SIZE and WRITE_SIZE runs, scaled by a plain copy),
    or None when the network's sources changed after the counters were taken."""
    try:
        txt = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    vals = {}
    for line in txt.splitlines():
        if ":" in line and line.strip().startswith(("traffic_bytes_per_launch", "source_sha256")):
            k, v = line.strip().split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_sha256") != network_digest() or "traffic_bytes_per_launch" not in vals:
        return None
    return float(vals["traffic_bytes_per_launch"])


def make_inputs(cfg, dev):
    """Seeded network weights and the measured signal of the box scene."""
    import numpy as np
    import torch
    from synth import MLPSpec, mlp_init
    spec = MLPSpec(n_layers=cfg.n_layers, width=cfg.width, pe_octaves=cfg.pe_octaves,
                   head_width=cfg.head_width, head_layers=cfg.head_layers, beta=cfg.beta,
                   centre=tuple(cfg.cube_centre), half_size=cfg.cube_side / 2)
    params = torch.from_numpy(mlp_init(spec, cfg.seed)).to(dev)
    # oracle render of the analytic box + 10 dB noise, written once by
    # tests/golden/make_box_target.py
    data = np.load(os.path.join(ROOT, "tests", "golden", "box_target.npz"))
    noisy = data["noisy"]
    target = torch.from_numpy(np.stack([noisy.real, noisy.imag], -1).astype(np.float32)).to(dev)
    return params, target


def host_threads() -> int:
    """Host cores this process may use: OMP_NUM_THREADS when the environment
    sets it (a shared host's share), else the CPUs of the affinity mask."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return int(os.environ.get("OMP_NUM_THREADS", n))


def cpu_baseline(cfg, threads=None):
    """The FP64 oracle timed on this host on a bounded sample of the workload,
    scaled with the thread count so that it takes about the same time."""
    import numpy as np
    threads = threads or host_threads()
    os.environ["OMP_NUM_THREADS"] = str(threads)
    from oracle import render as orc
    from synth import Box, freq_grid, line_points, planar_aperture, scene_fields
    f0, df = freq_grid(cfg.n_freq)
    tx = planar_aperture(*cfg.ap, cfg.pitch).astype(np.float64)
    xyz, _ = line_points(cfg.cube_centre, cfg.cube_side, cfg.lines[0], cfg.lines[1], cfg.n_z)
    sdf, grad, refl = scene_fields(Box(cfg.cube_centre, (0.04, 0.03, 0.02), 0.8), xyz)
    xyz = xyz.astype(np.float64)
    F = orc.Fields(sdf=sdf.astype(np.float64), grad=grad.astype(np.float64), refl=refl.astype(np.float64),
                   s=cfg.s, amp=1.0)
    n_pts = xyz.shape[0] * xyz.shape[1]
    rng = np.random.default_rng(0)
    sel = np.arange(2 * threads)                               # measurements for point reductions
    k_rays = min(16, threads)
    rays = np.arange(0, xyz.shape[0], xyz.shape[0] // k_rays)[:k_rays]  # rays for frequency reductions
    q = xyz[rays].reshape(-1, 3)
    ap_sel = orc.Aperture(tx=tx[sel], f0=f0, df=df, n_freq=cfg.n_freq)
    ap_all = orc.Aperture(tx=tx, f0=f0, df=df, n_freq=cfg.n_freq)
    gs = rng.normal(size=(tx.shape[0], cfg.n_freq)) + 1j * rng.normal(size=(tx.shape[0], cfg.n_freq))
    terms = 0
    t0 = time.perf_counter()
    s = orc.render(ap_sel, xyz, F)                                        # forward, all points
    terms += n_pts * len(sel) * cfg.n_freq
    z, P = orc.mf(ap_all, q, gs)                                          # MF, sampled rays
    terms += q.shape[0] * tx.shape[0] * cfg.n_freq
    zz = rng.normal(size=n_pts) + 1j * rng.normal(size=n_pts)
    orc.mf_adjoint(ap_sel, xyz.reshape(-1, 3), zz, np.abs(zz), rng.normal(size=n_pts))
    terms += n_pts * len(sel) * cfg.n_freq                                # MF adjoint, all points
    Fr = orc.Fields(sdf=F.sdf[rays], grad=F.grad[rays], refl=F.refl[rays], s=cfg.s, amp=1.0)
    orc.render_adjoint(ap_all, xyz[rays], Fr, gs)                         # adjoint, sampled rays
    terms += q.shape[0] * tx.shape[0] * cfg.n_freq
    dt = time.perf_counter() - t0
    sample = (f"FP64 oracle (C + OpenMP, one sin/cos per term): signal tracing and matched-filter "
              f"adjoint over all {n_pts} points for {len(sel)} measurements, matched filter and "
              f"signal-tracing adjoint over {len(rays)} whole rays ({q.shape[0]} points) for all "
              f"{tx.shape[0]} measurements; {terms:.3e} terms in {dt:.1f} s")
    return dict(value=terms / dt, unit="terms/s", cores=threads, kind="oracle", sample=sample)


def cpu_baseline_both(cfg):
    """The oracle on all host cores available to this process, and on one
    core in a child process (OpenMP fixes its thread count when the library
    loads; the child touches no GPU)."""
    import subprocess
    full = cpu_baseline(cfg)
    code = ("import json, sys; sys.path.insert(0, %r); import bench; "
            "from paper_2605_29097_amd.train import StepConfig; "
            "print(json.dumps(bench.cpu_baseline(StepConfig(), threads=1)))" % ROOT)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=600)
    one = json.loads(r.stdout.strip().splitlines()[-1]) if r.returncode == 0 else None
    host = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    full["host_cpus"] = host
    full["single_core"] = None if one is None else {"value": one["value"], "unit": one["unit"], "cores": 1,
                                                    "sample": one["sample"]}
    return full


def probe(tr, which, reps):
    """Run one pass (a term pass or the network training backward) `reps`
    times on the workload's inputs."""
    import torch
    from paper_2605_29097_amd import rfvr as R
    c = tr.cfg
    xyz, u, origin = tr.samples()
    res = tr.reserve(xyz.shape[0] * xyz.shape[1])
    f, grad, a = R.mlp_forward(tr.net, xyz, reserve=res)
    g_f, g_g, g_a = torch.randn_like(f), torch.randn_like(grad), torch.randn_like(a)
    if which != "mlp_bwd":
        sm = R.Samples(xyz=xyz)
        fl = R.Fields(sdf=f.view(xyz.shape[:2]), grad=grad.view(*xyz.shape[:2], 3), refl=a.view(xyz.shape[:2]),
                      s=c.s, amp=1.0)
        sig = R.render_forward(tr.ap, sm, fl)
        z, p = R.mf_forward(tr.ap, xyz, sig)
        g_p = torch.randn_like(p)
        g_sig = R.mf_backward(tr.ap, xyz, z, p, g_p)
    torch.cuda.synchronize()
    for _ in range(reps):
        if which == "mlp_bwd":
            R.mlp_backward(tr.net, xyz, g_f, g_g, g_a, out=tr.g, reserve=res)
        elif which == "render_fwd":
            R.render_forward(tr.ap, sm, fl)
        elif which == "mf_fwd":
            R.mf_forward(tr.ap, xyz, sig)
        elif which == "mf_bwd":
            R.mf_backward(tr.ap, xyz, z, p, g_p)
        else:
            R.render_backward(tr.ap, sm, fl, g_sig)
    torch.cuda.synchronize()
    print(json.dumps({"probe": which, "reps": reps}))


def grid_points(centre, half, n):
    """Cell centres of an n^3 grid over the cube, float32 [n^3, 3] (x fastest)."""
    import numpy as np
    ax = [c - half + (np.arange(n) + 0.5) * (2 * half / n) for c in centre]
    z, y, x = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], 1).astype(np.float32)


def surface_points(f, centre, half):
    """Points of the zero level set of f sampled on the n^3 grid of
    grid_points (f indexed [z][y][x]): on every grid edge whose end values
    change sign, the linear interpolation of the crossing -- the vertices
    marching cubes places on that grid.  float64 [m, 3]."""
    import numpy as np
    f = np.asarray(f, np.float64)
    n = f.shape[0]
    h = 2 * half / n
    lo = np.asarray(centre, np.float64) - half + 0.5 * h
    out = []
    for ax in range(3):                     # array axis 0 = z, 1 = y, 2 = x
        a = np.take(f, np.arange(n - 1), axis=ax)
        b = np.take(f, np.arange(1, n), axis=ax)
        hit = (a < 0) != (b < 0)
        idx = np.argwhere(hit)
        fa, fb = a[hit], b[hit]
        t = fa / (fa - fb)
        pts = idx.astype(np.float64)
        pts[:, ax] += t
        out.append(lo[None, ::-1] + pts * h)              # (z, y, x) order
    return np.concatenate(out, 0)[:, ::-1].copy()          # -> (x, y, z)


def chamfer(a, b, n_sample=5000, seed=0):
    """Chamfer distance between point sets (App. C, Training Setup metrics):
    n_sample seeded samples per side, CD = mean_a min_b |a-b|^2 + mean_b
    min_a |a-b|^2 (the squared form), and the symmetric mean of the plain
    nearest distances.  Returns (cd_squared, cd_mean) in m^2 and m."""
    import numpy as np
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(seed)
    a = a[rng.choice(len(a), min(n_sample, len(a)), replace=False)]
    b = b[rng.choice(len(b), min(n_sample, len(b)), replace=False)]
    da, _ = cKDTree(b).query(a)
    db, _ = cKDTree(a).query(b)
    return float(np.mean(da ** 2) + np.mean(db ** 2)), float(0.5 * (np.mean(da) + np.mean(db)))


def network_grid_sdf(net, centre, half, n, dev):
    """f of the SDF network at the cell centres of the n^3 grid (GPU), numpy [n][n][n]."""
    import numpy as np
    import torch
    from paper_2605_29097_amd import rfvr as R
    x = torch.from_numpy(grid_points(centre, half, n)).to(dev)
    out = []
    for k in range(0, x.shape[0], 1 << 22):
        f, _, _ = R.mlp_forward(net, x[k:k + (1 << 22)].contiguous())
        out.append(f.cpu().numpy())
    return np.concatenate(out).reshape(n, n, n)


def fit_prior(net, scene, centre, half, steps, dev, lr=1e-3, n_pool=1 << 20, batch=1 << 16, seed=0):
    """Study scaffolding: fit the SDF network to an analytic prior scene by
    regression of f on its signed distance (loss rfvr_loss_l2 on f, gradient
    rfvr_mlp_backward, update rfvr_adamw), on a seeded pool of points in the
    cube.  Returns the final RMS error of f in metres."""
    import numpy as np
    import torch
    from paper_2605_29097_amd import rfvr as R
    from synth import scene_fields
    rng = np.random.default_rng(seed)
    pts = (np.asarray(centre) + rng.uniform(-half, half, (n_pool, 3))).astype(np.float32)
    sdf, _, _ = scene_fields(scene, pts)
    X = torch.from_numpy(pts).to(dev)
    Y = torch.from_numpy(np.ascontiguousarray(sdf, np.float32)).to(dev)
    n_par = net.param_count()
    g = torch.zeros(n_par, device=dev)
    m = torch.zeros(n_par, device=dev)
    v = torch.zeros(n_par, device=dev)
    gen = torch.Generator(device=dev).manual_seed(seed)
    for t in range(1, steps + 1):
        idx = torch.randint(0, n_pool, (batch,), device=dev, generator=gen)
        x, y = X[idx].contiguous(), Y[idx].contiguous()
        f, _, _ = R.mlp_forward(net, x)
        loss, g_f = R.loss_l2(f, y)
        R.mlp_backward(net, x, g_f, None, None, out=g)
        R.adamw(net.params, g, m, v, t, lr * 0.5 * (1 + np.cos(np.pi * t / steps)))
    f, _, _ = R.mlp_forward(net, X[: 1 << 18].contiguous())
    return float(torch.sqrt(torch.mean((f - Y[: 1 << 18]) ** 2)))


def proposal_study(args, dev):
    """Torus-behind-slab scene (or, with --study-scene box, the 8 x 6 x 4 cm
    box): full-space training (2^20 grid points) against
    proposal-sampled training (n_imp importance + n_uni uniform depths per ray)
    and the untrained control (n_imp + n_uni stratified uniform depths), from
    the same initial network.  Every run is evaluated by the full-space render
    of its network (judge_nz depths per ray) against the clean target: signal
    NRMSE and heatmap (filter output) NRMSE at the judge's points.  E* is the
    full-space run's error after its step budget; steps_to_e_star is the first
    evaluation at or below it, and ms_to_e_star the measured time of the steps
    up to it plus the proposal's warm-up (proposal-only steps before the SDF
    network trains).  --study-full-every N makes every N-th step of the
    proposal run a full-space step (the fallback).  Prints one JSON line.

    --study-prior fits every run's initial network to a coarse version of the
    scene (torus and slab displaced and thickened by a few mm) by SDF
    regression, the same parameters for every run; otherwise all runs start
    from the geometric (sphere) initialisation."""
    import numpy as np
    import torch
    from paper_2605_29097_amd import rfvr as R
    from paper_2605_29097_amd.train import ProposalConfig, ProposalTrainer, StepConfig, Trainer
    from synth import MLPSpec, Slab, Torus, Union, mlp_init
    flags = R.SPEC_CLAMP | (R.WEIGHT_SEGMENT if args.study_weight == "segment" else 0)
    from synth import Box
    box = args.study_scene == "box"
    # the scene, the coarse version of it the prior is fitted to, and its parts
    # for the Chamfer distances
    if box:
        centre = (0.0, 0.0, 0.30)
        truth = Union([Box((0.0, 0.0, 0.30), (0.04, 0.03, 0.02), 0.8)])
        prior_scene = Union([Box((0.003, -0.002, 0.302), (0.043, 0.032, 0.022), 0.8)])
        part_names = ("box",)
    else:
        centre = (0.0, 0.0, 0.28)
        truth = Union([Slab(0.20, 0.005, 0.1), Torus((0.0, 0.0, 0.30), 0.04, 0.01, 0.8)])
        prior_scene = Union([Slab(0.203, 0.007, 0.1), Torus((0.003, -0.002, 0.303), 0.043, 0.013, 0.8)])
        part_names = ("slab", "torus")
    cfg = StepConfig(cube_centre=centre, learn_s=args.study_learn_s, s=args.study_s,
                     render_flags=flags, judge_nz=args.study_judge_nz, amp0=args.study_amp0)
    spec = MLPSpec(centre=cfg.cube_centre, half_size=cfg.cube_side / 2)
    if args.study_target:
        target_name = args.study_target
    elif box:
        target_name = "box_target.npz"
    else:
        target_name = "torus_target.npz" if cfg.s == 64.0 else f"torus_target_s{int(cfg.s)}.npz"
    data = np.load(os.path.join(ROOT, "tests", "golden", target_name))      # rendered by the oracle
    to_t = lambda a: torch.from_numpy(np.stack([a.real, a.imag], -1).astype(np.float32)).to(dev)
    noisy, clean = to_t(data["noisy"]), to_t(data["clean"])
    p0 = torch.from_numpy(mlp_init(spec, cfg.seed)).to(dev)
    prior_rms = None
    if args.study_prior:
        net = R.MLP(params=p0.clone(), centre=cfg.cube_centre, half_size=cfg.cube_side / 2)
        prior_rms = fit_prior(net, prior_scene, cfg.cube_centre, cfg.cube_side / 2, args.study_prior, dev)
        p0 = net.params.detach().clone()
        print(f"[study] prior fit: {args.study_prior} steps, f rms {prior_rms * 1e3:.3f} mm", file=sys.stderr,
              flush=True)
    amp_fit = None
    if args.study_fit_amp:
        # the heatmap P = |z| scales with A' (z is linear in it): the least-squares
        # A' of the starting network's full-space render against the measured
        # heatmap, A' = <P1, P*> / <P1, P1> with P1 the render at A' = 1
        t0 = Trainer(dataclasses.replace(cfg, amp0=1.0), p0.clone(), noisy, device=dev)
        xyz, _, origin = t0.samples()
        f, g, a = R.mlp_forward(t0.net, xyz)
        phi_ray, phi_tx, _ = t0.origin_occupancy(origin, t0.tx)
        fl = R.Fields(sdf=f.view(xyz.shape[:2]), grad=g.view(*xyz.shape[:2], 3), refl=a.view(xyz.shape[:2]),
                      s=cfg.s, amp=1.0, phi_ray=phi_ray, phi_tx=phi_tx)
        sig = R.render_forward(t0.ap, R.Samples(xyz=xyz), fl, flags=cfg.render_flags)
        _, p1, _, p_star = R.mf_forward(t0.ap, xyz, sig, t0.target)
        amp_fit = float((p1 * p_star).sum() / (p1 * p1).sum())
        cfg = dataclasses.replace(cfg, amp0=amp_fit)
        del t0
        print(f"[study] fitted initial amplitude A' = {amp_fit:.4f}", file=sys.stderr, flush=True)
    # Chamfer distances on a 256^3 grid (App. C metrics): the true scene's
    # surface points, each assigned to the primitive it lies nearest to
    n_grid = args.study_grid

    def split(pts):
        d = np.stack([np.abs(p.eval(pts)[0]) for p in truth.parts])
        near = np.argmin(d, 0)
        return {name: pts[near == k] for k, name in enumerate(part_names)}

    gt = None
    if n_grid:
        g_pts = grid_points(cfg.cube_centre, cfg.cube_side / 2, n_grid).astype(np.float64)
        f_gt = np.concatenate([truth.eval(g_pts[k:k + (1 << 22)])[0] for k in range(0, len(g_pts), 1 << 22)])
        gt = split(surface_points(f_gt.reshape(n_grid, n_grid, n_grid), cfg.cube_centre, cfg.cube_side / 2))
        del g_pts, f_gt

    def chamfer_of(net):
        if gt is None:
            return None
        pts = surface_points(network_grid_sdf(net, cfg.cube_centre, cfg.cube_side / 2, n_grid, dev),
                             cfg.cube_centre, cfg.cube_side / 2)
        rec = split(pts)
        out = {}
        for k in part_names:
            if len(rec[k]) == 0:
                out[k] = None
                continue
            cd2, cd = chamfer(rec[k], gt[k])
            out[k] = {"cd_sq_mm2": round(cd2 * 1e6, 4), "cd_mean_mm": round(cd * 1e3, 4)}
        return out

    prior_cd = None
    pc = dict(n_imp=args.study_imp, n_uni=args.study_uni, loss_on_grid=args.study_loss_grid,
              dilate=args.study_dilate, jitter=not args.study_prop_fixed)
    # the sampled runs' learning rates (network, amplitude), scaled
    cfg_s = dataclasses.replace(cfg, lr_sdf=cfg.lr_sdf * args.study_prop_lr_scale,
                                lr_other=cfg.lr_other * args.study_prop_lr_scale)
    runs = {
        "full_space": (lambda p: Trainer(dataclasses.replace(
            cfg, n_z=args.study_full_nz or cfg.n_z,
            sampling=R.SAMPLE_STRATIFIED if args.study_full_stratified else cfg.sampling), p, noisy, device=dev),
            args.study_full_steps, 0),
        "proposal": (lambda p: ProposalTrainer(cfg_s, p, noisy,
                                               ProposalConfig(full_every=args.study_full_every, **pc), device=dev),
                     args.study_prop_steps, args.study_prop_warmup),
        "uniform": (lambda p: ProposalTrainer(cfg_s, p, noisy, ProposalConfig(train=False, **pc), device=dev),
                    args.study_prop_steps, 0),
    }
    every = args.study_eval_every
    out = {}
    e_star_hm = None                         # the full-space run's final heatmap error (it runs first)
    for name, (make, n_steps, warm) in runs.items():
        tr = make(p0.clone())
        warm_ms = 0.0
        if warm:
            # proposal-only steps: the proposal learns where the initial
            # network's blend weights are; their time is charged to the run
            tr.train_sdf = False
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(warm):
                tr.step()
            e1.record()
            e1.synchronize()
            warm_ms = e0.elapsed_time(e1)
            tr.train_sdf = True
        j = tr.evaluate(clean)
        curve = [(0, j["signal"], j["heatmap"])]
        at_e_star = None                     # (step, Chamfer) where the heatmap error first reaches E*
        step_ms = []
        cum_ms = {0: 0.0}                    # measured training time up to each evaluated step
        for k in range(1, n_steps + 1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            tr.step()
            e1.record()
            e1.synchronize()
            step_ms.append(e0.elapsed_time(e1))
            if k % every == 0 or k == n_steps:
                cum_ms[k] = float(np.sum(step_ms))
                j = tr.evaluate(clean)
                curve.append((k, j["signal"], j["heatmap"]))
                if e_star_hm is not None and at_e_star is None and j["heatmap"] <= e_star_hm:
                    at_e_star = {"step": k, "chamfer": chamfer_of(tr.net)}
                print(f"[study] {name} step {k} reference signal {j['signal']:.4f} heatmap {j['heatmap']:.4f} "
                      f"s {tr.s:.1f} ({np.median(step_ms):.2f} ms/step)", file=sys.stderr, flush=True)
        out[name] = {"ms_per_step": float(np.median(step_ms[2:] if len(step_ms) > 4 else step_ms)),
                     "ms_per_step_mean": float(np.mean(step_ms)), "cum_ms": cum_ms,
                     "steps": n_steps, "warmup_steps": warm, "warmup_ms": round(warm_ms, 1), "final_s": tr.s,
                     "reference": [[k, round(a, 5), round(b, 5)] for k, a, b in curve],
                     "chamfer": chamfer_of(tr.net), "at_e_star_heatmap": at_e_star}
        if e_star_hm is None:
            e_star_hm = round(curve[-1][2], 5)
        if prior_cd is None:
            prior_cd = chamfer_of(R.MLP(params=p0.clone(), centre=cfg.cube_centre, half_size=cfg.cube_side / 2))
        del tr
        torch.cuda.empty_cache()
    e_star = {"signal": out["full_space"]["reference"][-1][1], "heatmap": out["full_space"]["reference"][-1][2]}
    for name, r in out.items():
        for col, key in ((1, "signal"), (2, "heatmap")):
            hit = next((row[0] for row in r["reference"] if row[col] <= e_star[key]), None)
            r[f"steps_to_e_star_{key}"] = hit
            r[f"ms_to_e_star_{key}"] = None if hit is None else round(r["cum_ms"][hit] + r["warmup_ms"], 1)
    print(json.dumps({"study": "proposal_vs_full_space", "e_star": e_star, "eval_every": every,
                      "learn_s": cfg.learn_s, "s0": cfg.s, "weight": args.study_weight, "target": target_name,
                      "judge_nz": cfg.judge_nz or cfg.n_z, "prior_fit_steps": args.study_prior,
                      "prior_f_rms_m": prior_rms, "n_imp": args.study_imp, "n_uni": args.study_uni,
                      "loss_on_grid": args.study_loss_grid, "target_dilation_bins": args.study_dilate,
                      "full_every": args.study_full_every, "amp0": cfg.amp0, "amp0_fitted": amp_fit,
                      "full_sampling": "stratified" if args.study_full_stratified else "grid",
                      "prop_lr_scale": args.study_prop_lr_scale, "prop_fixed_levels": args.study_prop_fixed,
                      "full_nz": args.study_full_nz or cfg.n_z,
                      "chamfer_grid": n_grid, "chamfer_initial": prior_cd,
                      "scene": ("box 8x6x4 cm (a=0.8) at 0.30 m; 32x32 aperture, 128 freqs, 20 cm cube at 0.30 m; "
                                "10 dB noise") if box else
                               ("torus R=4 cm r=1 cm at 0.30 m behind a 1 cm slab (a=0.1) at 0.20 m; "
                                "32x32 aperture, 128 freqs, 20 cm cube at 0.28 m; 10 dB noise"),
                      "runs": out}))


def naive_compare(args, dev):
    """Forward cost of the per-antenna method vs lensless sampling at one size:
    the 8x256 network, an n x n aperture, 32 x 32 rays x 64 depths, 128
    frequencies.  Prints one JSON line."""
    import torch
    from paper_2605_29097_amd import rfvr as R
    from paper_2605_29097_amd.naive import naive_forward
    from synth import MLPSpec, mlp_init
    from paper_2605_29097_amd.train import StepConfig, aperture_positions
    out = {"study": "naive_vs_lensless_forward", "runs": []}
    spec = MLPSpec()
    net = R.MLP(params=torch.from_numpy(mlp_init(spec, 0)).to(dev))
    for n_ap in args.naive_apertures:
        cfg = StepConfig(ap=(n_ap, n_ap))
        tx = torch.from_numpy(aperture_positions(cfg)).to(dev)
        ap = R.Aperture(tx=tx, f0=77e9, df=4e9 / 127, n_freq=128)

        def lensless():
            xyz, _, _ = R.sample_points(cfg.cube_centre, 0.1, (0, 0, 1), 32, 32, 64, device=dev)
            f, g, a = R.mlp_forward(net, xyz)
            fl = R.Fields(sdf=f.view(1024, 64), grad=g.view(1024, 64, 3), refl=a.view(1024, 64), s=64.0)
            return R.render_forward(ap, R.Samples(xyz=xyz), fl)

        def naive():
            return naive_forward(net, ap, cfg.cube_centre, 0.1, (0, 0, 1), 32, 32, 64, s=64.0)

        row = {"n_ant": n_ap * n_ap, "points_lensless": 32 * 32 * 64, "points_naive": n_ap * n_ap * 32 * 32 * 64}
        for name, fn in (("lensless", lensless), ("naive", naive)):
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(3):
                fn()
            e1.record()
            e1.synchronize()
            row[f"{name}_ms"] = round(e0.elapsed_time(e1) / 3, 3)
            print(f"[naive] n_ant {n_ap * n_ap} {name} {row[name + '_ms']} ms", file=sys.stderr, flush=True)
        out["runs"].append(row)
    print(json.dumps(out))


def network_precisions(args, dev):
    """Network call times at the 2^20-point workload (8 x 256 trunk, 2 x 64 head,
    6 octaves, the bench's points and parameters) for every matrix-operand form:
    the forward (f, grad_x f, a), the plain backward (recomputes the forward
    products), and the training pair (forward keeping the reserve, backward
    reading it), with upstream gradients of the size the render adjoint gives.
    HIP events around `--steps` calls of each after one warm-up call.  Prints
    one JSON line."""
    import torch
    from paper_2605_29097_amd import rfvr as R
    from paper_2605_29097_amd.train import StepConfig, Trainer
    cfg = StepConfig()
    params, target = make_inputs(cfg, dev)
    tr = Trainer(cfg, params, target, device=dev)
    xyz, _, _ = R.sample_points(cfg.cube_centre, cfg.cube_side / 2, (0.0, 0.0, 1.0), cfg.lines[0], cfg.lines[1],
                                cfg.n_z, device=dev)
    x = xyz.view(-1, 3)
    n = x.shape[0]
    gen = torch.Generator(device=dev).manual_seed(1)
    gf = torch.randn(n, device=dev, generator=gen)
    gg = torch.randn(n, 3, device=dev, generator=gen)
    gaa = torch.randn(n, device=dev, generator=gen)
    reps = max(1, min(args.steps, 10))

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        return round(e0.elapsed_time(e1) / reps, 2)

    out = {"study": "network_precisions", "points": n, "calls": reps, "ms": {}}
    for pname in ("fp32", "bf16", "bf16x3", "f16"):
        net = dataclasses.replace(tr.net, precision=getattr(R, "PREC_" + pname.upper()))
        res = R.mlp_reserve(net, n, dev)
        row = {"forward": timed(lambda: R.mlp_forward(net, x)),
               "backward_plain": timed(lambda: R.mlp_backward(net, x, gf, gg, gaa)),
               "forward_train": timed(lambda: R.mlp_forward(net, x, reserve=res)),
               "backward_train": timed(lambda: R.mlp_backward(net, x, gf, gg, gaa, reserve=res))}
        out["ms"][pname] = row
        print(f"[networks] {pname}: {row}", file=sys.stderr, flush=True)
        del res
        torch.cuda.empty_cache()
    print(json.dumps(out))


def batched8_study(args, dev):
    """The eight-scene workload: apertures of 32^2 .. 64^2 antennas at 2 mm
    (19,292 in all), 256 frequencies 77-81 GHz, 2^22 points per scene (128 x 128
    lensless rays x 256 depths in a 25 cm cube at the scene's range), one
    8 x 256 network per scene.  One call of each batched or grouped entry point
    over all eight scenes, in the order of a training step, timed with HIP
    events after a warm-up call; terms/s per term pass (sum over scenes of
    points x measurements x frequencies).  Prints one JSON line."""
    import torch
    from paper_2605_29097_amd import rfvr as R
    from synth import MLPSpec, freq_grid, mlp_init, planar_aperture
    from synth.configs import PITCH, batched8_scene, config
    c = config("batched8")
    m = c["mlp"]
    f0, df = freq_grid(c["n_freq"])
    nx, ny = c["lines"]
    nz = c["n_imp"] + c["n_uni"]
    geo = [batched8_scene(k) for k in range(len(c["ap_sides"]))]
    aps, xyzs = [], []
    for g in geo:
        tx = torch.from_numpy(planar_aperture(g["side"], g["side"], PITCH)).to(dev)
        aps.append(R.Aperture(tx=tx, f0=f0, df=df, n_freq=c["n_freq"]))
        xyz, _, _ = R.sample_points(g["centre"], g["half"], (0, 0, 1), nx, ny, nz, mode=R.SAMPLE_STRATIFIED,
                                    seed=g["seed"], device=dev)
        xyzs.append(xyz)
    terms = sum(x.shape[0] * x.shape[1] * a.n_meas * a.n_freq for a, x in zip(aps, xyzs))

    def timed(fn, reps=2):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            r = fn()
        e1.record()
        e1.synchronize()
        return r, e0.elapsed_time(e1) / reps

    out = {"study": "eight_scene_batched", "terms_per_pass": terms, "points": sum(x.numel() // 3 for x in xyzs),
           "networks": {}}
    gen = torch.Generator(device=dev).manual_seed(0)
    for pname, prec in (("bf16x3", R.PREC_BF16X3), ("f16", R.PREC_F16), ("bf16", R.PREC_BF16)):
        nets = []
        for k, g in enumerate(geo):
            spec = MLPSpec(n_layers=m["n_layers"], width=m["width"], pe_octaves=m["pe_octaves"],
                           head_width=m["head_width"], head_layers=m["head_layers"], beta=m["beta"],
                           centre=g["centre"], half_size=g["half"])
            nets.append(R.MLP(params=torch.from_numpy(mlp_init(spec, k)).to(dev), n_layers=spec.n_layers,
                              width=spec.width, pe_octaves=spec.pe_octaves, head_width=spec.head_width,
                              head_layers=spec.head_layers, beta=spec.beta, centre=spec.centre,
                              half_size=spec.half_size, precision=prec))
        row = {}
        fga, row["mlp_forward_grouped_ms"] = timed(lambda: R.mlp_forward_grouped(nets, xyzs))
        if pname == "bf16x3":
            scenes = [(a, R.Samples(xyz=x), R.Fields(sdf=f.view(x.shape[:2]), grad=gr.view(x.shape),
                                                     refl=al.view(x.shape[:2]), s=c["s"]))
                      for a, x, (f, gr, al) in zip(aps, xyzs, fga)]
            sig, t_rf = timed(lambda: R.render_forward_batched(scenes))
            zp, t_mf = timed(lambda: R.mf_forward_batched(scenes, sig))
            gps = [torch.randn(p.shape, generator=gen, device=dev) / p.numel() for _, p in zp]
            gsig, t_mb = timed(lambda: R.mf_backward_batched(scenes, [z for z, _ in zp], [p for _, p in zp], gps))
            gfl, t_rb = timed(lambda: R.render_backward_batched(scenes, gsig))
            for name, t in (("render_forward", t_rf), ("mf_forward", t_mf), ("mf_backward", t_mb),
                            ("render_backward", t_rb)):
                out[f"{name}_ms"] = round(t, 2)
                out[f"{name}_terms_per_s"] = terms / (t * 1e-3)
                print(f"[batched8] {name} {t:.1f} ms, {terms / (t * 1e-3):.3e} terms/s", file=sys.stderr,
                      flush=True)
        ups = [(d["sdf"].reshape(-1), d["grad"].reshape(-1, 3), d["refl"].reshape(-1)) for d in gfl]
        _, row["mlp_backward_grouped_ms"] = timed(lambda: R.mlp_backward_grouped(
            nets, xyzs, [u[0] for u in ups], [u[1] for u in ups], [u[2] for u in ups]))
        row = {k: round(v, 2) for k, v in row.items()}
        print(f"[batched8] networks {pname}: {row}", file=sys.stderr, flush=True)
        out["networks"][pname] = row
        del nets, fga
    print(json.dumps(out))


def batched8_train(args, dev):
    """Training steps of the eight-scene workload: per scene a proposal-sampled
    step (128 x 128 rays, 64 bins, 192 importance + 64 stratified depths, 2^22
    points; the measured heatmap recomputed at the new points) of its own
    network (8 x 256, split-BF16 or BF16 operands), the scenes stepped one
    after another and sharing one network reserve.  The measured signals are
    seeded random (a timing run).  Times whole eight-scene steps with HIP events
    after one warm-up step.  Prints one JSON line."""
    import numpy as np
    import torch
    from paper_2605_29097_amd import rfvr as R
    from paper_2605_29097_amd.train import ProposalConfig, ProposalTrainer, StepConfig
    from synth import MLPSpec, mlp_init
    from synth.configs import batched8_scene, config
    c = config("batched8")
    m = c["mlp"]
    out = {"study": "eight_scene_training_step", "runs": {}}
    for pname, prec in (("bf16x3", R.PREC_BF16X3), ("f16", R.PREC_F16), ("bf16", R.PREC_BF16)):
        trainers, shared = [], None
        for k in range(len(c["ap_sides"])):
            g = batched8_scene(k)
            cfg = StepConfig(ap=(g["side"], g["side"]), n_freq=c["n_freq"], cube_centre=g["centre"],
                             cube_side=c["cube_side"], lines=c["lines"], n_z=c["n_imp"] + c["n_uni"],
                             s=c["s"], n_layers=m["n_layers"], width=m["width"], pe_octaves=m["pe_octaves"],
                             head_width=m["head_width"], head_layers=m["head_layers"], beta=m["beta"],
                             precision=prec, seed=k)
            spec = MLPSpec(n_layers=m["n_layers"], width=m["width"], pe_octaves=m["pe_octaves"],
                           head_width=m["head_width"], head_layers=m["head_layers"], beta=m["beta"],
                           centre=g["centre"], half_size=g["half"])
            rng = np.random.default_rng(100 + k)
            target = torch.from_numpy((rng.normal(size=(cfg.n_meas, c["n_freq"], 2)) * 1e-3).astype(np.float32))
            tr = ProposalTrainer(cfg, torch.from_numpy(mlp_init(spec, k)), target,
                                 ProposalConfig(n_imp=c["n_imp"], n_uni=c["n_uni"], seed=k), device=dev)
            if shared is None:
                shared = R.mlp_reserve(tr.net, cfg.lines[0] * cfg.lines[1] * cfg.n_z, dev)
            tr.shared_reserve = shared
            trainers.append(tr)

        def step():
            return [tr.step() for tr in trainers]

        step()
        torch.cuda.synchronize()
        times = []
        for _ in range(args.steps if args.steps < 10 else 3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            losses = step()
            e1.record()
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
            print(f"[batched8-train] {pname} step {e0.elapsed_time(e1):.1f} ms, losses "
                  f"{[round(float(x.item()), 6) for x in losses]}", file=sys.stderr, flush=True)
        terms = 4 * sum(tr.cfg.n_meas * tr.cfg.n_freq * tr.cfg.lines[0] * tr.cfg.lines[1] * tr.cfg.n_z
                        for tr in trainers)
        ms = float(np.median(times))
        out["runs"][pname] = {"ms_per_step": round(ms, 1), "terms_per_step": terms,
                              "terms_per_s": terms / (ms * 1e-3)}
        del trainers, shared, tr
        torch.cuda.empty_cache()
    print(json.dumps(out))


def step_16bit(cfg, params, target, args, dev):
    """The same training step with the network on its FP16 form (FP16 forward
    products with the per-point operand split, BF16 backward products, FP32
    accumulation), which holds the rendered signal within 1e-2 of the FP64
    oracle: a context figure beside the FP32 line, timed the same way."""
    import torch
    from paper_2605_29097_amd import rfvr as R
    from paper_2605_29097_amd.train import Trainer
    tr = Trainer(dataclasses.replace(cfg, precision=R.PREC_F16), params, target, device=dev)
    for _ in range(max(1, args.warmup)):
        tr.step()
    torch.cuda.synchronize()
    steps = max(1, min(args.steps, 10))
    t0 = time.perf_counter()
    for _ in range(steps):
        tr.step()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    print(f"[bench] FP16-network step {ms:.2f} ms", file=sys.stderr, flush=True)
    return {"precision": "RFVR_PREC_F16: FP16 forward products (per-point operand split in two), BF16 "
                         "backward products, FP32 accumulation; render FP32",
            "steps": steps, "ms_per_step": round(ms, 3),
            "terms_per_s": 4 * cfg.terms_per_pass() / (ms * 1e-3)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--phases", action="store_true", help="print per-phase times to stderr")
    ap.add_argument("--no-16bit-step", action="store_true",
                    help="leave out the context figure of the same step with the FP16 network form")
    ap.add_argument("--kernel-probe", choices=["mlp_bwd", "render_fwd", "mf_fwd", "mf_bwd", "render_bwd"],
                    help="run only one pass of the workload (for hardware-counter runs)")
    ap.add_argument("--probe-precision", choices=["fp32", "bf16", "bf16x3", "f16"], default="fp32",
                    help="network operand form of the kernel probe's workload")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a plain 1 GiB device copy (calibrates the HBM byte counters)")
    ap.add_argument("--proposal-study", action="store_true",
                    help="train full-space vs proposal-sampled vs uniform-20 on the torus scene")
    ap.add_argument("--study-full-steps", type=int, default=300)
    ap.add_argument("--study-prop-steps", type=int, default=1200)
    ap.add_argument("--study-eval-every", type=int, default=50)
    ap.add_argument("--study-learn-s", action="store_true", help="train log s in every run")
    ap.add_argument("--study-s", type=float, default=64.0,
                    help="initial s (1/m); the target is the oracle render of the scene at this s")
    ap.add_argument("--study-weight", choices=["sample", "segment"], default="sample",
                    help="render weight of every run (segment: RFVR_WEIGHT_SEGMENT)")
    ap.add_argument("--study-target", default=None, help="target file under tests/golden")
    ap.add_argument("--study-judge-nz", type=int, default=None, help="depths per ray of the judge render")
    ap.add_argument("--study-prior", type=int, default=0,
                    help="fit the initial network to a coarse scene for this many regression steps")
    ap.add_argument("--study-grid", type=int, default=256,
                    help="grid side of the Chamfer surface extraction (0: no Chamfer)")
    ap.add_argument("--study-loss-grid", action="store_true",
                    help="sampled runs take the heatmap loss on the full-space grid (render from their samples)")
    ap.add_argument("--study-scene", choices=["torus_slab", "box"], default="torus_slab",
                    help="torus behind a slab in a cube at 0.28 m, or the 8 x 6 x 4 cm box in a cube at 0.30 m")
    ap.add_argument("--study-full-every", type=int, default=0,
                    help="every this many steps the proposal run takes a full-space step (0: never)")
    ap.add_argument("--study-amp0", type=float, default=1.0, help="initial amplitude A' of every run")
    ap.add_argument("--study-prop-fixed", action="store_true",
                    help="the sampled runs put every depth at the middle of its stratum (no per-step draw)")
    ap.add_argument("--study-prop-lr-scale", type=float, default=1.0,
                    help="scale of the sampled runs' learning rates (network and amplitude)")
    ap.add_argument("--study-fit-amp", action="store_true",
                    help="every run starts from the least-squares A' of the starting network's heatmap")
    ap.add_argument("--study-full-nz", type=int, default=0,
                    help="depths per ray of the full-space run (0: the workload's 256)")
    ap.add_argument("--study-full-stratified", action="store_true",
                    help="the full-space run draws stratified depths each step instead of the fixed grid")
    ap.add_argument("--study-dilate", type=int, default=0,
                    help="proposal targets dilated in depth over this many bins")
    ap.add_argument("--study-imp", type=int, default=16)
    ap.add_argument("--study-uni", type=int, default=4)
    ap.add_argument("--study-prop-warmup", type=int, default=0,
                    help="proposal-only steps before the proposal run trains the SDF network")
    ap.add_argument("--naive-compare", action="store_true",
                    help="forward time of per-antenna sampling vs lensless sampling")
    ap.add_argument("--naive-apertures", type=int, nargs="+", default=[4, 8, 16])
    ap.add_argument("--network-precisions", action="store_true",
                    help="time the network calls at 2^20 points for every matrix-operand form")
    ap.add_argument("--batched8", action="store_true",
                    help="time the batched and grouped calls on the eight-scene workload")
    ap.add_argument("--batched8-train", action="store_true",
                    help="time proposal-sampled training steps of the eight-scene workload")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported; this build measures one MI355X "
              "(the multi-GPU sharding by points is a design, not a measured path)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2605_29097_amd import rfvr as R
    from paper_2605_29097_amd.train import StepConfig, Trainer
    R.lib()
    dev = torch.device("cuda:0")
    if args.copy_probe:
        x = torch.ones(1 << 28, dtype=torch.float32, device=dev)      # 1 GiB
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": x.numel() * 4}))
        return
    if args.proposal_study:
        proposal_study(args, dev)
        return
    if args.naive_compare:
        naive_compare(args, dev)
        return
    if args.network_precisions:
        network_precisions(args, dev)
        return
    if args.batched8:
        batched8_study(args, dev)
        return
    if args.batched8_train:
        batched8_train(args, dev)
        return
    cfg = StepConfig()
    if args.kernel_probe:
        cfg = dataclasses.replace(cfg, precision=getattr(R, "PREC_" + args.probe_precision.upper()))
    params, target = make_inputs(cfg, dev)
    tr = Trainer(cfg, params, target, device=dev)
    if args.kernel_probe:
        probe(tr, args.kernel_probe, args.steps)
        return
    for _ in range(args.warmup):
        tr.step()
    torch.cuda.synchronize()
    timers = {}
    t0 = time.perf_counter()
    for k in range(args.steps):
        tr.step(timers)
        print(f"[bench] step {k + 1}/{args.steps}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = 1e3 * wall / args.steps

    order = ["start", "sample", "mlp_fwd", "render_fwd", "mf_fwd", "mf_bwd", "render_bwd", "mlp_bwd",
             "adamw"]
    phases = {}
    for a, b in zip(order[:-1], order[1:]):
        phases[b] = sum(ea.elapsed_time(eb) for ea, eb in zip(timers[a], timers[b])) / args.steps
    # per-step spread from the same events (first to last mark of each step)
    per_step = np.array([ea.elapsed_time(eb) for ea, eb in zip(timers[order[0]], timers[order[-1]])])
    if args.phases:
        print(json.dumps({"phases_ms": phases}), file=sys.stderr)

    tpp = cfg.terms_per_pass()
    terms_step = 4 * tpp
    value = terms_step / (ms_step * 1e-3)
    # dominant part of the step: the network training backward, one C-ABI
    # call whose GEMMs (FP32 MFMA) take most of its time; timed by HIP events
    # on the stream the call launches on
    t_nb = phases["mlp_bwd"] * 1e-3
    achieved = cfg.n_pts * mlp_backward_flop(cfg) / t_nb / 1e12
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": measured_traffic(),
                "kernel": "rfvr_mlp_backward_train (per layer: tangent, adjoint and two weight-gradient "
                          "FP32 MFMA GEMMs, elementwise work in their epilogues)",
                "launch_ms": round(phases["mlp_bwd"], 3)}
    # the term kernels: signal tracing forward through its moments, priced at
    # the moment kernel's own work per (measurement, point) pair
    K = R.term_order(tr.ap, tr.samples()[0])
    t_rf = phases["render_fwd"] * 1e-3
    a_t = cfg.n_pts * cfg.n_meas * moment_flop_per_pair(K) / t_rf / 1e12
    roofline_terms = {"bound": "alu", "kernel": f"k_cheb_points<{K},0,CLAMP> (signal tracing forward, "
                                                f"order {K})", "order": K,
                      "achieved": round(a_t, 3), "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                      "frac": round(a_t / PEAK_FP32_VALU_TFLOPS, 4), "launch_ms": round(phases["render_fwd"], 3),
                      "flop_per_pair": moment_flop_per_pair(K),
                      "pairs_per_s": round(cfg.n_pts * cfg.n_meas / t_rf, 1),
                      "terms_per_s_direct_sum_equivalent": round(tpp / t_rf, 1)}
    out = {
        "metric": "fwd+bwd RF render terms/s",
        "value": value,
        "unit": "terms/s",
        # value counts the (point, measurement, frequency) triples of the four
        # term sums per second; the kernels evaluate each (point, measurement)
        # pair's frequencies through K Chebyshev moments of the range (order
        # chosen per launch, truncation 1e-6 of the summed term magnitudes)
        # rather than one by one, so no direct-sum FLOP rate can be read off it
        "value_kind": f"direct-sum equivalent: term triples per second, evaluated through order-{K} "
                      f"Chebyshev moments per (point, measurement) pair",
        "pairs_per_s": round(4 * cfg.n_pts * cfg.n_meas / (ms_step * 1e-3), 1),
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "step_ms_median_p10_p90": [round(float(np.median(per_step)), 3), round(float(np.percentile(per_step, 10)), 3),
                                   round(float(np.percentile(per_step, 90)), 3)],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "mlp_box: full-space training step, 2^20 points (64x64 primary rays "
                               "x 256 depths, 20 cm cube at 0.30 m), 32x32 monostatic aperture at "
                               "2 mm, 128 frequencies 77-81 GHz, 8x256 softplus(100) SDF MLP on a "
                               "6-octave encoding + 2x64 head, FP32, box target + 10 dB noise",
                   "terms_per_step": terms_step, "parallelism": "single GPU"},
        "phases_ms": {k: round(v, 3) for k, v in phases.items()},
        # detached occupancy at the ray feet and antennas on the aperture
        # plane (Eq. lens-less-transmittance) after the timed steps: the shift
        # it produces is 1 - min at most
        "phi_origins_min": float(tr.last["phi_origins"].min()),
        "roofline": roofline,
        "roofline_terms": roofline_terms,
    }
    if not args.no_16bit_step:
        out["step_16bit_network"] = step_16bit(cfg, params, target, args, dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_both(cfg)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
