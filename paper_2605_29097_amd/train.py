"""One training step of the lensless RF renderer (GeRaF, Sec. Overview steps 1-5),
driven through the C ABI with explicit forward / adjoint calls.

step():
  1. lensless primary-ray samples (Sec. Lensless Sampling)          rfvr_sample_points
  2. SDF network at the samples: f, grad_x f, a                      rfvr_mlp_forward_train
     and at the ray / antenna origins: detached Phi (Eq. lens-less-transmittance)
  3. signal tracing with lensless alpha blending (Eq. ref_sim)       rfvr_render_forward
  4. matched filter at the samples (Eq. mf-sm)                      rfvr_mf_forward
  5. L2 loss against the measured signal's filter output             rfvr_loss_l2
  then the adjoints in reverse (rfvr_mf_backward, rfvr_render_backward,
  rfvr_mlp_backward_train) and AdamW with cosine annealing (App. C)        rfvr_adamw
No host synchronisation happens inside a step.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import torch

from . import rfvr as R


@dataclass
class StepConfig:
    ap: tuple = (32, 32)
    pitch: float = 2e-3
    n_freq: int = 128
    f_lo: float = 77e9
    f_hi: float = 81e9
    cube_centre: tuple = (0.0, 0.0, 0.30)
    cube_side: float = 0.20
    lines: tuple = (64, 64)
    n_z: int = 256
    sampling: int = R.SAMPLE_GRID
    s: float = 64.0
    amp0: float = 1.0
    n_layers: int = 8
    width: int = 256
    pe_octaves: int = 6
    head_width: int = 64
    head_layers: int = 2
    beta: float = 100.0
    lr_sdf: float = 1e-4
    lr_other: float = 1e-3
    total_steps: int = 50000
    seed: int = 0
    render_flags: int = R.SPEC_CLAMP       # specular mode, optionally | R.WEIGHT_SEGMENT
    judge_nz: Optional[int] = None         # depths of the full-space judge render (None: n_z)
    bank_patch: Optional[tuple] = None     # (px, py) antennas per Signal Tracing Bank patch
    learn_s: bool = False                  # train log s with the head's learning rate
    precision: int = R.PREC_FP32           # network matrix operands (R.PREC_FP32 / BF16 / BF16X3 / F16)
    keep_activations: bool = True          # network training pair: the backward reads the
                                           # forward's layer activations from a reserve
    mask_tau: Optional[tuple] = None       # (tau_hi, tau_lo): dynamic loss masking on
    origin_phi: str = "network"            # Phi at the ray origins and antennas: "network" evaluates the
                                           # SDF network there (Eq. lens-less-transmittance as written);
                                           # "volume" takes space outside the sample cube as air, so with
                                           # every origin and antenna outside it the shift is 0

    @property
    def n_pts(self) -> int:
        return self.lines[0] * self.lines[1] * self.n_z

    @property
    def n_meas(self) -> int:
        return self.ap[0] * self.ap[1]

    def terms_per_pass(self) -> int:
        return self.n_pts * self.n_meas * self.n_freq


def aperture_positions(cfg: StepConfig) -> np.ndarray:
    nx, ny = cfg.ap
    ix = (np.arange(nx) - (nx - 1) / 2.0) * cfg.pitch
    iy = (np.arange(ny) - (ny - 1) / 2.0) * cfg.pitch
    gx, gy = np.meshgrid(ix, iy, indexing="xy")
    return np.stack([gx.ravel(), gy.ravel(), np.zeros(nx * ny)], 1).astype(np.float32)


def patch_order(cfg: StepConfig) -> np.ndarray:
    """Measurement ids (i = iy * nx + ix) in patch-major order: the aperture is
    cut into px x py tiles (Sec. Signal Tracing Bank), tiles in row-major order,
    antennas row-major inside a tile.  With this order every patch is one
    contiguous block of rows of the signal."""
    nx, ny = cfg.ap
    px, py = cfg.bank_patch
    if nx % px or ny % py:
        raise ValueError(f"patch {px}x{py} does not tile the {nx}x{ny} aperture")
    ids = [iy * nx + ix
           for by in range(ny // py) for bx in range(nx // px)
           for iy in range(by * py, (by + 1) * py) for ix in range(bx * px, (bx + 1) * px)]
    return np.asarray(ids, np.int64)


class Trainer:
    """State of one reconstruction: network, amplitude, optimiser moments, target."""

    def __init__(self, cfg: StepConfig, params: torch.Tensor, target_signal: torch.Tensor,
                 device="cuda"):
        self.cfg = cfg
        self.dev = torch.device(device)
        f0 = cfg.f_lo
        df = 0.0 if cfg.n_freq == 1 else (cfg.f_hi - cfg.f_lo) / (cfg.n_freq - 1)
        tx = aperture_positions(cfg)
        self.perm = None
        if cfg.bank_patch is not None:
            # measurements are held in patch-major order (the target's rows too)
            self.perm = patch_order(cfg)
            tx = tx[self.perm]
            self.patch_len = cfg.bank_patch[0] * cfg.bank_patch[1]
            self.n_patch = cfg.n_meas // self.patch_len
            self.bank = None
        self.tx = torch.from_numpy(np.ascontiguousarray(tx)).to(self.dev)
        self.f0, self.df = f0, df
        self.ap = R.Aperture(tx=self.tx, f0=f0, df=df, n_freq=cfg.n_freq)
        self.net = R.MLP(params=params.to(self.dev).contiguous(), n_layers=cfg.n_layers,
                         width=cfg.width, pe_octaves=cfg.pe_octaves, head_width=cfg.head_width,
                         head_layers=cfg.head_layers, beta=cfg.beta,
                         centre=tuple(cfg.cube_centre), half_size=cfg.cube_side / 2,
                         precision=cfg.precision)
        n_par = self.net.param_count()
        assert self.net.params.numel() == n_par
        self.m = torch.zeros(n_par, device=self.dev)
        self.v = torch.zeros(n_par, device=self.dev)
        self.g = torch.zeros(n_par, device=self.dev)
        self._res = {}                  # training-pair reserves by point count (at most two kept)
        self.keep_alpha = False         # keep the full-space render's alpha and T in self.last
        # a reserve shared by trainers that step one after another (each step
        # fills it in its forward and reads it in its backward); None: own one
        self.shared_reserve = None
        # the SDF branch (trunk + sdf output) comes first in the flat layout
        w, L, in0 = cfg.width, cfg.n_layers, 3 + 6 * cfg.pe_octaves
        self.n_sdf = w * in0 + w + (L - 1) * (w * w + w) + w + 1
        self.amp = torch.tensor([cfg.amp0], device=self.dev)
        self.amp_m = torch.zeros(1, device=self.dev)
        self.amp_v = torch.zeros(1, device=self.dev)
        target = target_signal.to(self.dev)
        if self.perm is not None:
            target = target[torch.from_numpy(self.perm).to(self.dev)]
        self.target = target.contiguous()
        self.s0 = float(cfg.s)
        # a learnable s lives on the device as log s: the kernels read it there
        # and AdamW updates it there, so a step never waits for the host
        self.log_s = None
        if cfg.learn_s:
            self.log_s = torch.tensor([math.log(cfg.s)], device=self.dev)
            self.log_s_m = torch.zeros(1, device=self.dev)
            self.log_s_v = torch.zeros(1, device=self.dev)
        self.history = None                    # per-point filter-output history (masking)
        # the ray origins lie on the plane through the world origin normal to
        # the primary direction (z = 0 here), the antennas at tx
        h = cfg.cube_side / 2
        outside = lambda p: bool(np.any(np.abs(np.asarray(p, np.float64) - np.asarray(cfg.cube_centre)) > h, axis=-1).all())
        self.origins_in_air = (cfg.origin_phi == "volume" and abs(cfg.cube_centre[2]) > h and outside(tx))
        if cfg.origin_phi not in ("network", "volume"):
            raise ValueError(f"origin_phi must be 'network' or 'volume', not {cfg.origin_phi!r}")
        self.t = 0
        self.p_star = None
        self._xyz_key = None
        self.origin_pts = None

    # ------------------------------------------------------------------ helpers
    def origin_occupancy(self, origin, tx):
        """Detached Phi at the primary-ray origins and the antennas:
        (phi_ray, phi_tx, both), or (None, None, None) when they all lie in air
        (origin_phi = "volume", all outside the sample cube: no shift)."""
        if self.origins_in_air:
            return None, None, None
        f_org, _, _ = R.mlp_forward(self.net, torch.cat([origin, tx], 0))
        phi = R.occupancy(self.s_arg, f_org)
        n = origin.shape[0]
        return phi[:n].contiguous(), phi[n:].contiguous(), phi

    def samples(self):
        c = self.cfg
        return R.sample_points(c.cube_centre, c.cube_side / 2, (0.0, 0.0, 1.0), c.lines[0], c.lines[1],
                               c.n_z, mode=c.sampling, seed=c.seed, step=self.t, device=self.dev)

    def lr(self, base: float) -> float:
        T = self.cfg.total_steps
        return 0.5 * base * (1.0 + math.cos(math.pi * min(self.t, T) / T))

    # ------------------------------------------------------------------ step
    def step(self, timers: Optional[dict] = None):
        """One full training step; returns the loss tensor (device, not synced)."""
        c = self.cfg
        ev = timers if timers is not None else None

        def mark(name):
            if ev is not None:
                e = torch.cuda.Event(enable_timing=True)
                e.record()
                ev.setdefault(name, []).append(e)

        mark("start")
        xyz, u, origin = self.samples()
        n = xyz.shape[0] * xyz.shape[1]
        mark("sample")
        res = self.reserve(n)
        f, grad, a = R.mlp_forward(self.net, xyz, reserve=res)
        # detached occupancies at the primary-ray origins and the antennas
        phi_ray, phi_tx, phi = self.origin_occupancy(origin, self.tx)
        mark("mlp_fwd")
        sm = R.Samples(xyz=xyz)
        fl = R.Fields(sdf=f.view(xyz.shape[:2]), grad=grad.view(*xyz.shape[:2], 3),
                      refl=a.view(xyz.shape[:2]), s=self.s0, amp=1.0, amp_dev=self.amp,
                      log_s_dev=self.log_s,
                      phi_ray=phi_ray, phi_tx=phi_tx)
        ap_r, fl_r = self.ap, fl
        if c.bank_patch is None:
            if self.keep_alpha:
                sig, alpha_f, trans_f = R.render_forward(self.ap, sm, fl, flags=c.render_flags, want_alpha=True)
            else:
                sig = R.render_forward(self.ap, sm, fl, flags=c.render_flags)
        else:
            # Signal Tracing Bank: trace only the current patch's antennas into
            # its rows of the bank; the other rows keep earlier results
            if self.bank is None:
                self.bank = R.render_forward(self.ap, sm, fl, flags=c.render_flags)
            k = self.t % self.n_patch
            i0, i1 = k * self.patch_len, (k + 1) * self.patch_len
            ap_r = R.Aperture(tx=self.tx[i0:i1], f0=self.f0, df=self.df, n_freq=c.n_freq)
            n_ray = origin.shape[0]
            fl_r = R.Fields(sdf=fl.sdf, grad=fl.grad, refl=fl.refl, s=self.s0, amp=1.0, amp_dev=self.amp,
                            log_s_dev=self.log_s,
                            phi_ray=fl.phi_ray, phi_tx=None if phi_tx is None else phi_tx[i0:i1].contiguous())
            R.render_forward(ap_r, sm, fl_r, flags=c.render_flags, out=self.bank[i0:i1])
            sig = self.bank
        mark("render_fwd")
        key = (c.sampling, None if c.sampling == R.SAMPLE_GRID else self.t)
        if self.p_star is None or key != self._xyz_key:
            z, p, _, p_star = R.mf_forward(self.ap, xyz, sig, self.target)
            self.p_star, self._xyz_key = p_star, key
        else:
            z, p = R.mf_forward(self.ap, xyz, sig)
        mark("mf_fwd")
        mask = None
        if c.mask_tau is not None:
            # dynamic loss masking (Sec. Optimization): per sample point, so the
            # sample set must be the same every step (grid or stratified cells)
            if self.history is None:
                self.history = torch.zeros_like(p)
            mask = R.mask_update(p, self.p_star, self.history, *c.mask_tau)
        loss, g_p = R.loss_l2(p, self.p_star, mask=mask)
        self.last_mask = mask
        # the filter has no parameters: only the traced rows carry gradient
        g_sig = R.mf_backward(ap_r, xyz, z, p, g_p)
        mark("mf_bwd")
        gr = R.render_backward(ap_r, sm, fl_r, g_sig, flags=c.render_flags)
        mark("render_bwd")
        R.mlp_backward(self.net, xyz, gr["sdf"].view(-1), gr["grad"].view(-1, 3), gr["refl"].view(-1),
                       out=self.g, reserve=res)
        mark("mlp_bwd")
        self.t += 1
        P, G, M, V = self.net.params, self.g, self.m, self.v
        ns = self.n_sdf
        R.adamw(P[:ns], G[:ns], M[:ns], V[:ns], self.t, self.lr(c.lr_sdf))
        R.adamw(P[ns:], G[ns:], M[ns:], V[ns:], self.t, self.lr(c.lr_other))
        R.adamw(self.amp, gr["amp"], self.amp_m, self.amp_v, self.t, self.lr(c.lr_other))
        mark("adamw")
        if c.learn_s:
            self.update_s(gr["s"])
        self.last = dict(signal=sig, loss=loss, phi_origins=phi, u=u)
        if self.keep_alpha and c.bank_patch is None:
            self.last.update(alpha=alpha_f, trans=trans_f)
        return loss

    def reserve(self, n: int):
        """Reserve of the network's training pair for n points (None when off)."""
        if not self.cfg.keep_activations:
            return None
        if self.shared_reserve is not None:
            return self.shared_reserve
        if n not in self._res:
            if len(self._res) >= 2:
                self._res.pop(next(iter(self._res)))
            self._res[n] = R.mlp_reserve(self.net, n, self.dev)
        return self._res[n]

    def update_s(self, g_log_s: torch.Tensor):
        """AdamW step on log s, on the device (the render adjoint returns the
        gradient in log s when the fields carry log_s_dev)."""
        R.adamw(self.log_s, g_log_s, self.log_s_m, self.log_s_v, self.t, self.lr(self.cfg.lr_other))

    @property
    def s_arg(self):
        """s as the occupancy call takes it: log s on the device, or the fixed value."""
        return self.log_s if self.log_s is not None else self.s0

    @property
    def s(self) -> float:
        """Current s (reads the device value back when s is learnt)."""
        return float(torch.exp(self.log_s).item()) if self.log_s is not None else self.s0

    # ------------------------------------------------------- reference evaluation
    def reference_signal(self):
        """Full-space render of the current network on the uniform grid of the
        configured sample cube (lensless primary rays, c.lines x c.judge_nz
        depths, c.n_z by default)."""
        c = self.cfg
        xyz, _, origin = R.sample_points(c.cube_centre, c.cube_side / 2, (0.0, 0.0, 1.0), c.lines[0],
                                         c.lines[1], c.judge_nz or c.n_z, mode=R.SAMPLE_GRID, device=self.dev)
        f, grad, a = R.mlp_forward(self.net, xyz)
        phi_ray, phi_tx, _ = self.origin_occupancy(origin, self.tx)
        fl = R.Fields(sdf=f.view(xyz.shape[:2]), grad=grad.view(*xyz.shape[:2], 3),
                      refl=a.view(xyz.shape[:2]), s=self.s0, amp=1.0, amp_dev=self.amp,
                      log_s_dev=self.log_s, phi_ray=phi_ray, phi_tx=phi_tx)
        self._ref_xyz = xyz
        return R.render_forward(self.ap, R.Samples(xyz=xyz), fl, flags=c.render_flags)

    def evaluate(self, clean: torch.Tensor) -> dict:
        """Judge errors of the full-space render against a clean target signal:
        signal NRMSE, and NRMSE of the filter output (heatmap) on the full-space
        grid."""
        sig = self.reference_signal()
        _, p, _, p_ref = R.mf_forward(self.ap, self._ref_xyz, sig, clean)
        return {"signal": nrmse(sig, clean), "heatmap": nrmse(p, p_ref)}


class MultiPlaneTrainer(Trainer):
    """Training on several scanning planes with one shared network (the paper's
    multi-plane scans, Sec. Number of Radar Scanning Planes).  Each plane has its
    own aperture, primary direction (the plane normal), lensless primary rays
    through the sample cube with their own alpha/T scans, and its own measured
    signal.  A step visits ``planes_per_step`` planes in cyclic order; their
    heatmap losses add, the network and amplitude gradients accumulate
    (RFVR_ACCUMULATE), and one AdamW update follows.

    planes: list of dict(tx [n_meas, 3] float32, w [3] unit primary direction,
    offset: plane {x : x . w = offset}); targets: per-plane signals
    [n_meas, n_freq, 2]."""

    def __init__(self, cfg: StepConfig, params: torch.Tensor, planes, targets, device="cuda",
                 planes_per_step: Optional[int] = None):
        if cfg.bank_patch is not None:
            raise ValueError("the Signal Tracing Bank is per plane; not combined with multi-plane steps")
        super().__init__(cfg, params, targets[0], device)
        self.planes = []
        for pl, tg in zip(planes, targets):
            tx = torch.from_numpy(np.ascontiguousarray(pl["tx"], np.float32)).to(self.dev)
            self.planes.append({
                "tx": tx, "ap": R.Aperture(tx=tx, f0=self.f0, df=self.df, n_freq=cfg.n_freq),
                "w": tuple(float(v) for v in pl["w"]), "offset": float(pl["offset"]),
                "target": tg.to(self.dev).contiguous(), "p_star": None})
        self.pps = planes_per_step or len(self.planes)
        self.g_amp = torch.zeros(1, device=self.dev)
        self.loss_sum = torch.zeros(1, device=self.dev)

    def plane_samples(self, k: int):
        c, pl = self.cfg, self.planes[k]
        return R.sample_points(c.cube_centre, c.cube_side / 2, pl["w"], c.lines[0], c.lines[1], c.n_z,
                               mode=c.sampling, seed=c.seed, step=self.t * len(self.planes) + k,
                               device=self.dev, plane_offset=pl["offset"])

    def step(self, timers: Optional[dict] = None):
        c = self.cfg
        n_pl = len(self.planes)
        for j in range(self.pps):
            k = (self.t * self.pps + j) % n_pl
            pl = self.planes[k]
            xyz, u, origin = self.plane_samples(k)
            n_ray = origin.shape[0]
            res = self.reserve(xyz.shape[0] * xyz.shape[1])
            f, grad, a = R.mlp_forward(self.net, xyz, reserve=res)
            f_org, _, _ = R.mlp_forward(self.net, torch.cat([origin, pl["tx"]], 0))
            phi = R.occupancy(self.s_arg, f_org)
            sm = R.Samples(xyz=xyz)
            fl = R.Fields(sdf=f.view(xyz.shape[:2]), grad=grad.view(*xyz.shape[:2], 3),
                          refl=a.view(xyz.shape[:2]), s=self.s0, amp=1.0, amp_dev=self.amp,
                      log_s_dev=self.log_s,
                          phi_ray=phi[:n_ray].contiguous(), phi_tx=phi[n_ray:].contiguous())
            sig = R.render_forward(pl["ap"], sm, fl, flags=c.render_flags)
            if pl["p_star"] is None or c.sampling != R.SAMPLE_GRID:
                z, p, _, p_star = R.mf_forward(pl["ap"], xyz, sig, pl["target"])
                if c.sampling == R.SAMPLE_GRID:
                    pl["p_star"] = p_star
            else:
                z, p = R.mf_forward(pl["ap"], xyz, sig)
                p_star = pl["p_star"]
            loss, g_p = R.loss_l2(p, p_star)
            g_sig = R.mf_backward(pl["ap"], xyz, z, p, g_p)
            gr = R.render_backward(pl["ap"], sm, fl, g_sig, flags=c.render_flags)
            R.mlp_backward(self.net, xyz, gr["sdf"].view(-1), gr["grad"].view(-1, 3), gr["refl"].view(-1),
                           flags=R.ACCUMULATE if j > 0 else 0, out=self.g, reserve=res)
            if j == 0:
                self.g_amp.copy_(gr["amp"])
                self.loss_sum.copy_(loss)
            else:
                self.g_amp.add_(gr["amp"])
                self.loss_sum.add_(loss)
        self.t += 1
        P, G, M, V = self.net.params, self.g, self.m, self.v
        ns = self.n_sdf
        R.adamw(P[:ns], G[:ns], M[:ns], V[:ns], self.t, self.lr(c.lr_sdf))
        R.adamw(P[ns:], G[ns:], M[ns:], V[ns:], self.t, self.lr(c.lr_other))
        R.adamw(self.amp, self.g_amp, self.amp_m, self.amp_v, self.t, self.lr(c.lr_other))
        self.last = dict(loss=self.loss_sum)
        return self.loss_sum


def nrmse(sig: torch.Tensor, ref: torch.Tensor) -> float:
    """||sig - ref|| / ||ref|| over all measurements and frequencies."""
    return float(torch.linalg.vector_norm(sig - ref) / torch.linalg.vector_norm(ref))


@dataclass
class ProposalConfig:
    n_bins: int = 64
    n_imp: int = 16
    n_uni: int = 4
    pe_octaves: int = 4
    width: int = 64
    layers: int = 2
    lr: float = 1e-3
    train: bool = True          # False: the untrained control, a uniform pdf (stratified samples only)
    seed: int = 0
    loss_on_grid: bool = False  # heatmap loss on the full-space grid (its target cached) instead of
                                # at the drawn samples; the signal is still rendered from the samples
    dilate: int = 0             # targets dilated in depth over this many bins (rfvr_proposal_targets)
    full_every: int = 0         # every this many steps a full-space step (the fallback): it trains the
                                # network on the full grid and the proposal on the grid's blend weights
    jitter: bool = True         # False: every depth at the middle of its stratum (depths then move only
                                # with the proposal's pdf, not from step to step)


class ProposalTrainer(Trainer):
    """Training step with proposal-guided samples: the proposal network scores
    n_bins depth bins per primary ray, n_imp depths are drawn from its pdf and
    n_uni stratified uniform depths keep the whole range covered.  The SDF
    network is trained exactly as in full-space training (matched-filter loss,
    the measured signal's filter output recomputed at the new points); the
    proposal is trained on the render's own blend weights T alpha at the drawn
    depths (binned, normalised, BCE)."""

    def __init__(self, cfg: StepConfig, params: torch.Tensor, target_signal: torch.Tensor,
                 pcfg: ProposalConfig, prop_params: Optional[torch.Tensor] = None, device="cuda"):
        super().__init__(cfg, params, target_signal, device)
        self.pc = pcfg
        n_ray = cfg.lines[0] * cfg.lines[1]
        h = cfg.cube_side / 2
        self.bin_xyz, _, _ = R.sample_points(cfg.cube_centre, h, (0.0, 0.0, 1.0), cfg.lines[0], cfg.lines[1],
                                             pcfg.n_bins, mode=R.SAMPLE_GRID, device=self.dev)
        self.lo = float(np.float32(cfg.cube_centre[2]) - np.float32(h))
        self.hi = float(np.float32(cfg.cube_centre[2]) + np.float32(h))
        self.zero_logits = torch.zeros(n_ray, pcfg.n_bins, device=self.dev)
        self.prop = None
        if pcfg.train:
            if prop_params is None:
                from synth.mlp_init import ProposalSpec, proposal_init
                spec = ProposalSpec(pcfg.pe_octaves, pcfg.width, pcfg.layers, tuple(cfg.cube_centre), h)
                prop_params = torch.from_numpy(proposal_init(spec, pcfg.seed))
            self.prop = R.Proposal(params=prop_params.to(self.dev).contiguous(), pe_octaves=pcfg.pe_octaves,
                                   width=pcfg.width, layers=pcfg.layers, centre=tuple(cfg.cube_centre),
                                   half_size=h)
            npp = self.prop.param_count()
            assert self.prop.params.numel() == npp
            self.pg = torch.zeros(npp, device=self.dev)
            self.pm = torch.zeros(npp, device=self.dev)
            self.pv = torch.zeros(npp, device=self.dev)
        self.train_sdf = True
        self.keep_alpha = pcfg.full_every > 0

    def logits(self):
        n_ray = self.cfg.lines[0] * self.cfg.lines[1]
        if self.prop is None:
            return self.zero_logits
        return R.proposal_forward(self.prop, self.bin_xyz).view(n_ray, self.pc.n_bins)

    def proposal_samples(self, logits):
        c, pc = self.cfg, self.pc
        return R.sample_importance(c.cube_centre, c.cube_side / 2, (0.0, 0.0, 1.0), c.lines[0], c.lines[1],
                                   logits, pc.n_imp, pc.n_uni, seed=c.seed, step=self.t, jitter=pc.jitter)

    def full_step(self, timers: Optional[dict] = None):
        """A full-space step (the fallback): the network trains on the full grid
        as in Trainer.step, and the proposal on that render's blend weights
        binned over the grid's depths."""
        loss = Trainer.step(self, timers)
        if self.prop is not None:
            pc = self.pc
            u = self.last["u"]
            n_ray, n_z = u.shape
            logits = self.logits()
            t = R.proposal_targets(u, self.last["alpha"].view(n_ray, n_z), self.last["trans"].view(n_ray, n_z),
                                   self.lo, self.hi, pc.n_bins, pc.dilate)
            ploss, g_z = R.bce(logits, t)
            R.proposal_backward(self.prop, self.bin_xyz, g_z, out=self.pg)
            R.adamw(self.prop.params, self.pg, self.pm, self.pv, self.t, pc.lr)
            self.last_proposal_loss = ploss
        return loss

    def step(self, timers: Optional[dict] = None):
        c, pc = self.cfg, self.pc
        if pc.full_every and self.train_sdf and self.t % pc.full_every == 0:
            return self.full_step(timers)
        ev = timers

        def mark(name):
            if ev is not None:
                e = torch.cuda.Event(enable_timing=True)
                e.record()
                ev.setdefault(name, []).append(e)

        mark("start")
        logits = self.logits()
        xyz, u, origin = self.proposal_samples(logits)
        n_ray, K = u.shape
        mark("propose")
        res = self.reserve(n_ray * K) if self.train_sdf else None
        f, grad, a = R.mlp_forward(self.net, xyz, reserve=res)
        phi_ray, phi_tx, _ = self.origin_occupancy(origin, self.tx)
        mark("mlp_fwd")
        sm = R.Samples(xyz=xyz)
        fl = R.Fields(sdf=f.view(n_ray, K), grad=grad.view(n_ray, K, 3), refl=a.view(n_ray, K), s=self.s0,
                      amp=1.0, amp_dev=self.amp, log_s_dev=self.log_s, phi_ray=phi_ray, phi_tx=phi_tx)
        sig, alpha, trans = R.render_forward(self.ap, sm, fl, flags=c.render_flags, want_alpha=True)
        mark("render_fwd")
        self.t += 1
        loss = None
        if self.train_sdf:
            if pc.loss_on_grid:
                # the filter and the loss at the full-space grid, whose target
                # heatmap is fixed (computed once): the samples only render
                if self.p_star is None:
                    self.grid_xyz = R.sample_points(c.cube_centre, c.cube_side / 2, (0.0, 0.0, 1.0), c.lines[0],
                                                    c.lines[1], c.n_z, mode=R.SAMPLE_GRID, device=self.dev)[0]
                    _, self.p_star = R.mf_forward(self.ap, self.grid_xyz, self.target)
                xq, p_star = self.grid_xyz, self.p_star
                z, p = R.mf_forward(self.ap, xq, sig)
            else:
                xq = xyz
                z, p, _, p_star = R.mf_forward(self.ap, xq, sig, self.target)
            mark("mf_fwd")
            loss, g_p = R.loss_l2(p, p_star)
            g_sig = R.mf_backward(self.ap, xq, z, p, g_p)
            mark("mf_bwd")
            gr = R.render_backward(self.ap, sm, fl, g_sig, flags=c.render_flags)
            mark("render_bwd")
            R.mlp_backward(self.net, xyz, gr["sdf"].view(-1), gr["grad"].view(-1, 3), gr["refl"].view(-1),
                           out=self.g, reserve=res)
            mark("mlp_bwd")
            P, G, M, V = self.net.params, self.g, self.m, self.v
            ns = self.n_sdf
            R.adamw(P[:ns], G[:ns], M[:ns], V[:ns], self.t, self.lr(c.lr_sdf))
            R.adamw(P[ns:], G[ns:], M[ns:], V[ns:], self.t, self.lr(c.lr_other))
            R.adamw(self.amp, gr["amp"], self.amp_m, self.amp_v, self.t, self.lr(c.lr_other))
            mark("adamw")
            if c.learn_s:
                self.update_s(gr["s"])
        if self.prop is not None:
            t = R.proposal_targets(u, alpha.view(n_ray, K), trans.view(n_ray, K), self.lo, self.hi, pc.n_bins,
                                   pc.dilate)
            ploss, g_z = R.bce(logits, t)
            R.proposal_backward(self.prop, self.bin_xyz, g_z, out=self.pg)
            R.adamw(self.prop.params, self.pg, self.pm, self.pv, self.t, pc.lr)
            self.last_proposal_loss = ploss
            mark("proposal")
        self.last = dict(signal=sig, loss=loss, xyz=xyz, u=u, alpha=alpha, trans=trans)
        return loss

