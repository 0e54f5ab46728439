"""One training step of the lensless RF renderer (GeRaF, Sec. Overview steps 1-5),
driven through the C ABI with explicit forward / adjoint calls.

step():
  1. lensless primary-ray samples (Sec. Lensless Sampling)          rfvr_sample_points
  2. SDF network at the samples: f, grad_x f, a                      rfvr_mlp_forward
     and at the ray / antenna origins: detached Phi (Eq. lens-less-transmittance)
  3. signal tracing with lensless alpha blending (Eq. ref_sim)       rfvr_render_forward
  4. matched filter at the samples (Eq. mf-sm)                      rfvr_mf_forward
  5. L2 loss against the measured signal's filter output             rfvr_loss_l2
  then the adjoints in reverse (rfvr_mf_backward, rfvr_render_backward,
  rfvr_mlp_backward) and AdamW with cosine annealing (App. C)        rfvr_adamw
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
    spec_flags: int = R.SPEC_CLAMP

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


class Trainer:
    """State of one reconstruction: network, amplitude, optimiser moments, target."""

    def __init__(self, cfg: StepConfig, params: torch.Tensor, target_signal: torch.Tensor,
                 device="cuda"):
        self.cfg = cfg
        self.dev = torch.device(device)
        f0 = cfg.f_lo
        df = 0.0 if cfg.n_freq == 1 else (cfg.f_hi - cfg.f_lo) / (cfg.n_freq - 1)
        self.tx = torch.from_numpy(aperture_positions(cfg)).to(self.dev)
        self.ap = R.Aperture(tx=self.tx, f0=f0, df=df, n_freq=cfg.n_freq)
        self.net = R.MLP(params=params.to(self.dev).contiguous(), n_layers=cfg.n_layers,
                         width=cfg.width, pe_octaves=cfg.pe_octaves, head_width=cfg.head_width,
                         head_layers=cfg.head_layers, beta=cfg.beta,
                         centre=tuple(cfg.cube_centre), half_size=cfg.cube_side / 2)
        n_par = self.net.param_count()
        assert self.net.params.numel() == n_par
        self.m = torch.zeros(n_par, device=self.dev)
        self.v = torch.zeros(n_par, device=self.dev)
        self.g = torch.zeros(n_par, device=self.dev)
        # the SDF branch (trunk + sdf output) comes first in the flat layout
        w, L, in0 = cfg.width, cfg.n_layers, 3 + 6 * cfg.pe_octaves
        self.n_sdf = w * in0 + w + (L - 1) * (w * w + w) + w + 1
        self.amp = torch.tensor([cfg.amp0], device=self.dev)
        self.amp_m = torch.zeros(1, device=self.dev)
        self.amp_v = torch.zeros(1, device=self.dev)
        self.target = target_signal.to(self.dev).contiguous()
        self.t = 0
        self.p_star = None
        self._xyz_key = None
        self.origin_pts = None

    # ------------------------------------------------------------------ helpers
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
        f, grad, a = R.mlp_forward(self.net, xyz)
        # detached occupancies at the primary-ray origins and the antennas
        org = torch.cat([origin, self.tx], 0)
        f_org, _, _ = R.mlp_forward(self.net, org)
        phi = R.occupancy(c.s, f_org)
        mark("mlp_fwd")
        sm = R.Samples(xyz=xyz)
        fl = R.Fields(sdf=f.view(xyz.shape[:2]), grad=grad.view(*xyz.shape[:2], 3),
                      refl=a.view(xyz.shape[:2]), s=c.s, amp=1.0, amp_dev=self.amp,
                      phi_ray=phi[:origin.shape[0]].contiguous(), phi_tx=phi[origin.shape[0]:].contiguous())
        sig = R.render_forward(self.ap, sm, fl, flags=c.spec_flags)
        mark("render_fwd")
        key = (c.sampling, None if c.sampling == R.SAMPLE_GRID else self.t)
        if self.p_star is None or key != self._xyz_key:
            z, p, _, p_star = R.mf_forward(self.ap, xyz, sig, self.target)
            self.p_star, self._xyz_key = p_star, key
        else:
            z, p = R.mf_forward(self.ap, xyz, sig)
        mark("mf_fwd")
        loss, g_p = R.loss_l2(p, self.p_star)
        g_sig = R.mf_backward(self.ap, xyz, z, p, g_p)
        mark("mf_bwd")
        gr = R.render_backward(self.ap, sm, fl, g_sig, flags=c.spec_flags)
        mark("render_bwd")
        R.mlp_backward(self.net, xyz, gr["sdf"].view(-1), gr["grad"].view(-1, 3), gr["refl"].view(-1),
                       out=self.g)
        mark("mlp_bwd")
        self.t += 1
        P, G, M, V = self.net.params, self.g, self.m, self.v
        ns = self.n_sdf
        R.adamw(P[:ns], G[:ns], M[:ns], V[:ns], self.t, self.lr(c.lr_sdf))
        R.adamw(P[ns:], G[ns:], M[ns:], V[ns:], self.t, self.lr(c.lr_other))
        R.adamw(self.amp, gr["amp"], self.amp_m, self.amp_v, self.t, self.lr(c.lr_other))
        mark("adamw")
        self.last = dict(signal=sig, loss=loss)
        return loss

