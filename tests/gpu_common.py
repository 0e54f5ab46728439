"""Shared helpers of the GPU parity tests: seeded synthetic cases built from
``synth`` and handed identically to the oracle (float64, CPU) and to librfvr."""
from __future__ import annotations

import numpy as np

from oracle import render as orc
from synth import (Box, Sphere, freq_grid, line_points, planar_aperture, scene_fields)
from synth.configs import small_sphere_centre


def rel_rms(got, ref):
    got = np.asarray(got)
    ref = np.asarray(ref)
    return float(np.linalg.norm((got - ref).ravel()) / max(np.linalg.norm(ref.ravel()), 1e-300))


def max_rel(got, ref):
    got = np.asarray(got)
    ref = np.asarray(ref)
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def as_complex(t):
    a = t.detach().cpu().numpy().astype(np.float64)
    return a[..., 0] + 1j * a[..., 1]


class Case:
    """One render problem: aperture, points, fields (float32 numpy)."""

    def __init__(self, tx, f0, df, n_freq, xyz, sdf, grad, refl, s=64.0, amp=1.0,
                 phi_ray=None, phi_tx=None, ray_w=None, rx=None, phi_rx=None):
        self.tx = np.ascontiguousarray(tx, np.float32)
        self.rx = None if rx is None else np.ascontiguousarray(rx, np.float32)
        self.phi_rx = None if phi_rx is None else np.ascontiguousarray(phi_rx, np.float32)
        self.f0, self.df, self.n_freq = f0, df, n_freq
        self.xyz = np.ascontiguousarray(xyz, np.float32)
        self.sdf = np.ascontiguousarray(sdf, np.float32)
        self.grad = np.ascontiguousarray(grad, np.float32)
        self.refl = np.ascontiguousarray(refl, np.float32)
        self.s, self.amp = float(s), float(amp)
        self.phi_ray = None if phi_ray is None else np.ascontiguousarray(phi_ray, np.float32)
        self.phi_tx = None if phi_tx is None else np.ascontiguousarray(phi_tx, np.float32)
        self.ray_w = None if ray_w is None else np.ascontiguousarray(ray_w, np.float32)

    # oracle side
    def o_ap(self, sel=None):
        pick = lambda a: None if a is None else (a if sel is None else a[sel]).astype(np.float64)
        return orc.Aperture(tx=pick(self.tx), f0=self.f0, df=self.df, n_freq=self.n_freq, rx=pick(self.rx))

    def o_fields(self, rays=None, sel=None):
        r = slice(None) if rays is None else rays
        return orc.Fields(sdf=self.sdf[r], grad=self.grad[r], refl=self.refl[r], s=self.s, amp=self.amp,
                          phi_ray=None if self.phi_ray is None else self.phi_ray[r],
                          phi_tx=None if self.phi_tx is None else
                          (self.phi_tx if sel is None else self.phi_tx[sel]),
                          phi_rx=None if self.phi_rx is None else
                          (self.phi_rx if sel is None else self.phi_rx[sel]))

    # GPU side
    def g(self, dev):
        import torch
        from paper_2605_29097_amd import rfvr as R
        t = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        ap = R.Aperture(tx=t(self.tx), f0=self.f0, df=self.df, n_freq=self.n_freq, rx=t(self.rx))
        sm = R.Samples(xyz=t(self.xyz), ray_weight=t(self.ray_w))
        fl = R.Fields(sdf=t(self.sdf), grad=t(self.grad), refl=t(self.refl), s=self.s, amp=self.amp,
                      phi_ray=t(self.phi_ray), phi_tx=t(self.phi_tx), phi_rx=t(self.phi_rx))
        return ap, sm, fl


def small_sphere_case(seed=0):
    """8x8 aperture at 2 mm, 32 freqs 77-81 GHz, 16^3 points in a 10 cm cube,
    sphere R = 3 cm at (0,0,0.30) + seeded +-5 mm, s = 64, a = 0.8, A' = 1."""
    f0, df = freq_grid(32)
    tx = planar_aperture(8, 8, 2e-3)
    xyz, _ = line_points((0.0, 0.0, 0.30), 0.10, 16, 16, 16)
    sdf, grad, refl = scene_fields(Sphere(small_sphere_centre(seed), 0.03, 0.8), xyz)
    return Case(tx, f0, df, 32, xyz, sdf, grad, refl, s=64.0, amp=1.0)


def ragged_case(seed=1, n_ax=(7, 5), n_freq=45, lines=(13, 1), n_z=70, phi=True, weights=True):
    """Odd sizes on purpose: 35 measurements, 45 frequencies, 70 samples per ray,
    lensless origin shift and per-ray weights on."""
    rng = np.random.default_rng(seed)
    f0, df = freq_grid(n_freq)
    tx = planar_aperture(n_ax[0], n_ax[1], 2e-3) + rng.uniform(-2e-4, 2e-4, (n_ax[0] * n_ax[1], 3)).astype(np.float32)
    xyz, _ = line_points((0.0, 0.0, 0.30), 0.08, lines[0], lines[1], n_z, jitter_seed=seed)
    sph = Sphere((0.003, -0.002, 0.30), 0.025, 0.8)
    sdf, grad, refl = scene_fields(sph, xyz)
    grad = grad + rng.normal(0, 0.05, grad.shape).astype(np.float32)
    refl = refl * rng.uniform(0.6, 1.0, refl.shape).astype(np.float32)
    n_ray = xyz.shape[0]
    return Case(tx, f0, df, n_freq, xyz, sdf, grad, refl, s=48.0, amp=1.7,
                phi_ray=rng.uniform(0.97, 1.0, n_ray) if phi else None,
                phi_tx=rng.uniform(0.97, 1.0, tx.shape[0]) if phi else None,
                ray_w=rng.uniform(0.5, 1.5, n_ray) if weights else None)


def full_box_case():
    """The 2^20-point workload: 32x32 aperture, 128 freqs, 64x64 lines x 256 depths
    in a 20 cm cube at 0.30 m, analytic box 8x6x4 cm (a = 0.8)."""
    f0, df = freq_grid(128)
    tx = planar_aperture(32, 32, 2e-3)
    xyz, _ = line_points((0.0, 0.0, 0.30), 0.20, 64, 64, 256)
    sdf, grad, refl = scene_fields(Box((0.0, 0.0, 0.30), (0.04, 0.03, 0.02), 0.8), xyz)
    return Case(tx, f0, df, 128, xyz, sdf, grad, refl, s=64.0, amp=1.0)
