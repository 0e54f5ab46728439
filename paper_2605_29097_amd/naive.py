"""Per-antenna ("naive") rendering: the brute-force Monte Carlo of Sec.
Integration that lensless sampling replaces.  Every antenna traces its own
rays (rfvr_sample_naive), so the network runs at n_ant x n_ray x n_z points and
each antenna's signal is rendered from its own samples alone, with transmittance
accumulated along its real rays and each sample weighted by its volume
(rfvr_samples.point_weight).  Used to validate the lensless approximation and
to measure what it saves."""
from __future__ import annotations

import torch

from . import rfvr as R


def render_naive(ap: R.Aperture, xyz: torch.Tensor, jac: torch.Tensor, sdf: torch.Tensor, grad: torch.Tensor,
                 refl: torch.Tensor, s: float, amp: float = 1.0, flags: int = 0) -> torch.Tensor:
    """signal [n_ant, n_freq, 2]; xyz [n_ant, n_ray, n_z, 3], jac / sdf / refl
    [n_ant, n_ray, n_z], grad [n_ant, n_ray, n_z, 3]."""
    n_ant = xyz.shape[0]
    sig = torch.empty(n_ant, ap.n_freq, 2, dtype=torch.float32, device=xyz.device)
    for i in range(n_ant):
        ap_i = R.Aperture(tx=ap.tx[i:i + 1], f0=ap.f0, df=ap.df, n_freq=ap.n_freq)
        sm = R.Samples(xyz=xyz[i], point_weight=jac[i])
        fl = R.Fields(sdf=sdf[i], grad=grad[i], refl=refl[i], s=s, amp=amp)
        R.render_forward(ap_i, sm, fl, flags=flags, out=sig[i:i + 1])
    return sig


def naive_forward(net: R.MLP, ap: R.Aperture, centre, half_extent, primary_dir, n_ray_x, n_ray_y, n_z,
                  s: float, amp: float = 1.0, flags: int = 0) -> torch.Tensor:
    """Per-antenna sampling, the network at every antenna's samples, and the
    per-antenna render: one forward pass of the brute-force method."""
    xyz, jac = R.sample_naive(centre, half_extent, primary_dir, n_ray_x, n_ray_y, n_z, ap.tx)
    f, g, a = R.mlp_forward(net, xyz.view(-1, 3))
    shp = xyz.shape[:3]
    return render_naive(ap, xyz, jac, f.view(shp), g.view(*shp, 3), a.view(shp), s, amp, flags)
