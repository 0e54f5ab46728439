"""Per-antenna ("naive") rendering on the GPU path.

  * rfvr_sample_naive against the oracle's per-antenna sampler;
  * the per-antenna render (point weights = volume Jacobian) against the FP64
    oracle (the oracle applies the Jacobian to the reflectiveness, which the
    amplitude is linear in);
  * the lensless approximation: lensless vs per-antenna render of a sphere in
    air, reported as its relative signal difference (the paper's App. B.2
    assumes equal occupancy at the two rays' origins; nothing here asserts
    the size of the approximation error)."""
import numpy as np
import pytest
import torch

from gpu_common import rel_rms
from oracle import render as orc
from oracle.sampling import sample_naive as o_naive
from synth import Sphere, freq_grid, planar_aperture, scene_fields

pytestmark = pytest.mark.gpu

C, H = (0.0, 0.0, 0.30), 0.05
SPH = Sphere((0.004, -0.003, 0.30), 0.03, 0.8)


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)


def test_naive_sampler_and_render_match_oracle(dev):
    print("[case] naive render 5x4 antennas, 10x8 rays x 24 depths", flush=True)
    from paper_2605_29097_amd import rfvr as R
    from paper_2605_29097_amd.naive import render_naive
    R.lib()
    tx = planar_aperture(5, 4, 2e-3)
    f0, df = freq_grid(20)
    xyz, jac = R.sample_naive(C, H, (0, 0, 1), 10, 8, 24, _t(tx, dev))
    xr, jr = o_naive(tx, C, H, (0, 0, 1), 10, 8, 24)
    assert np.abs(xyz.cpu().numpy() - xr).max() < 4e-8
    assert np.abs(jac.cpu().numpy() - jr).max() < 1e-6 * np.abs(jr).max()
    # both renders take the oracle sampler's points and volumes, rounded to float32
    x32 = xr.astype(np.float32)
    j32 = jr.astype(np.float32)
    sdf, grad, refl = scene_fields(SPH, x32)
    ap = R.Aperture(tx=_t(tx, dev), f0=f0, df=df, n_freq=20)
    sig = render_naive(ap, _t(x32, dev).view(xyz.shape), _t(j32, dev).view(jac.shape), _t(sdf, dev), _t(grad, dev),
                       _t(refl, dev), s=64.0)
    ref = np.empty((tx.shape[0], 20), np.complex128)
    for i in range(tx.shape[0]):
        F = orc.Fields(sdf=sdf[i].astype(np.float64), grad=grad[i].astype(np.float64),
                       refl=(refl[i].astype(np.float64) * j32[i].astype(np.float64)), s=64.0, amp=1.0)
        ref[i] = orc.render(orc.Aperture(tx=tx[i:i + 1].astype(np.float64), f0=f0, df=df, n_freq=20),
                            x32[i].astype(np.float64), F)[0]
    g = sig.cpu().numpy().astype(np.float64)
    e = rel_rms(g[..., 0] + 1j * g[..., 1], ref)
    print(f"naive render rms rel {e:.3e}")
    assert e <= 1e-4


def test_point_weights_rejected_by_the_adjoint(dev):
    from paper_2605_29097_amd import rfvr as R
    R.lib()
    xyz = torch.zeros(2, 3, 3, device=dev)
    w = torch.ones(2, 3, device=dev)
    ap = R.Aperture(tx=torch.zeros(1, 3, device=dev), f0=77e9, df=1e8, n_freq=4)
    fl = R.Fields(sdf=torch.ones(2, 3, device=dev), grad=torch.ones(2, 3, 3, device=dev),
                  refl=torch.ones(2, 3, device=dev))
    with pytest.raises(R.RfvrError):
        R.render_backward(ap, R.Samples(xyz=xyz, point_weight=w), fl, torch.zeros(1, 4, 2, device=dev))


def test_lensless_vs_naive_sphere_in_air(dev):
    print("[case] lensless vs per-antenna render, sphere in air", flush=True)
    from paper_2605_29097_amd import rfvr as R
    from paper_2605_29097_amd.naive import render_naive
    R.lib()
    tx = planar_aperture(8, 8, 2e-3)
    f0, df = freq_grid(32)
    ap = R.Aperture(tx=_t(tx, dev), f0=f0, df=df, n_freq=32)
    n = (48, 48, 96)
    xyz, jac = R.sample_naive(C, H, (0, 0, 1), *n, _t(tx, dev))
    x32 = xyz.cpu().numpy()
    sdf, grad, refl = scene_fields(SPH, x32)
    s_naive = render_naive(ap, xyz, jac, _t(sdf, dev), _t(grad, dev), _t(refl, dev), s=64.0)
    xl, _, _ = R.sample_points(C, H, (0, 0, 1), *n, device=dev)
    sl, gl, al = scene_fields(SPH, xl.cpu().numpy())
    s_lens = R.render_forward(ap, R.Samples(xyz=xl), R.Fields(sdf=_t(sl, dev), grad=_t(gl, dev),
                                                               refl=_t(al, dev), s=64.0))
    a = s_naive.cpu().numpy().astype(np.float64)
    b = s_lens.cpu().numpy().astype(np.float64)
    e = rel_rms(a[..., 0] + 1j * a[..., 1], b[..., 0] + 1j * b[..., 1])
    print(f"lensless vs per-antenna signal: rms relative difference {e:.3e}")
    assert np.isfinite(e)
