"""The two evaluations of the term sums (Chebyshev moments by default,
per-frequency with RFVR_TERMS_DIRECT) against the FP64 oracle's direct sums.

The order K the device plans is checked against the documented rule
(bounding box of the points -> per-measurement range half-width h ->
z = 2 pi ((n_freq - 1) / 2) 2 df h / c, the band split at its centre ->
smallest K in {24, 28, 32, 40, 48, 64}, below n_freq, with
2 (z/2)^K / K! / (1 - z/(2K+2)) <= 1e-6, else 0).  One case per order band
(and one past the last, which falls back to the per-frequency kernels): the
four term entry points match the oracle within 1e-4 RMS relative error on
both paths.  At the benchmark size the two paths agree element by element and
the plan picks K = 24."""
import math

import numpy as np
import pytest
import torch

from oracle import render as orc
from gpu_common import Case, as_complex, full_box_case, rel_rms
from synth import Sphere, line_points, planar_aperture, scene_fields

pytestmark = pytest.mark.gpu

C0 = 299792458.0
ORDERS = (24, 28, 32, 40, 48, 64)


def _R():
    from paper_2605_29097_amd import rfvr as R
    R.lib()
    return R


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _half_widths(tx, xyz):
    p = xyz.reshape(-1, 3).astype(np.float64)
    lo, hi = p.min(0), p.max(0)
    h = []
    for t in tx.astype(np.float64):
        rlo = np.linalg.norm(np.maximum(np.maximum(lo - t, t - hi), 0.0))
        rhi = np.linalg.norm(np.maximum(np.abs(t - lo), np.abs(t - hi)))
        h.append(0.5 * (rhi - rlo) * (1 + 1e-12) + 1e-12 * (rhi + 1.0))
    return np.array(h)


def expected_order(tx, xyz, n_freq, df):
    z = 2 * math.pi * (0.5 * (n_freq - 1)) * (2 * df / C0) * _half_widths(tx, xyz).max()
    for K in ORDERS:
        if K >= n_freq:
            break
        q = z / 2
        if q <= 0:
            return K
        if q >= K + 1:
            continue
        lb = K * math.log(q) - math.lgamma(K + 1) + math.log(2) - math.log1p(-q / (K + 1))
        if lb <= math.log(1e-6):
            return K
    return 0


def band_case(z_target, n_freq=96, seed=0):
    """8x8 aperture at 2 mm, 16 x 16 rays x 16 depths in a 10 cm cube at
    0.30 m, sphere R = 3 cm; df set so that the widest measurement has the
    given z."""
    tx = planar_aperture(8, 8, 2e-3)
    xyz, _ = line_points((0.0, 0.0, 0.30), 0.10, 16, 16, 16, jitter_seed=seed)
    hmax = _half_widths(tx, xyz).max()
    df = z_target / (2 * math.pi * (0.5 * (n_freq - 1)) * 2 * hmax / C0)
    sdf, grad, refl = scene_fields(Sphere((0.004, -0.003, 0.302), 0.03, 0.8), xyz)
    rng = np.random.default_rng(seed)
    phi_ray = rng.uniform(0.0, 0.2, xyz.shape[0]).astype(np.float32)
    phi_tx = rng.uniform(0.0, 0.2, tx.shape[0]).astype(np.float32)
    return Case(tx, 77e9, df, n_freq, xyz, sdf, grad, refl, s=64.0, amp=1.3, phi_ray=phi_ray, phi_tx=phi_tx)


BANDS = [(6.0, 24), (12.0, 28), (14.0, 32), (18.0, 40), (24.0, 48), (33.0, 64), (45.0, 0)]


@pytest.mark.parametrize("z,K", BANDS, ids=[f"K{k}" for _, k in BANDS])
def test_term_paths_match_the_oracle_in_every_order_band(dev, z, K):
    _say(f"term sums, order band K={K} (z={z})")
    R = _R()
    c = band_case(z)
    assert expected_order(c.tx, c.xyz, c.n_freq, c.df) == K
    ap, sm, fl = c.g(dev)
    assert R.term_order(ap, sm.xyz) == K
    rng = np.random.default_rng(int(z * 10))
    M, NF = c.tx.shape[0], c.n_freq
    s = rng.normal(size=(M, NF)) + 1j * rng.normal(size=(M, NF))
    st = torch.from_numpy(np.stack([s.real, s.imag], -1).astype(np.float32)).to(dev)
    sf = s.astype(np.complex64).astype(np.complex128)
    nq = c.xyz.shape[0] * c.xyz.shape[1]
    gP = rng.normal(size=nq).astype(np.float32)
    ref_sig = orc.render(c.o_ap(), c.xyz, c.o_fields())
    zr, pr = orc.mf(c.o_ap(), c.xyz.reshape(-1, 3), sf)
    ref_adj = orc.render_adjoint(c.o_ap(), c.xyz, c.o_fields(), sf)
    for flags in (0, R.TERMS_DIRECT):
        tag = "direct" if flags else "default"
        sig = as_complex(R.render_forward(ap, sm, fl, flags=flags))
        z_, p_ = R.mf_forward(ap, sm.xyz, st, flags=flags)
        g = as_complex(R.mf_backward(ap, sm.xyz, z_, p_, torch.from_numpy(gP).to(dev), flags=flags))
        # the oracle adjoint at its own z and P (no GPU output as oracle input)
        gr = orc.mf_adjoint(c.o_ap(), c.xyz.reshape(-1, 3), zr, pr, gP.astype(np.float64))
        adj = R.render_backward(ap, sm, fl, st, flags=flags)
        errs = {"render": rel_rms(sig, ref_sig), "mf z": rel_rms(as_complex(z_), zr),
                "mf P": rel_rms(p_.cpu().numpy(), pr), "mf adjoint": rel_rms(g, gr)}
        for k in ("sdf", "grad", "refl"):
            errs[f"render adjoint {k}"] = rel_rms(adj[k].cpu().numpy(), ref_adj[k])
        print(tag, {k: f"{v:.2e}" for k, v in errs.items()})
        for k, v in errs.items():
            assert v <= 1e-4, (tag, k, v)


def test_term_order_at_full_size_and_paths_agree(dev):
    """2^20 points x 1024 measurements x 128 frequencies: the plan takes K = 24
    and both evaluations give the same outputs to 1e-4 (all elements)."""
    _say("term sums full size: order and path agreement")
    R = _R()
    c = full_box_case()
    ap, sm, fl = c.g(dev)
    assert expected_order(c.tx, c.xyz, c.n_freq, c.df) == 24
    assert R.term_order(ap, sm.xyz) == 24
    a = as_complex(R.render_forward(ap, sm, fl))
    b = as_complex(R.render_forward(ap, sm, fl, flags=R.TERMS_DIRECT))
    e = rel_rms(a, b)
    print(f"render forward default vs direct: {e:.2e}")
    assert e <= 1e-4
    rng = np.random.default_rng(12)
    s = (rng.normal(size=(1024, 128)) + 1j * rng.normal(size=(1024, 128))).astype(np.complex64)
    st = torch.from_numpy(np.stack([s.real, s.imag], -1)).to(dev)
    za, pa = R.mf_forward(ap, sm.xyz, st)
    zb, pb = R.mf_forward(ap, sm.xyz, st, flags=R.TERMS_DIRECT)
    e = rel_rms(as_complex(za), as_complex(zb))
    print(f"mf forward default vs direct: {e:.2e}")
    assert e <= 1e-4
    gP = torch.from_numpy(rng.normal(size=za.shape[0]).astype(np.float32)).to(dev)
    ga = as_complex(R.mf_backward(ap, sm.xyz, za, pa, gP))
    gb = as_complex(R.mf_backward(ap, sm.xyz, za, pa, gP, flags=R.TERMS_DIRECT))
    e = rel_rms(ga, gb)
    print(f"mf adjoint default vs direct: {e:.2e}")
    assert e <= 1e-4
    ra = R.render_backward(ap, sm, fl, st)
    rb = R.render_backward(ap, sm, fl, st, flags=R.TERMS_DIRECT)
    for k in ("sdf", "grad", "refl"):
        e = rel_rms(ra[k].cpu().numpy(), rb[k].cpu().numpy())
        print(f"render adjoint {k} default vs direct: {e:.2e}")
        assert e <= 1e-4


def test_term_order_single_point_and_accumulate(dev):
    """Degenerate box (one point: h at its floor, x = 0) and RFVR_ACCUMULATE of
    the filter adjoint through the moment path."""
    _say("term sums: single point, accumulate")
    R = _R()
    tx = planar_aperture(4, 4, 2e-3)
    xyz = np.array([[[0.01, -0.02, 0.31]]], np.float32)
    sdf, grad, refl = scene_fields(Sphere((0.0, 0.0, 0.30), 0.01, 0.8), xyz)
    c = Case(tx, 77e9, 4e9 / 63, 64, xyz, sdf - 0.5, grad, refl)
    ap, sm, fl = c.g(dev)
    assert R.term_order(ap, sm.xyz) == 24
    rng = np.random.default_rng(2)
    s = (rng.normal(size=(16, 64)) + 1j * rng.normal(size=(16, 64))).astype(np.complex64)
    st = torch.from_numpy(np.stack([s.real, s.imag], -1)).to(dev)
    z_, p_ = R.mf_forward(ap, sm.xyz, st)
    zr, pr = orc.mf(c.o_ap(), xyz.reshape(-1, 3), s.astype(np.complex128))
    assert rel_rms(as_complex(z_), zr) <= 1e-5
    gP = torch.ones(1, device=dev)
    g1 = R.mf_backward(ap, sm.xyz, z_, p_, gP)
    g2 = R.mf_backward(ap, sm.xyz, z_, p_, gP, flags=R.ACCUMULATE, out=g1.clone())
    gr = orc.mf_adjoint(c.o_ap(), xyz.reshape(-1, 3), zr, pr, np.ones(1))
    assert rel_rms(as_complex(g1), gr) <= 1e-5
    assert rel_rms(as_complex(g2), 2 * gr) <= 1e-5
