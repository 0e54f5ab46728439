"""GPU parity of the render's segment weight (RFVR_WEIGHT_SEGMENT): each
sample's segment to the next sample carries the exact integral of T^2 rho
over it, alpha T clamp(T (1 - alpha/2) + dPhi, 0, 1), at the segment's
midpoint.  Forward and adjoint against the FP64 oracle's weight="segment",
on ragged sizes with the lensless shift and ray weights, through both term
evaluations, and at the 2^20-point workload's size on sampled outputs."""
import numpy as np
import pytest
import torch

from oracle import render as orc
from gpu_common import as_complex, full_box_case, ragged_case, rel_rms

pytestmark = pytest.mark.gpu

SPEC = {"clamp": 0, "raw": 1, "off": 2}


def _R():
    from paper_2605_29097_amd import rfvr as R
    R.lib()
    return R


@pytest.mark.parametrize("spec", ["clamp", "raw", "off"])
def test_segment_render_forward_and_adjoint_ragged(dev, spec):
    print(f"[case] segment weight, ragged, spec={spec}", flush=True)
    R = _R()
    c = ragged_case(seed=4)
    # push the shifted transmittance past both clamps for some pairs
    rng = np.random.default_rng(41)
    c.phi_ray = rng.uniform(0.4, 0.8, c.xyz.shape[0]).astype(np.float32)
    c.phi_tx = rng.uniform(0.1, 1.0, c.tx.shape[0]).astype(np.float32)
    ap, sm, fl = c.g(dev)
    ref = orc.render(c.o_ap(), c.xyz, c.o_fields(), spec=spec, ray_w=c.ray_w, weight="segment")
    gs = rng.normal(size=ref.shape) + 1j * rng.normal(size=ref.shape)
    gt = torch.from_numpy(np.stack([gs.real, gs.imag], -1).astype(np.float32)).to(dev)
    ref_adj = orc.render_adjoint(c.o_ap(), c.xyz, c.o_fields(), gs.astype(np.complex64).astype(np.complex128),
                                 spec=spec, ray_w=c.ray_w, weight="segment")
    for flags in (0, R.TERMS_DIRECT):
        f = SPEC[spec] | R.WEIGHT_SEGMENT | flags
        sig = as_complex(R.render_forward(ap, sm, fl, flags=f))
        out = R.render_backward(ap, sm, fl, gt, flags=f)
        errs = {"signal": rel_rms(sig, ref)}
        for k in ("sdf", "grad", "refl"):
            errs[k] = rel_rms(out[k].cpu().numpy(), ref_adj[k])
        for k in ("amp", "s"):
            errs[k] = abs(out[k].item() - ref_adj[k]) / abs(ref_adj[k])
        print("direct" if flags else "moments", {k: f"{v:.2e}" for k, v in errs.items()})
        for k, v in errs.items():
            assert v <= 1e-4, (flags, k, v)
    # the weight differs from the sample weight on these samples
    assert rel_rms(orc.render(c.o_ap(), c.xyz, c.o_fields(), spec=spec, ray_w=c.ray_w), ref) > 1e-2


def test_segment_render_full_size_sampled(dev):
    """2^20 points x 1024 measurements x 128 frequencies: the forward at three
    measurements over all points, and the adjoint along six whole rays."""
    print("[case] segment weight, full size", flush=True)
    R = _R()
    c = full_box_case()
    ap, sm, fl = c.g(dev)
    sig = as_complex(R.render_forward(ap, sm, fl, flags=R.WEIGHT_SEGMENT))
    sel = np.array([0, 527, 1023])
    ref = orc.render(c.o_ap(sel), c.xyz, c.o_fields(), weight="segment")
    e = rel_rms(sig[sel], ref)
    print(f"forward at 3 measurements: rms rel {e:.2e}")
    assert e <= 1e-4
    rng = np.random.default_rng(13)
    gs = (rng.normal(size=(1024, 128)) + 1j * rng.normal(size=(1024, 128))).astype(np.complex64)
    out = R.render_backward(ap, sm, fl, torch.from_numpy(np.stack([gs.real, gs.imag], -1)).to(dev),
                            flags=R.WEIGHT_SEGMENT)
    rays = np.array([0, 2080, 2100, 2111, 4095])
    ref = orc.render_adjoint(c.o_ap(), c.xyz[rays], c.o_fields(rays=rays), gs.astype(np.complex128),
                             weight="segment")
    for k in ("sdf", "grad", "refl"):
        e = rel_rms(out[k].cpu().numpy()[rays], ref[k])
        print(f"adjoint {k} on 5 rays: rms rel {e:.2e}")
        assert e <= 1e-4, k
