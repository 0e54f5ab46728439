"""A learnable s kept on the device as log s (rfvr_fields.log_s_ptr): the render
and its adjoint read s = exp(log s) at kernel time and return the gradient in
log s; the trainer updates log s with rfvr_adamw, with no host round trip."""
import math

import numpy as np
import pytest
import torch

from gpu_common import as_complex, ragged_case, rel_rms

pytestmark = pytest.mark.gpu


def test_log_s_on_the_device_matches_the_host_value(dev):
    print("[case] render / adjoint / occupancy with log s on the device", flush=True)
    from paper_2605_29097_amd import rfvr as R
    R.lib()
    c = ragged_case(seed=7)
    ap, sm, fl = c.g(dev)
    log_s = torch.tensor([math.log(c.s)], device=dev)
    s_dev = float(torch.exp(log_s).item())               # the value the kernels use
    fl_h = R.Fields(sdf=fl.sdf, grad=fl.grad, refl=fl.refl, s=s_dev, amp=fl.amp, phi_ray=fl.phi_ray,
                    phi_tx=fl.phi_tx)
    fl_d = R.Fields(sdf=fl.sdf, grad=fl.grad, refl=fl.refl, s=1.0, amp=fl.amp, phi_ray=fl.phi_ray,
                    phi_tx=fl.phi_tx, log_s_dev=log_s)
    for flags in (0, R.WEIGHT_SEGMENT):
        a = as_complex(R.render_forward(ap, sm, fl_h, flags=flags))
        b = as_complex(R.render_forward(ap, sm, fl_d, flags=flags))
        assert rel_rms(b, a) <= 1e-6
        rng = np.random.default_rng(3)
        gs = rng.normal(size=(c.tx.shape[0], c.n_freq, 2)).astype(np.float32)
        gh = R.render_backward(ap, sm, fl_h, torch.from_numpy(gs).to(dev), flags=flags)
        gd = R.render_backward(ap, sm, fl_d, torch.from_numpy(gs).to(dev), flags=flags)
        for k in ("sdf", "grad", "refl", "amp"):
            assert rel_rms(gd[k].cpu().numpy(), gh[k].cpu().numpy()) <= 1e-5, k
        e = abs(gd["s"].item() - s_dev * gh["s"].item()) / abs(s_dev * gh["s"].item())
        print(f"flags {flags}: dL/dlog s {gd['s'].item():.6e} vs s dL/ds {s_dev * gh['s'].item():.6e} ({e:.1e})")
        assert e <= 1e-5
    f = torch.linspace(-0.05, 0.05, 1001, device=dev)
    assert torch.allclose(R.occupancy(log_s, f), R.occupancy(s_dev, f), rtol=0, atol=2e-7)


def test_trainer_updates_log_s_on_the_device(dev):
    print("[case] trainer with learnable s: AdamW step on log s on the device", flush=True)
    from paper_2605_29097_amd import rfvr as R
    from paper_2605_29097_amd.train import StepConfig, Trainer
    from synth import MLPSpec, mlp_init
    R.lib()
    cfg = StepConfig(ap=(4, 4), n_freq=16, cube_side=0.08, lines=(6, 6), n_z=16, n_layers=3, width=64,
                     pe_octaves=2, head_width=64, head_layers=1, s=64.0, learn_s=True)
    spec = MLPSpec(n_layers=3, width=64, pe_octaves=2, head_width=64, head_layers=1, centre=cfg.cube_centre,
                   half_size=cfg.cube_side / 2)
    target = torch.from_numpy(np.random.default_rng(1).normal(size=(16, 16, 2)).astype(np.float32) * 1e-2)
    tr = Trainer(cfg, torch.from_numpy(mlp_init(spec, 1)), target, device=dev)
    before = tr.log_s.clone()
    tr.step()
    torch.cuda.synchronize()
    d = float((tr.log_s - before).abs().item())
    lr1 = tr.lr(cfg.lr_other)
    # AdamW's first step moves log s by lr (bias-corrected m / sqrt(v) = sign(g))
    print(f"|d log s| after one step {d:.7f}, lr {lr1:.7f}; s = {tr.s:.4f}")
    assert 0.99 * lr1 <= d <= lr1 * (1 + 1e-6)
