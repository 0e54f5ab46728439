"""The proposal trainer's full-space fallback step (ProposalConfig.full_every).

Every full_every-th step of a proposal run is a full-space step: the network
trains on the full grid exactly as the full-space trainer's step does, and the
proposal network trains on that dense render's blend weights.  Checked on the
2^20-point workload: the fallback step leaves the network, amplitude and
optimiser moments bitwise equal to a full-space trainer's first step from the
same parameters; the proposal's parameters move, with a finite loss; the
steps in between take the proposal's samples."""
import os

import numpy as np
import pytest
import torch

from synth import MLPSpec, mlp_init

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def test_fallback_step_is_the_full_space_step(dev):
    print("[case] proposal fallback step vs full-space step, 2^20 points", flush=True)
    from paper_2605_29097_amd import rfvr as R
    from paper_2605_29097_amd.train import ProposalConfig, ProposalTrainer, StepConfig, Trainer
    R.lib()
    cfg = StepConfig()
    spec = MLPSpec(centre=cfg.cube_centre, half_size=cfg.cube_side / 2)
    params = torch.from_numpy(mlp_init(spec, 0))
    data = np.load(os.path.join(HERE, "golden", "box_target.npz"))
    noisy = data["noisy"]
    target = torch.from_numpy(np.stack([noisy.real, noisy.imag], -1).astype(np.float32))
    full = Trainer(cfg, params.clone(), target, device=dev)
    hyb = ProposalTrainer(cfg, params.clone(), target, ProposalConfig(full_every=2), device=dev)
    p0 = hyb.prop.params.clone()
    full.step()
    hyb.step()                                              # t = 0: the fallback step
    torch.cuda.synchronize()
    assert torch.equal(hyb.net.params, full.net.params)
    assert torch.equal(hyb.m, full.m) and torch.equal(hyb.v, full.v)
    assert torch.equal(hyb.amp, full.amp)
    assert hyb.last["u"].shape == (cfg.lines[0] * cfg.lines[1], cfg.n_z)
    assert not torch.equal(hyb.prop.params, p0)
    assert torch.isfinite(hyb.last_proposal_loss).all()
    hyb.step()                                              # t = 1: a proposal step
    n_ray = cfg.lines[0] * cfg.lines[1]
    assert hyb.last["u"].shape == (n_ray, hyb.pc.n_imp + hyb.pc.n_uni)
    assert torch.isfinite(hyb.last["loss"]).all()
    hyb.step()                                              # t = 2: the fallback again
    assert hyb.last["u"].shape == (n_ray, cfg.n_z)
    assert torch.isfinite(hyb.net.params).all()
