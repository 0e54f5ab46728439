"""Signal Tracing Bank (Sec. Signal Tracing Bank) on the GPU path.

With the network held fixed (learning rate 0) the bank stays exact, so:
  * the bank filled at the first step equals the full-aperture render;
  * every patch step sees the full-aperture loss;
  * the patch gradients of one cycle over all patches sum to the gradient of
    one full-aperture step (the filter adjoint's rows are split by patch and
    the render adjoint is linear in them).
Then a few steps with the paper's learning rates check the bank keeps its
untouched rows and refreshes the traced patch."""
import numpy as np
import pytest
import torch

from gpu_common import rel_rms
from synth import MLPSpec, mlp_init

pytestmark = pytest.mark.gpu


def _setup(dev, bank, lr=0.0):
    from paper_2605_29097_amd import rfvr as R
    from paper_2605_29097_amd.train import StepConfig, Trainer
    R.lib()
    cfg = StepConfig(ap=(8, 8), n_freq=32, cube_side=0.10, lines=(16, 16), n_z=32, n_layers=4, width=64,
                     pe_octaves=3, head_width=64, head_layers=2, lr_sdf=lr, lr_other=lr,
                     bank_patch=(4, 4) if bank else None)
    spec = MLPSpec(n_layers=4, width=64, pe_octaves=3, head_width=64, head_layers=2,
                   centre=cfg.cube_centre, half_size=cfg.cube_side / 2)
    p = mlp_init(spec, 2).astype(np.float64)
    p = (p + 0.2 * np.random.default_rng(3).normal(size=p.shape) / 8.0).astype(np.float32)
    rng = np.random.default_rng(4)
    target = torch.from_numpy(rng.normal(size=(64, 32, 2)).astype(np.float32) * 1e-3)
    return R, Trainer(cfg, torch.from_numpy(p), target, device=dev)


def test_bank_fill_loss_and_gradient_partition(dev):
    print("[case] signal tracing bank: fill, loss, gradient partition", flush=True)
    R, full = _setup(dev, bank=False)
    _, bk = _setup(dev, bank=True)
    L_full = full.step()
    g_full = full.g.clone()
    sig_full = full.last["signal"]
    perm = torch.from_numpy(bk.perm).to(dev)
    g_sum = torch.zeros_like(g_full)
    losses = []
    for k in range(bk.n_patch):
        L = bk.step()
        if k == 0:
            e_fill = rel_rms(bk.bank.cpu().numpy(), sig_full[perm].cpu().numpy())
        losses.append(L.item())
        g_sum += bk.g
    e_g = rel_rms(g_sum.cpu().numpy(), g_full.cpu().numpy())
    print(f"bank vs full render rms rel {e_fill:.2e}; losses {losses} vs {L_full.item():.6e}; "
          f"gradient partition rms rel {e_g:.2e}")
    assert e_fill <= 1e-5
    for L in losses:
        assert abs(L - L_full.item()) <= 1e-5 * abs(L_full.item())
    assert e_g <= 1e-4


def test_bank_refreshes_only_the_traced_patch(dev):
    print("[case] signal tracing bank: refresh", flush=True)
    R, bk = _setup(dev, bank=True, lr=1e-3)
    bk.step()                                   # fills the bank, traces patch 0, updates the network
    before = bk.bank.clone()
    bk.step()                                   # traces patch 1 with the updated network
    after = bk.bank
    L = bk.patch_len
    changed = [(after[k * L:(k + 1) * L] != before[k * L:(k + 1) * L]).any().item() for k in range(bk.n_patch)]
    print(f"rows changed per patch: {changed}")
    assert changed == [False, True, False, False]
