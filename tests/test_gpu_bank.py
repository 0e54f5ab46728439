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


def test_stale_bank_rows_filter_and_step_against_oracle(dev):
    """Sec. Signal Tracing Bank against the FP64 oracle, with a network that
    changes every step (learning rates 1e-3): before each step the parameters
    and A' are snapshotted; the oracle renders each patch's rows with the
    snapshot of the step that traced them (the first step's fill with the
    first snapshot), assembles its own bank, filters the whole stale bank at
    the samples, takes the loss against the measured signal's filter output,
    and runs the patch's filter adjoint, render adjoint and network backward
    at that step's snapshot.  The GPU bank after every step, its filter output
    and the step's network gradient are compared with these."""
    print("[case] signal tracing bank vs oracle over a cycle of patches", flush=True)
    from oracle import mlp as omlp
    from oracle import render as orc
    from oracle import sampling as osmp
    from gpu_common import as_complex
    R, bk = _setup(dev, bank=True, lr=1e-3)
    c = bk.cfg
    spec = MLPSpec(n_layers=4, width=64, pe_octaves=3, head_width=64, head_layers=2,
                   centre=c.cube_centre, half_size=c.cube_side / 2)
    xyz, _, org = osmp.sample_points(c.cube_centre, c.cube_side / 2, (0.0, 0.0, 1.0), c.lines[0], c.lines[1],
                                     c.n_z)
    xyz = xyz.astype(np.float32).astype(np.float64)
    org = org.astype(np.float32).astype(np.float64)
    # both sides take the same float32 samples: the trainer's sampler is
    # replaced by these (the GPU sampler agrees with them to float32 rounding,
    # checked on its own elsewhere; one position ulp moves a phase by ~1e-4)
    gx = torch.from_numpy(xyz.astype(np.float32)).to(dev)
    go = torch.from_numpy(org.astype(np.float32)).to(dev)
    bk.samples = lambda: (gx, None, go)
    xq = xyz.reshape(-1, 3)
    shp = xyz.shape[:2]
    n_ray = org.shape[0]
    tx = bk.tx.cpu().numpy().astype(np.float64)          # patch-major order
    oap = orc.Aperture(tx=tx, f0=bk.f0, df=bk.df, n_freq=c.n_freq)
    tgt = bk.target.cpu().numpy().astype(np.float64)
    _, P_star = orc.mf(oap, xq, tgt[..., 0] + 1j * tgt[..., 1])
    L = bk.patch_len
    bank_o = None
    for t in range(bk.n_patch + 1):
        p_t = bk.net.params.detach().cpu().numpy().astype(np.float64)
        amp_t = float(bk.amp.item())
        bk.step()
        torch.cuda.synchronize()
        f, g, a = omlp.forward(p_t, spec, xq)
        f_o, _, _ = omlp.forward(p_t, spec, np.concatenate([org, tx], 0))
        phi = orc.logistic(c.s * f_o)
        F = orc.Fields(sdf=f.reshape(shp), grad=g.reshape(*shp, 3), refl=a.reshape(shp), s=c.s, amp=amp_t,
                       phi_ray=phi[:n_ray], phi_tx=phi[n_ray:])
        if bank_o is None:
            bank_o = orc.render(oap, xyz, F)
        k = t % bk.n_patch
        rows = slice(k * L, (k + 1) * L)
        oap_k = orc.Aperture(tx=tx[rows], f0=bk.f0, df=bk.df, n_freq=c.n_freq)
        F_k = orc.Fields(**{**F.__dict__, "phi_tx": phi[n_ray:][rows]})
        bank_o[rows] = orc.render(oap_k, xyz, F_k)
        z, P = orc.mf(oap, xq, bank_o)
        _, gP = orc.loss_l2(P, P_star)
        gsig = orc.mf_adjoint(oap_k, xq, z, P, gP)
        gr = orc.render_adjoint(oap_k, xyz, F_k, gsig)
        g_o = omlp.backward(p_t, spec, xq, gr["sdf"].ravel(), gr["grad"].reshape(-1, 3), gr["refl"].ravel())

        bank_g = as_complex(bk.bank)
        _, p_g = R.mf_forward(bk.ap, bk.samples()[0], bk.bank)
        e_rows = [rel_rms(bank_g[j * L:(j + 1) * L], bank_o[j * L:(j + 1) * L]) for j in range(bk.n_patch)]
        e_p = rel_rms(p_g.cpu().numpy(), P)
        g_g = bk.g.cpu().numpy().astype(np.float64)
        e_g = rel_rms(g_g, g_o)
        cos = float(g_g @ g_o / (np.linalg.norm(g_g) * np.linalg.norm(g_o)))
        print(f"step {t} (patch {k}): bank rows per patch rms rel {[f'{e:.1e}' for e in e_rows]}, "
              f"filter {e_p:.2e}, network gradient {e_g:.2e} (cosine {cos:.8f})")
        assert max(e_rows) <= 1e-4
        assert e_p <= 1e-4
        assert e_g <= 1e-3 and cos > 0.999999
