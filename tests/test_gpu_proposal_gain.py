"""What the trained proposal gains over sampling without it.

The SDF network is held at its geometric initialisation (a sphere of radius
5 cm at the centre of a 20 cm sample cube) and only the proposal network is
trained, on the blend weights T alpha that the library's own render returns at
the proposal's samples.  The reference is a dense full-space render on the uniform
64 x 64 x 256 grid: its blend weights, binned into the proposal's 64 bins, mark
the bins that hold at least half of a ray's maximum weight (the surface bins).

Checks, on the GPU path end to end:
  * after training, the proposal pdf puts most of its mass on the surface bins,
    several times what the uniform pdf (the method without a proposal) puts there;
  * the drawn importance samples land in the surface bins at that rate;
  * the sum of binned blend weights seen by the proposal's samples approaches
    the dense reference's, far closer than the same number of uniform samples.
"""
import numpy as np
import pytest
import torch

from synth import MLPSpec, mlp_init

pytestmark = pytest.mark.gpu

S_SHARP = 300.0       # 1/m: surface transition ~1.2 cm wide (logistic FWHM 3.5/s)


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _trainer(dev, train):
    from paper_2605_29097_amd import rfvr as R
    from paper_2605_29097_amd.train import ProposalConfig, ProposalTrainer, StepConfig
    R.lib()
    cfg = StepConfig(cube_centre=(0.0, 0.0, 0.28), s=S_SHARP, seed=0)
    spec = MLPSpec(centre=cfg.cube_centre, half_size=cfg.cube_side / 2)
    params = torch.from_numpy(mlp_init(spec, 0))
    target = torch.zeros(cfg.n_meas, cfg.n_freq, 2)
    tr = ProposalTrainer(cfg, params, target, ProposalConfig(train=train, lr=5e-3), device=dev)
    tr.train_sdf = False
    return R, tr


def _reference_bins(R, tr):
    """Dense blend weights of the reference grid, binned: [n_ray, n_bins]."""
    c = tr.cfg
    xyz, u, origin = R.sample_points(c.cube_centre, c.cube_side / 2, (0, 0, 1), c.lines[0], c.lines[1],
                                     c.n_z, mode=R.SAMPLE_GRID, device=tr.dev)
    f, g, a = R.mlp_forward(tr.net, xyz)
    fl = R.Fields(sdf=f.view(u.shape), grad=g.view(*u.shape, 3), refl=a.view(u.shape), s=c.s, amp=1.0)
    _, alpha, trans = R.render_forward(tr.ap, R.Samples(xyz=xyz), fl, want_alpha=True)
    w = (alpha * trans).view(u.shape).double().cpu().numpy()
    ub = u.double().cpu().numpy()
    b = np.clip(np.floor((ub - tr.lo) / (tr.hi - tr.lo) * tr.pc.n_bins).astype(int), 0, tr.pc.n_bins - 1)
    W = np.zeros((u.shape[0], tr.pc.n_bins))
    np.add.at(W, (np.repeat(np.arange(u.shape[0]), u.shape[1]), b.ravel()), w.ravel())
    return W


def _pdf(logits):
    z = logits.double().cpu().numpy()
    q = 1.0 / (1.0 + np.exp(-z)) + 1e-3
    return q / q.sum(1, keepdims=True)


def test_trained_proposal_concentrates_samples_on_the_surface(dev):
    _say("proposal gain: 400 proposal-only steps, sphere SDF, s=300/m")
    R, tr = _trainer(dev, train=True)
    _, ctl = _trainer(dev, train=False)
    W = _reference_bins(R, tr)
    hit = W.max(1) > 1e-3                                  # rays that meet the sphere
    hot = (W >= 0.5 * W.max(1, keepdims=True)) & hit[:, None]
    assert hit.sum() > 500
    for _ in range(400):
        tr.step()
    torch.cuda.synchronize()
    logits = tr.logits()
    pdf = _pdf(logits)
    mass_trained = float((pdf * hot).sum(1)[hit].mean())
    mass_uniform = float((_pdf(ctl.logits()) * hot).sum(1)[hit].mean())
    print(f"pdf mass on surface bins: trained {mass_trained:.3f}, uniform {mass_uniform:.3f}; "
          f"proposal BCE {tr.last_proposal_loss.item():.4f}")
    assert mass_trained >= 0.5 and mass_trained >= 4.0 * mass_uniform

    # the drawn samples, and the blend weight they see, for trained and control
    def seen(trainer):
        lg = trainer.logits()
        xyz, u, _ = trainer.proposal_samples(lg)
        n_ray, K = u.shape
        f, g, a = R.mlp_forward(trainer.net, xyz)
        fl = R.Fields(sdf=f.view(n_ray, K), grad=g.view(n_ray, K, 3), refl=a.view(n_ray, K), s=trainer.cfg.s,
                      amp=1.0)
        _, alpha, trans = R.render_forward(trainer.ap, R.Samples(xyz=xyz), fl, want_alpha=True)
        ub = u.double().cpu().numpy()
        b = np.clip(np.floor((ub - trainer.lo) / (trainer.hi - trainer.lo) * 64).astype(int), 0, 63)
        in_hot = np.take_along_axis(hot, b, 1)[hit]
        frac_hot = float(in_hot[:, :].mean())
        # second-order weight sum sum_k T_k^2 alpha_k (the round-trip amplitude
        # factor), vs the dense reference's value on the same rays
        w2 = (trans * trans * alpha).view(n_ray, K).double().cpu().numpy().sum(1)
        return frac_hot, w2

    fh_t, w2_t = seen(tr)
    fh_c, w2_c = seen(ctl)
    c = tr.cfg
    xyz, u, _ = R.sample_points(c.cube_centre, c.cube_side / 2, (0, 0, 1), c.lines[0], c.lines[1], c.n_z,
                                device=dev)
    f, g, a = R.mlp_forward(tr.net, xyz)
    fl = R.Fields(sdf=f.view(u.shape), grad=g.view(*u.shape, 3), refl=a.view(u.shape), s=c.s, amp=1.0)
    _, alpha, trans = R.render_forward(tr.ap, R.Samples(xyz=xyz), fl, want_alpha=True)
    w2_dense = (trans * trans * alpha).view(u.shape).double().cpu().numpy().sum(1)
    e_t = float(np.abs(w2_t - w2_dense)[hit].mean() / w2_dense[hit].mean())
    e_c = float(np.abs(w2_c - w2_dense)[hit].mean() / w2_dense[hit].mean())
    print(f"samples in surface bins: trained {fh_t:.3f}, uniform {fh_c:.3f}; "
          f"round-trip weight error vs dense: trained {e_t:.3f}, uniform {e_c:.3f}")
    assert fh_t >= 0.5 and fh_t >= 3.0 * fh_c
    assert e_t < 0.5 * e_c
