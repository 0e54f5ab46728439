"""GPU parity of the proposal sampler entry points against the float64 oracle:
network logits and parameter gradient (1e-4 RMS relative, the FP32 target),
importance depths (FP64 CDF and inversion on both sides, so the bins agree and
the depths match to float32 rounding), binned targets (bin decisions in FP64
on both sides: bin-exact) and the BCE loss."""
import numpy as np
import pytest
import torch

from oracle import proposal as op
from oracle.sampling import sample_points as o_sample_points
from synth import ProposalSpec, proposal_init, proposal_layout
from gpu_common import rel_rms

pytestmark = pytest.mark.gpu


def _R():
    from paper_2605_29097_amd import rfvr as R
    R.lib()
    return R


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _net(R, spec, p, dev):
    return R.Proposal(params=_t(p.astype(np.float32), dev), pe_octaves=spec.pe_octaves, width=spec.width,
                      layers=spec.layers, centre=spec.centre, half_size=spec.half_size)


def _params(spec, seed):
    p = proposal_init(spec, seed).astype(np.float64)
    p += 0.1 * np.random.default_rng(seed + 7).normal(size=p.shape)     # non-zero biases too
    return p.astype(np.float32)


NETS = [
    ("L4-2x64", ProposalSpec(), 70001),
    ("L2-1x64", ProposalSpec(pe_octaves=2, layers=1), 999),
    ("L5-4x64", ProposalSpec(pe_octaves=5, layers=4), 4097),
]


@pytest.mark.parametrize("name,spec,n", NETS, ids=[c[0] for c in NETS])
def test_proposal_network_forward_backward(dev, name, spec, n):
    _say(f"proposal network {name} n={n}")
    R = _R()
    p = _params(spec, 3)
    rng = np.random.default_rng(5)
    x = (np.array(spec.centre) + rng.uniform(-1.2, 1.2, (n, 3)) * spec.half_size).astype(np.float32)
    net = _net(R, spec, p, dev)
    assert net.param_count() == proposal_layout(spec)["__total__"][0]
    z = R.proposal_forward(net, _t(x, dev)).cpu().numpy()
    zo = op.forward(p.astype(np.float64), spec, x.astype(np.float64))
    e = rel_rms(z, zo)
    print(f"logits rel rms {e:.2e}")
    assert e < 1e-4
    g = rng.normal(size=n).astype(np.float32)
    gp = R.proposal_backward(net, _t(x, dev), _t(g, dev)).cpu().numpy()
    go = op.backward(p.astype(np.float64), spec, x.astype(np.float64), g.astype(np.float64))
    lay = proposal_layout(spec)
    for k, (o, shp) in lay.items():
        if k.startswith("__"):
            continue
        sl = slice(o, o + int(np.prod(shp)))
        ek = rel_rms(gp[sl], go[sl])
        print(f"  d{k} rel rms {ek:.2e}")
        assert ek < 1e-4, k
    # accumulate into an existing gradient
    base = torch.ones(len(gp), device=dev)
    R.proposal_backward(net, _t(x, dev), _t(g, dev), flags=R.ACCUMULATE, out=base)
    assert rel_rms(base.cpu().numpy() - 1.0, go) < 1e-4


SAMPLE_CASES = [
    # (rays x, rays y, n_bins, n_imp, n_uni, direction)
    (7, 5, 64, 16, 4, (0.0, 0.0, 1.0)),
    (3, 11, 37, 27, 0, (0.1, -0.2, 1.0)),
    (4, 4, 1, 0, 9, (0.0, 0.0, 1.0)),
    (9, 2, 64, 60, 4, (0.0, 1.0, 0.05)),
    # more slots than lanes: several slots per lane, ragged last register
    (5, 3, 64, 192, 64, (0.0, 0.0, 1.0)),
    (3, 2, 17, 700, 1, (0.2, 0.1, 1.0)),
    (2, 2, 64, 1000, 24, (0.0, 0.0, 1.0)),        # RFVR_MAX_RAY_SAMPLES exactly
    (2, 3, 16, 0, 130, (0.0, 0.0, 1.0)),          # uniform slots only, three registers
    (2, 2, 64, 200, 0, (0.3, 0.0, 1.0)),          # importance slots only, four registers
]


@pytest.mark.parametrize("jitter", [True, False], ids=["drawn", "fixed"])
@pytest.mark.parametrize("case", SAMPLE_CASES, ids=[f"{c[0]}x{c[1]}-b{c[2]}-i{c[3]}-u{c[4]}" for c in SAMPLE_CASES])
def test_sample_importance(dev, case, jitter):
    nx, ny, n_bins, n_imp, n_uni, wdir = case
    _say(f"sample_importance {case} jitter={jitter}")
    R = _R()
    rng = np.random.default_rng(n_bins + n_imp)
    n_ray = nx * ny
    z = rng.normal(0, 4, (n_ray, n_bins)).astype(np.float32)
    z[0] = -50.0                                 # nothing: pdf is the floor, uniform
    if n_ray > 1:
        z[1] = -50.0
        z[1, n_bins // 2] = 50.0                 # one hot bin
    centre, h, seed, step = (0.01, 0.0, 0.28), 0.1, 12345, 6
    xyz, u, o = R.sample_importance(centre, h, wdir, nx, ny, _t(z, dev), n_imp, n_uni, seed=seed, step=step,
                                    jitter=jitter)
    # oracle: ray origins and range from the grid sampler, depths from the proposal
    _, _, o_ref = o_sample_points(centre, h, wdir, nx, ny, 1)
    w = np.asarray(wdir, np.float64)
    w /= np.linalg.norm(w)
    cw = float(np.dot(np.asarray(centre, np.float64), w))
    lo, hi = cw - h, cw + h
    u_ref, _ = op.importance_depths(z.astype(np.float64), lo, hi, n_imp, n_uni, seed, step, jitter=jitter)
    x_ref = o_ref[:, None, :] + u_ref[..., None] * w
    ug = u.cpu().numpy().astype(np.float64)
    err_u = np.abs(ug - u_ref).max()
    err_x = np.abs(xyz.cpu().numpy() - x_ref).max()
    print(f"max |du| {err_u:.2e} m, max |dx| {err_x:.2e} m")
    assert err_u <= 4e-8 and err_x <= 4e-8          # float32 rounding of values below 0.5 m
    np.testing.assert_allclose(o.cpu().numpy(), o_ref, rtol=0, atol=4e-8)
    assert np.all(np.diff(ug, axis=1) >= 0)


def test_sample_importance_full_size(dev):
    """64 x 64 rays, 64 bins, 16 + 4 samples: every ray against the oracle."""
    _say("sample_importance 64x64 b64 i16 u4")
    R = _R()
    rng = np.random.default_rng(0)
    z = rng.normal(-3, 4, (4096, 64)).astype(np.float32)
    xyz, u, o = R.sample_importance((0.0, 0.0, 0.28), 0.1, (0, 0, 1), 64, 64, _t(z, dev), 16, 4, seed=1, step=99)
    u_ref, _ = op.importance_depths(z.astype(np.float64), 0.18, 0.38, 16, 4, 1, 99)
    err = np.abs(u.cpu().numpy() - u_ref).max()
    print(f"max |du| {err:.2e}")
    assert err <= 4e-8


@pytest.mark.parametrize("n_ray,n_k,n_bins,dilate", [(5, 64, 64, 0), (300, 20, 64, 0), (33, 7, 13, 0),
                                                      (40, 256, 64, 0), (6, 1000, 37, 0), (3, 1024, 64, 0),
                                                      (4, 129, 1, 0), (300, 20, 64, 2), (33, 7, 13, 12),
                                                      (40, 256, 64, 63)])
def test_proposal_targets(dev, n_ray, n_k, n_bins, dilate):
    _say(f"proposal_targets n_ray={n_ray} n_k={n_k} n_bins={n_bins} dilate={dilate}")
    R = _R()
    rng = np.random.default_rng(n_ray)
    lo, hi = np.float32(0.18), np.float32(0.38)
    u = np.sort(rng.uniform(lo, hi, (n_ray, n_k)), 1).astype(np.float32)
    # depths exactly on bin edges (as float32), and both ends of the range
    edges = (lo.astype(np.float64) + np.arange(n_bins + 1) * (hi - lo) / n_bins).astype(np.float32)
    u[0, : min(n_k, n_bins + 1)] = edges[: min(n_k, n_bins + 1)]
    u[0] = np.sort(u[0])
    # past 64 samples, small alphas keep the transmittance (and with it the
    # weight of every register of samples) away from zero
    alpha = rng.uniform(0, 1.0 if n_k <= 64 else 4.0 / n_k, (n_ray, n_k)).astype(np.float32)
    trans = np.cumprod(1 - alpha, 1).astype(np.float32)
    alpha[min(2, n_ray - 1)] = 1e-6                # floor case
    t = R.proposal_targets(_t(u, dev), _t(alpha, dev), _t(trans, dev), float(lo), float(hi), n_bins, dilate)
    w = trans.astype(np.float32) * alpha.astype(np.float32)          # same float32 product
    W = op.bin_weights(u.astype(np.float64), w.astype(np.float64), float(lo), float(hi), n_bins)
    t_ref = op.targets(W, dilate)
    err = np.abs(t.cpu().numpy() - t_ref).max()
    print(f"max |dt| {err:.2e}")
    assert err <= 1e-5


@pytest.mark.parametrize("n", [1, 1000, 262144])
def test_bce(dev, n):
    _say(f"bce n={n}")
    R = _R()
    rng = np.random.default_rng(n)
    z = rng.normal(0, 5, n).astype(np.float32)
    t = rng.uniform(size=n).astype(np.float32)
    loss, g = R.bce(_t(z, dev), _t(t, dev))
    L, g_ref = op.bce(z.astype(np.float64), t.astype(np.float64))
    print(f"bce {loss.item():.8e} vs {L:.8e}")
    assert abs(loss.item() - L) <= 1e-5 * abs(L)
    assert rel_rms(g.cpu().numpy(), g_ref) < 1e-5


def test_proposal_entry_points_reject_bad_arguments(dev):
    R = _R()
    z = torch.zeros(4, 65, device=dev)
    with pytest.raises(R.RfvrError):
        R.sample_importance((0, 0, 0.3), 0.1, (0, 0, 1), 2, 2, z, 8, 2)       # 65 bins
    z = torch.zeros(4, 8, device=dev)
    with pytest.raises(R.RfvrError):
        R.sample_importance((0, 0, 0.3), 0.1, (0, 0, 1), 2, 2, z, 1000, 25)   # 1025 samples
    u = torch.zeros(2, 1025, device=dev)
    with pytest.raises(R.RfvrError):
        R.proposal_targets(u, u, u, 0.2, 0.4, 64)                             # 1025 samples
    u = torch.zeros(2, 16, device=dev)
    with pytest.raises(R.RfvrError):
        R.proposal_targets(u, u, u, 0.2, 0.4, 64, dilate=64)                  # dilation past the bins
    bad = _net(R, ProposalSpec(layers=5), np.zeros(10, np.float32), dev)
    assert bad.param_count() == -1
    with pytest.raises(R.RfvrError):
        R.proposal_forward(bad, torch.zeros(3, 3, device=dev))
