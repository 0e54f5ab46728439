"""Precision study of the network + render + matched-filter chain on the GPU:
network matrix operands {FP32, 16-bit forms with FP32 accumulation} x phase
{FP64 path length and reduction (default), naive FP32 radians}, each against
the FP64 oracle chain on the same inputs.

Network operand precisions: FP32; BF16 (each operand rounded once); BF16x3
(split operands, three BF16 products); F16 (in the forward products FP16
weights rounded once and the per-point operand split in FP16, two products; in
the backward's products BF16 operands).  Reported per combination: RMS
and max relative error of the rendered signal s and of the filter output P,
and the cosine similarity of the network parameter gradient of the heatmap
loss.  Bars: FP32 network + FP64 phase <= 1e-4 on s and P; the 16-bit network
paths that meet it, the split form BF16x3 and F16, + FP64 phase <= 1e-2.
Single-rounded BF16 misses the 1e-2 bar (3.5e-2 measured on this network): its
row is an expected failure held to the 1e-2 bar, so that it is reported and
would show if it ever passed.  The naive-phase rows are reported with a sanity
bound only.

Workload (scaled so the FP64 oracle runs in seconds): 16 x 16 aperture at
2 mm, 64 frequencies 77-81 GHz, 32 x 32 primary rays x 16 depths in a 20 cm
cube at 0.30 m, the 8 x 256 network with its 2 x 64 head (geometric
initialisation plus seeded perturbation), s = 64 /m, clamped specular factor."""
import numpy as np
import pytest
import torch

from gpu_common import max_rel, rel_rms
from oracle import mlp as omlp
from oracle import render as orc
from synth import MLPSpec, freq_grid, line_points, mlp_init, planar_aperture

pytestmark = pytest.mark.gpu

_ORACLE = {}


def _case():
    spec = MLPSpec(centre=(0.0, 0.0, 0.30), half_size=0.10)
    rng = np.random.default_rng(21)
    p = mlp_init(spec, 5).astype(np.float64)
    p = (p + 0.3 * rng.normal(size=p.shape) / np.sqrt(spec.width)).astype(np.float32)
    f0, df = freq_grid(64)
    tx = planar_aperture(16, 16, 2e-3)
    xyz, _ = line_points((0.0, 0.0, 0.30), 0.20, 32, 32, 16, jitter_seed=3)
    p_star = (rng.uniform(size=xyz.shape[0] * xyz.shape[1]) * 10).astype(np.float32)
    return spec, p, f0, df, tx, xyz, p_star


def _oracle():
    if _ORACLE:
        return _ORACLE
    spec, p, f0, df, tx, xyz, p_star = _case()
    x64 = xyz.astype(np.float64)
    f, g, a = omlp.forward(p.astype(np.float64), spec, x64.reshape(-1, 3))
    shp = xyz.shape[:2]
    F = orc.Fields(sdf=f.reshape(shp), grad=g.reshape(*shp, 3), refl=a.reshape(shp), s=64.0, amp=1.0)
    oap = orc.Aperture(tx=tx.astype(np.float64), f0=f0, df=df, n_freq=64)
    sig = orc.render(oap, x64, F)
    z, P = orc.mf(oap, x64.reshape(-1, 3), sig)
    L, gP = orc.loss_l2(P, p_star)
    gsig = orc.mf_adjoint(oap, x64.reshape(-1, 3), z, P, gP)
    gr = orc.render_adjoint(oap, x64, F, gsig)
    gp = omlp.backward(p.astype(np.float64), spec, x64.reshape(-1, 3), gr["sdf"].ravel(),
                       gr["grad"].reshape(-1, 3), gr["refl"].ravel())
    _ORACLE.update(sig=sig, P=P, gp=gp, f=f)
    return _ORACLE


_BF16_MISS = pytest.mark.xfail(strict=True, reason="single-rounded BF16 operands leave ~3.5e-2 signal error on "
                                                 "the 8x256 network, above the 1e-2 bar (split BF16 meets it)")
ROWS = [("fp32", "fp64rr"), ("bf16x3", "fp64rr"), ("f16", "fp64rr"), pytest.param("bf16", "fp64rr", marks=_BF16_MISS),
        ("fp32", "naive32"), ("bf16", "naive32")]


@pytest.mark.parametrize("prec,phase", ROWS, ids=["fp32-fp64rr", "bf16x3-fp64rr", "f16-fp64rr", "bf16-fp64rr",
                                                  "fp32-naive32", "bf16-naive32"])
def test_precision_study(dev, prec, phase):
    print(f"[case] precision study net={prec} phase={phase}", flush=True)
    from paper_2605_29097_amd import autograd as A
    from paper_2605_29097_amd import rfvr as R
    R.lib()
    spec, p, f0, df, tx, xyz, p_star = _case()
    ref = _oracle()
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    net = R.MLP(params=t(p), n_layers=spec.n_layers, width=spec.width, pe_octaves=spec.pe_octaves,
                head_width=spec.head_width, head_layers=spec.head_layers, centre=spec.centre,
                half_size=spec.half_size,
                precision=getattr(R, "PREC_" + prec.upper()))
    flags = R.PHASE_NAIVE32 if phase == "naive32" else 0
    ap = R.Aperture(tx=t(tx), f0=f0, df=df, n_freq=64)
    x = t(xyz)
    params = t(p).requires_grad_()
    amp = torch.tensor([1.0], device=dev, requires_grad=True)
    s = torch.tensor([64.0], device=dev, requires_grad=True)
    f, g, a = A.MLPFn.apply(params, x.view(-1, 3), net)
    shp = xyz.shape[:2]
    sig = A.RenderFn.apply(f.view(shp), g.view(*shp, 3), a.view(shp), amp, s, ap, x, None, None, flags)
    z, P = A.MFFn.apply(sig, ap, x.view(-1, 3), flags)
    L = A.LossFn.apply(P, t(p_star))
    L.backward()
    sg = sig.detach().cpu().numpy().astype(np.float64)
    sg = sg[..., 0] + 1j * sg[..., 1]
    Pg = P.detach().cpu().numpy()
    gp = params.grad.cpu().numpy().astype(np.float64)
    e_f = rel_rms(f.detach().cpu().numpy(), ref["f"])
    e_s, m_s = rel_rms(sg, ref["sig"]), max_rel(sg, ref["sig"])
    e_p, m_p = rel_rms(Pg, ref["P"]), max_rel(Pg, ref["P"])
    cos = float(gp @ ref["gp"] / (np.linalg.norm(gp) * np.linalg.norm(ref["gp"])))
    print(f"[precision] net={prec:5s} phase={phase:8s} sdf rms {e_f:.2e} | signal rms {e_s:.2e} max {m_s:.2e} "
          f"| P rms {e_p:.2e} max {m_p:.2e} | grad cosine {cos:.6f}", flush=True)
    assert np.isfinite(e_s) and np.isfinite(e_p) and np.isfinite(cos)
    if phase == "fp64rr" and prec == "fp32":
        assert e_s <= 1e-4 and e_p <= 1e-4 and cos >= 0.9999
    elif phase == "fp64rr" and prec in ("bf16x3", "f16"):
        assert e_s <= 1e-2 and e_p <= 1e-2 and cos >= 0.999
    elif phase == "fp64rr":
        # single-rounded BF16 operands, held to the BF16 bar (expected to miss
        # it: both operands' 8-bit rounding leaves ~3.5e-2 on this network, and
        # a float64 emulation of the rounding reproduces that)
        assert e_s <= 1e-2 and e_p <= 1e-2
    else:
        # naive FP32 radians: reported, sanity bound only
        assert e_s <= 1e-1 and e_p <= 1e-1 and cos >= 0.99


# ---------------------------------------------------------------- seeds 0-4

_SEEDS = {}


def _seed_case(seed):
    """The scaled workload with the network's initialisation, its perturbation
    and the points' jitter drawn from `seed`; the oracle's signal there."""
    if seed not in _SEEDS:
        spec = MLPSpec(centre=(0.0, 0.0, 0.30), half_size=0.10)
        rng = np.random.default_rng(1000 + seed)
        p = mlp_init(spec, seed).astype(np.float64)
        p = (p + 0.3 * rng.normal(size=p.shape) / np.sqrt(spec.width)).astype(np.float32)
        f0, df = freq_grid(64)
        tx = planar_aperture(16, 16, 2e-3)
        xyz, _ = line_points((0.0, 0.0, 0.30), 0.20, 32, 32, 16, jitter_seed=seed)
        x64 = xyz.astype(np.float64)
        f, g, a = omlp.forward(p.astype(np.float64), spec, x64.reshape(-1, 3))
        shp = xyz.shape[:2]
        F = orc.Fields(sdf=f.reshape(shp), grad=g.reshape(*shp, 3), refl=a.reshape(shp), s=64.0, amp=1.0)
        sig = orc.render(orc.Aperture(tx=tx.astype(np.float64), f0=f0, df=df, n_freq=64), x64, F)
        _SEEDS[seed] = (spec, p, f0, df, tx, xyz, sig)
    return _SEEDS[seed]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "f16"])
def test_precision_over_seeds(dev, prec):
    """The rendered signal's error against the FP64 oracle over seeds 0-4 (the
    network's initialisation and perturbation, the points' jitter), FP64 phase
    reduction: every seed within the bar of its path (1e-4 FP32, 1e-2 for the
    16-bit forms); mean and largest error reported."""
    print(f"[case] precision over seeds 0-4, net={prec}", flush=True)
    from paper_2605_29097_amd import rfvr as R
    R.lib()
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    errs = []
    for seed in range(5):
        spec, p, f0, df, tx, xyz, ref = _seed_case(seed)
        net = R.MLP(params=t(p), n_layers=spec.n_layers, width=spec.width, pe_octaves=spec.pe_octaves,
                    head_width=spec.head_width, head_layers=spec.head_layers, centre=spec.centre,
                    half_size=spec.half_size, precision=getattr(R, "PREC_" + prec.upper()))
        x = t(xyz)
        f, g, a = R.mlp_forward(net, x.view(-1, 3))
        shp = xyz.shape[:2]
        fl = R.Fields(sdf=f.view(shp), grad=g.view(*shp, 3), refl=a.view(shp), s=64.0, amp=1.0)
        sig = R.render_forward(R.Aperture(tx=t(tx), f0=f0, df=df, n_freq=64), R.Samples(xyz=x), fl)
        sg = sig.cpu().numpy().astype(np.float64)
        errs.append(rel_rms(sg[..., 0] + 1j * sg[..., 1], ref))
    errs = np.array(errs)
    print(f"[precision seeds] net={prec:6s} signal rms per seed {', '.join(f'{e:.2e}' for e in errs)} | "
          f"mean {errs.mean():.2e} max {errs.max():.2e}", flush=True)
    assert np.isfinite(errs).all()
    assert errs.max() <= (1e-4 if prec == "fp32" else 1e-2)


# ---------------------------------------------------------------- full shape

_FULL = {}
FULL_SEL = np.array([0, 527, 1023])                    # two corners and a centre antenna


def _full_case():
    """The 2^20-point workload's shape: 32 x 32 aperture at 2 mm, 128
    frequencies, 64 x 64 primary rays x 256 depths in a 20 cm cube at 0.30 m,
    the 8 x 256 network with its 2 x 64 head (geometric initialisation plus a
    seeded perturbation), s = 64 /m."""
    spec = MLPSpec(centre=(0.0, 0.0, 0.30), half_size=0.10)
    rng = np.random.default_rng(31)
    p = mlp_init(spec, 7).astype(np.float64)
    p = (p + 0.3 * rng.normal(size=p.shape) / np.sqrt(spec.width)).astype(np.float32)
    f0, df = freq_grid(128)
    tx = planar_aperture(32, 32, 2e-3)
    xyz, _ = line_points((0.0, 0.0, 0.30), 0.20, 64, 64, 256)
    rows = np.concatenate([np.arange(r * 256, (r + 1) * 256) for r in (0, 2080, 2111, 4095)])
    return spec, p, f0, df, tx, xyz, rows


def _full_oracle():
    """FP64 network at every point (in chunks), the signal at FULL_SEL over all
    points (a sum over rays, so over disjoint ray chunks in threads), and the
    network's parameter gradient for seeded upstream gradients on four whole
    rays."""
    if _FULL:
        return _FULL
    from concurrent.futures import ThreadPoolExecutor
    spec, p, f0, df, tx, xyz, rows = _full_case()
    p64 = p.astype(np.float64)
    x64 = xyz.astype(np.float64).reshape(-1, 3)
    parts = [omlp.forward(p64, spec, x64[k:k + 32768]) for k in range(0, x64.shape[0], 32768)]
    f = np.concatenate([q[0] for q in parts])
    g = np.concatenate([q[1] for q in parts])
    a = np.concatenate([q[2] for q in parts])
    shp = xyz.shape[:2]
    F = orc.Fields(sdf=f.reshape(shp), grad=g.reshape(*shp, 3), refl=a.reshape(shp), s=64.0, amp=1.0)
    oap = orc.Aperture(tx=tx[FULL_SEL].astype(np.float64), f0=f0, df=df, n_freq=128)
    chunks = np.array_split(np.arange(shp[0]), 16)
    x3 = xyz.astype(np.float64)

    def part(r):
        Fr = orc.Fields(sdf=F.sdf[r], grad=F.grad[r], refl=F.refl[r], s=64.0, amp=1.0)
        return orc.render(oap, x3[r], Fr)

    with ThreadPoolExecutor(16) as ex:
        sig = sum(ex.map(part, chunks))
    rng = np.random.default_rng(32)
    up = (rng.normal(size=rows.size), rng.normal(size=(rows.size, 3)), rng.normal(size=rows.size))
    up = tuple(u.astype(np.float32) for u in up)
    gp = omlp.backward(p64, spec, x64[rows], *(u.astype(np.float64) for u in up))
    _FULL.update(sig=sig, f=f, g=g, up=up, gp=gp)
    return _FULL


FULL_ROWS = [("fp32", "fp64rr"), ("bf16x3", "fp64rr"), ("f16", "fp64rr"),
             pytest.param("bf16", "fp64rr", marks=_BF16_MISS), ("fp32", "naive32")]


@pytest.mark.timeout(600)     # the first case also runs the FP64 network at 2^20 points on the host
@pytest.mark.parametrize("prec,phase", FULL_ROWS, ids=["fp32-fp64rr", "bf16x3-fp64rr", "f16-fp64rr",
                                                       "bf16-fp64rr", "fp32-naive32"])
def test_precision_study_full_shape(dev, prec, phase):
    """The precision study at the 2^20-point workload's shape, in the launch
    configuration of the benchmark: the GPU network at all 2^20 points and the
    render over all of them, against the oracle at three measurements (every
    frequency); the network backward over all points with upstream gradients on
    four whole rays, against the oracle's on those rays."""
    print(f"[case] precision study at full shape net={prec} phase={phase}", flush=True)
    from paper_2605_29097_amd import rfvr as R
    R.lib()
    spec, p, f0, df, tx, xyz, rows = _full_case()
    ref = _full_oracle()
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    net = R.MLP(params=t(p), n_layers=spec.n_layers, width=spec.width, pe_octaves=spec.pe_octaves,
                head_width=spec.head_width, head_layers=spec.head_layers, centre=spec.centre,
                half_size=spec.half_size,
                precision=getattr(R, "PREC_" + prec.upper()))
    flags = R.PHASE_NAIVE32 if phase == "naive32" else 0
    x = t(xyz)
    f, g, a = R.mlp_forward(net, x.view(-1, 3))
    shp = xyz.shape[:2]
    ap = R.Aperture(tx=t(tx), f0=f0, df=df, n_freq=128)
    fl = R.Fields(sdf=f.view(shp), grad=g.view(*shp, 3), refl=a.view(shp), s=64.0, amp=1.0)
    sig = R.render_forward(ap, R.Samples(xyz=x), fl, flags=flags)
    n = shp[0] * shp[1]
    up = ref["up"]
    g_f, g_g, g_a = (torch.zeros(n, device=dev), torch.zeros(n, 3, device=dev), torch.zeros(n, device=dev))
    idx = t(rows.astype(np.int64))
    g_f[idx], g_g[idx], g_a[idx] = t(up[0]), t(up[1]), t(up[2])
    gp = R.mlp_backward(net, x.view(-1, 3), g_f, g_g, g_a).cpu().numpy().astype(np.float64)
    sg = sig.cpu().numpy().astype(np.float64)
    sg = (sg[..., 0] + 1j * sg[..., 1])[FULL_SEL]
    e_f = rel_rms(f.cpu().numpy(), ref["f"])
    e_s, m_s = rel_rms(sg, ref["sig"]), max_rel(sg, ref["sig"])
    e_gp = rel_rms(gp, ref["gp"])
    cos = float(gp @ ref["gp"] / (np.linalg.norm(gp) * np.linalg.norm(ref["gp"])))
    print(f"[precision full] net={prec:6s} phase={phase:8s} sdf rms {e_f:.2e} | signal rms {e_s:.2e} "
          f"max {m_s:.2e} | network gradient rms {e_gp:.2e} cosine {cos:.7f}", flush=True)
    assert np.isfinite(e_s) and np.isfinite(cos)
    if phase == "fp64rr" and prec == "fp32":
        assert e_s <= 1e-4 and e_gp <= 1e-3
    elif phase == "fp64rr":
        assert e_s <= 1e-2 and cos >= 0.999
    else:
        assert e_s <= 1e-1
