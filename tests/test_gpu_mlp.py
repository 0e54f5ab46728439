"""GPU parity of the SDF network entry points (MFMA FP32) against the float64
torch oracle: f, grad_x f, a, and the parameter gradient of
J = sum g_f f + g_grad . grad_x f + g_a a (second-order path included).
Tolerance: 1e-4 RMS relative error per tensor (the FP32 target)."""
import numpy as np
import pytest
import torch

from oracle import mlp as omlp
from synth import MLPSpec, mlp_init, mlp_layout
from gpu_common import rel_rms

pytestmark = pytest.mark.gpu

PASS = 1 << 20          # points per internal pass of the network calls


def _R():
    from paper_2605_29097_amd import rfvr as R
    R.lib()
    return R


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _net(R, spec, params, dev):
    return R.MLP(params=torch.from_numpy(params.astype(np.float32)).to(dev), n_layers=spec.n_layers,
                 width=spec.width, pe_octaves=spec.pe_octaves, head_width=spec.head_width,
                 head_layers=spec.head_layers, beta=spec.beta, centre=spec.centre,
                 half_size=spec.half_size)


def _params(spec, seed, noise=0.3):
    p = mlp_init(spec, seed).astype(np.float64)
    rng = np.random.default_rng(seed + 1000)
    return (p + noise * rng.normal(size=p.shape) / np.sqrt(spec.width)).astype(np.float32)


def _pts(n, spec, seed):
    rng = np.random.default_rng(seed)
    c = np.array(spec.centre)
    return (c + rng.uniform(-spec.half_size, spec.half_size, (n, 3))).astype(np.float32)


CASES = [
    ("full-8x256-pe6", MLPSpec(), 3001),
    ("small-3x64-pe2", MLPSpec(n_layers=3, width=64, pe_octaves=2, head_width=64, head_layers=1), 517),
    ("mid-4x128-pe4-head3", MLPSpec(n_layers=4, width=128, pe_octaves=4, head_width=64, head_layers=3), 1000),
]


@pytest.mark.parametrize("name,spec,n", CASES, ids=[c[0] for c in CASES])
def test_mlp_forward(dev, name, spec, n):
    _say(f"mlp_forward {name} n={n}")
    R = _R()
    p = _params(spec, 3)
    x = _pts(n, spec, 4)
    net = _net(R, spec, p, dev)
    assert net.param_count() == mlp_layout(spec)["__total__"][0]
    f, g, a = R.mlp_forward(net, torch.from_numpy(x).to(dev))
    fr, gr, ar = omlp.forward(p.astype(np.float64), spec, x.astype(np.float64))
    ef, eg, ea = rel_rms(f.cpu().numpy(), fr), rel_rms(g.cpu().numpy(), gr), rel_rms(a.cpu().numpy(), ar)
    print(f"f {ef:.2e} grad {eg:.2e} a {ea:.2e}")
    assert ef <= 1e-4 and eg <= 1e-4 and ea <= 1e-4


@pytest.mark.parametrize("name,spec,n", CASES, ids=[c[0] for c in CASES])
def test_mlp_backward(dev, name, spec, n):
    _say(f"mlp_backward {name} n={n}")
    R = _R()
    p = _params(spec, 5)
    x = _pts(n, spec, 6)
    rng = np.random.default_rng(7)
    gf = rng.normal(size=n).astype(np.float32)
    gg = rng.normal(size=(n, 3)).astype(np.float32)
    gaa = rng.normal(size=n).astype(np.float32)
    net = _net(R, spec, p, dev)
    t = lambda a: torch.from_numpy(a).to(dev)
    gp = R.mlp_backward(net, t(x), t(gf), t(gg), t(gaa)).cpu().numpy()
    ref = omlp.backward(p.astype(np.float64), spec, x.astype(np.float64), gf, gg, gaa)
    e = rel_rms(gp, ref)
    lay = mlp_layout(spec)
    worst = []
    for k, (off, shp) in lay.items():
        if k.startswith("__"):
            continue
        sz = int(np.prod(shp))
        worst.append((rel_rms(gp[off:off + sz], ref[off:off + sz]), k))
    worst.sort(reverse=True)
    print(f"global {e:.2e}; worst tensors {worst[:4]}")
    assert e <= 1e-4
    assert worst[0][0] <= 1e-3


def test_mlp_backward_partial_inputs_and_accumulate(dev):
    """Missing upstream gradients count as zero; RFVR_ACCUMULATE adds."""
    _say("mlp_backward partial inputs")
    R = _R()
    spec = CASES[1][1]
    p = _params(spec, 8)
    x = _pts(300, spec, 9)
    gg = np.random.default_rng(10).normal(size=(300, 3)).astype(np.float32)
    net = _net(R, spec, p, dev)
    t = lambda a: torch.from_numpy(a).to(dev)
    g1 = R.mlp_backward(net, t(x), None, t(gg), None)
    ref = omlp.backward(p.astype(np.float64), spec, x.astype(np.float64), np.zeros(300), gg, np.zeros(300))
    assert rel_rms(g1.cpu().numpy(), ref) <= 1e-4
    g2 = R.mlp_backward(net, t(x), None, t(gg), None, flags=R.ACCUMULATE, out=g1.clone())
    assert rel_rms(g2.cpu().numpy(), 2 * ref) <= 1e-4


def test_mlp_chunked_large_batch_sampled(dev):
    """More points than one internal pass (2^20): spot-check rows against the oracle."""
    _say("mlp_forward chunked")
    R = _R()
    spec = MLPSpec()
    p = _params(spec, 11)
    n = PASS + 777
    x = _pts(n, spec, 12)
    net = _net(R, spec, p, dev)
    f, g, a = R.mlp_forward(net, torch.from_numpy(x).to(dev))
    idx = np.r_[0:5, PASS - 3:PASS + 3, n - 5:n]
    fr, gr, ar = omlp.forward(p.astype(np.float64), spec, x[idx].astype(np.float64))
    assert rel_rms(f.cpu().numpy()[idx], fr) <= 1e-4
    assert rel_rms(g.cpu().numpy()[idx], gr) <= 1e-4
    assert rel_rms(a.cpu().numpy()[idx], ar) <= 1e-4


@pytest.mark.parametrize("name,spec,n", CASES, ids=[c[0] for c in CASES])
def test_mlp_training_pair(dev, name, spec, n):
    """Training forward = plain forward bit for bit; training backward (layer
    activations read from the reserve) against the oracle and the plain call."""
    _say(f"mlp training pair {name} n={n}")
    R = _R()
    p = _params(spec, 5)
    x = _pts(n, spec, 6)
    rng = np.random.default_rng(7)
    gf = rng.normal(size=n).astype(np.float32)
    gg = rng.normal(size=(n, 3)).astype(np.float32)
    gaa = rng.normal(size=n).astype(np.float32)
    net = _net(R, spec, p, dev)
    t = lambda a: torch.from_numpy(a).to(dev)
    res = R.mlp_reserve(net, n, dev)
    assert res.numel() >= 2 * spec.n_layers * n * spec.width * 4
    f, g, a = R.mlp_forward(net, t(x), reserve=res)
    f0, g0, a0 = R.mlp_forward(net, t(x))
    assert torch.equal(f, f0) and torch.equal(g, g0) and torch.equal(a, a0)
    gp = R.mlp_backward(net, t(x), t(gf), t(gg), t(gaa), reserve=res).cpu().numpy()
    gp0 = R.mlp_backward(net, t(x), t(gf), t(gg), t(gaa)).cpu().numpy()
    ref = omlp.backward(p.astype(np.float64), spec, x.astype(np.float64), gf, gg, gaa)
    e, e0 = rel_rms(gp, ref), rel_rms(gp, gp0)
    print(f"training backward vs oracle {e:.2e}, vs plain backward {e0:.2e}")
    assert e <= 1e-4
    assert e0 <= 1e-5


def test_mlp_backward_chunked_sparse_upstream(dev):
    """More points than one internal pass (2^20) with upstream gradients on a
    few rows only (around the pass boundary and at the tail): the parameter
    gradient then equals the oracle's over those rows alone.  Both the plain
    and the training backward (reserve offsets per pass)."""
    _say("mlp_backward chunked, sparse upstream")
    R = _R()
    spec = MLPSpec()
    p = _params(spec, 13)
    n = PASS + 777
    x = _pts(n, spec, 14)
    idx = np.r_[0:3, PASS - 3:PASS + 3, n - 3:n]
    rng = np.random.default_rng(15)
    gf = np.zeros(n, np.float32)
    gg = np.zeros((n, 3), np.float32)
    gaa = np.zeros(n, np.float32)
    gf[idx] = rng.normal(size=idx.size)
    gg[idx] = rng.normal(size=(idx.size, 3))
    gaa[idx] = rng.normal(size=idx.size)
    net = _net(R, spec, p, dev)
    t = lambda a: torch.from_numpy(a).to(dev)
    ref = omlp.backward(p.astype(np.float64), spec, x[idx].astype(np.float64), gf[idx].astype(np.float64),
                        gg[idx].astype(np.float64), gaa[idx].astype(np.float64))
    gp0 = R.mlp_backward(net, t(x), t(gf), t(gg), t(gaa)).cpu().numpy()
    res = R.mlp_reserve(net, n, dev)
    R.mlp_forward(net, t(x), reserve=res)
    gp = R.mlp_backward(net, t(x), t(gf), t(gg), t(gaa), reserve=res).cpu().numpy()
    del res
    e0, e = rel_rms(gp0, ref), rel_rms(gp, ref)
    print(f"plain {e0:.2e}, training pair {e:.2e}")
    assert e0 <= 1e-4 and e <= 1e-4


def test_mlp_training_backward_is_bitwise_reproducible(dev):
    """The training backward runs its weight-gradient products on a second
    stream beside the adjoint chain: the gradient is the same bit for bit over
    repeated calls, and equals the plain backward's to rounding (2^20 + 777
    points, two passes)."""
    _say("mlp training backward determinism")
    R = _R()
    spec = MLPSpec()
    p = _params(spec, 21)
    n = PASS + 777
    x = _pts(n, spec, 22)
    rng = np.random.default_rng(23)
    t = lambda a: torch.from_numpy(a.astype(np.float32)).to(dev)
    gf, gg, gaa = t(rng.normal(size=n)), t(rng.normal(size=(n, 3))), t(rng.normal(size=n))
    net = _net(R, spec, p, dev)
    res = R.mlp_reserve(net, n, dev)
    R.mlp_forward(net, t(x), reserve=res)
    runs = [R.mlp_backward(net, t(x), gf, gg, gaa, reserve=res) for _ in range(3)]
    torch.cuda.synchronize()
    assert all(torch.equal(runs[0], r) for r in runs[1:])
    gp0 = R.mlp_backward(net, t(x), gf, gg, gaa)
    e = rel_rms(runs[0].cpu().numpy(), gp0.cpu().numpy())
    print(f"training vs plain backward {e:.2e}")
    assert e <= 1e-5
