"""The network's FP16 form (RFVR_PREC_F16): in the forward products FP16
weights rounded once and the per-point operand split in two FP16 parts (two
products), in the backward's products BF16 operands (one product), FP32
accumulation.

Against the float64 oracle on the three network shapes: f, grad_x f and a
within the 16-bit bar of 1e-2 RMS relative error per tensor; the parameter
gradient of J = sum g_f f + g_grad . grad_x f + g_a a with cosine >= 0.999 and
RMS relative error <= 3e-2, from both the plain backward (which recomputes the
forward products in FP16) and the training pair.  The training forward equals
the plain forward bit for bit.  At the 2^20-point workload's shape the
signal bar itself is checked by the precision study."""
import numpy as np
import pytest
import torch

from oracle import mlp as omlp
from gpu_common import rel_rms
from test_gpu_mlp import CASES, _params, _pts

pytestmark = pytest.mark.gpu


def _cos(a, b):
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))


@pytest.mark.parametrize("name,spec,n", CASES, ids=[c[0] for c in CASES])
def test_mlp_f16_against_oracle(dev, name, spec, n):
    print(f"[case] mlp F16 {name} n={n}", flush=True)
    from paper_2605_29097_amd import rfvr as R
    R.lib()
    p = _params(spec, 11)
    x = _pts(n, spec, 12)
    rng = np.random.default_rng(13)
    gf = rng.normal(size=n).astype(np.float32)
    gg = rng.normal(size=(n, 3)).astype(np.float32)
    gaa = rng.normal(size=n).astype(np.float32)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    net = R.MLP(params=t(p), n_layers=spec.n_layers, width=spec.width, pe_octaves=spec.pe_octaves,
                head_width=spec.head_width, head_layers=spec.head_layers, beta=spec.beta,
                centre=spec.centre, half_size=spec.half_size, precision=R.PREC_F16)
    f, g, a = R.mlp_forward(net, t(x))
    fr, gr, ar = omlp.forward(p.astype(np.float64), spec, x.astype(np.float64))
    ef, eg, ea = (rel_rms(f.cpu().numpy(), fr), rel_rms(g.cpu().numpy(), gr), rel_rms(a.cpu().numpy(), ar))
    res = R.mlp_reserve(net, n, dev)
    f1, g1, a1 = R.mlp_forward(net, t(x), reserve=res)
    assert torch.equal(f, f1) and torch.equal(g, g1) and torch.equal(a, a1)
    gp_plain = R.mlp_backward(net, t(x), t(gf), t(gg), t(gaa)).cpu().numpy().astype(np.float64)
    gp_train = R.mlp_backward(net, t(x), t(gf), t(gg), t(gaa), reserve=res).cpu().numpy().astype(np.float64)
    ref = omlp.backward(p.astype(np.float64), spec, x.astype(np.float64), gf, gg, gaa)
    ep, et = rel_rms(gp_plain, ref), rel_rms(gp_train, ref)
    cp, ct = _cos(gp_plain, ref), _cos(gp_train, ref)
    print(f"[f16] {name}: f {ef:.2e} grad {eg:.2e} a {ea:.2e} | parameter gradient plain {ep:.2e} "
          f"(cos {cp:.6f}), training pair {et:.2e} (cos {ct:.6f})", flush=True)
    assert ef <= 1e-2 and eg <= 1e-2 and ea <= 1e-2
    assert np.isfinite(gp_plain).all() and np.isfinite(gp_train).all()
    assert ep <= 3e-2 and et <= 3e-2 and cp >= 0.999 and ct >= 0.999


@pytest.mark.parametrize("prec,layers", [("f16", 8), ("bf16", 8), ("f16", 1)], ids=["f16", "bf16", "f16-one-layer"])
def test_training_backward_bf16_storage(dev, prec, layers):
    """With single-rounded BF16 backward products (the F16 and BF16 forms) the
    training backward keeps its tangents and adjoints in BF16 storage; the
    plain backward keeps them in FP32.  Both round every such operand to BF16
    before its product, so the two gradients agree to the BF16 rounding of the
    few FP32 consumers (the tangent's use in the adjoint epilogue, the
    encoding layer's weight gradient): RMS relative difference <= 2e-2,
    cosine >= 0.999, on the 8 x 256 network (and a one-layer trunk, whose top
    layer reads the encoding) at 2^20 + 777 points (two passes)."""
    from test_gpu_mlp import PASS
    print(f"[case] training backward with BF16 storage, {prec}, {layers} layers", flush=True)
    import dataclasses
    from paper_2605_29097_amd import rfvr as R
    R.lib()
    spec = dataclasses.replace(CASES[0][1], n_layers=layers)
    n = PASS + 777
    p = _params(spec, 31)
    x = _pts(n, spec, 32)
    rng = np.random.default_rng(33)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    gf, gg, gaa = t(rng.normal(size=n)), t(rng.normal(size=(n, 3))), t(rng.normal(size=n))
    net = R.MLP(params=t(p), n_layers=spec.n_layers, width=spec.width, pe_octaves=spec.pe_octaves,
                head_width=spec.head_width, head_layers=spec.head_layers, beta=spec.beta,
                centre=spec.centre, half_size=spec.half_size, precision=getattr(R, "PREC_" + prec.upper()))
    res = R.mlp_reserve(net, n, dev)
    R.mlp_forward(net, t(x), reserve=res)
    g1 = R.mlp_backward(net, t(x), gf, gg, gaa, reserve=res)
    g2 = R.mlp_backward(net, t(x), gf, gg, gaa, reserve=res)
    assert torch.equal(g1, g2)
    del res
    g0 = R.mlp_backward(net, t(x), gf, gg, gaa).cpu().numpy().astype(np.float64)
    g1 = g1.cpu().numpy().astype(np.float64)
    e, c = rel_rms(g1, g0), _cos(g1, g0)
    print(f"[f16] {prec}, {layers} layers: training backward (BF16 storage) vs plain backward {e:.2e}, "
          f"cosine {c:.6f}", flush=True)
    assert np.isfinite(g1).all() and e <= 2e-2 and c >= 0.999
