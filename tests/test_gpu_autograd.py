"""Gradients of the full FP32 GPU pipeline (network -> render -> matched filter
-> loss) through the autograd wrappers, checked against central finite
differences of the same GPU forward with eps = 1e-3 (directional, relative to
the perturbed quantity's scale), and against the FP64 oracle gradient."""
import numpy as np
import pytest
import torch

from gpu_common import rel_rms
from oracle import mlp as omlp
from oracle import render as orc
from synth import MLPSpec, freq_grid, line_points, mlp_init, planar_aperture

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _setup(dev, seed=0):
    from paper_2605_29097_amd import rfvr as R
    R.lib()
    spec = MLPSpec(n_layers=4, width=64, pe_octaves=3, head_width=64, head_layers=2,
                   centre=(0.0, 0.0, 0.30), half_size=0.05)
    rng = np.random.default_rng(seed)
    p = mlp_init(spec, seed).astype(np.float64)
    p = (p + 0.2 * rng.normal(size=p.shape) / 8.0).astype(np.float32)
    f0, df = freq_grid(24)
    tx = planar_aperture(5, 4, 2e-3)
    xyz, _ = line_points((0.0, 0.0, 0.30), 0.10, 6, 5, 24, jitter_seed=seed)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    net = R.MLP(params=t(p), n_layers=4, width=64, pe_octaves=3, head_width=64, head_layers=2,
                centre=spec.centre, half_size=spec.half_size)
    ap = R.Aperture(tx=t(tx), f0=f0, df=df, n_freq=24)
    return R, spec, p, net, ap, t(xyz), tx, xyz, f0, df


def _loss(R, A, net, ap, xyz, params, amp, s, p_star):
    f, g, a = A.MLPFn.apply(params, xyz.view(-1, 3), net)
    shp = xyz.shape[:2]
    sig = A.RenderFn.apply(f.view(shp), g.view(*shp, 3), a.view(shp), amp, s, ap, xyz)
    z, p = A.MFFn.apply(sig, ap, xyz.view(-1, 3))
    return A.LossFn.apply(p, p_star)


def _field_loss(R, A, ap, xyz, sdf, grad, refl, amp, s, p_star):
    sig = A.RenderFn.apply(sdf, grad, refl, amp, s, ap, xyz)
    z, p = A.MFFn.apply(sig, ap, xyz.view(-1, 3))
    return A.LossFn.apply(p, p_star)


def _fd_ok(fd, an, L, eps, rtol):
    # FP32 forward: allow a rounding floor of ~1e-6 |L| in the loss difference
    return abs(fd - an) <= rtol * abs(an) + 1e-6 * abs(L) / (2 * eps)


def test_pipeline_gradient_finite_differences(dev):
    """Central differences with eps = 1e-3 along random unit directions, in the
    network parameters and in each per-point field entering the render (sdf,
    grad, refl); relative eps = 1e-3 for A' and s."""
    _say("autograd pipeline vs finite differences (eps=1e-3)")
    from paper_2605_29097_amd import autograd as A
    R, spec, p_np, net, ap, xyz, *_ = _setup(dev)
    params = torch.from_numpy(p_np).to(dev).requires_grad_()
    amp = torch.tensor([1.3], device=dev, requires_grad=True)
    s = torch.tensor([64.0], device=dev, requires_grad=True)
    p_star = torch.rand(xyz.shape[0] * xyz.shape[1], device=dev, generator=torch.Generator(dev).manual_seed(1)) * 50
    L = _loss(R, A, net, ap, xyz, params, amp, s, p_star)
    L.backward()
    Lv = L.item()
    gp, ga, gs = params.grad.clone(), amp.grad.clone(), s.grad.clone()
    gen = torch.Generator(dev).manual_seed(2)
    eps = 1e-3
    for k in range(3):
        d = torch.randn(params.shape, device=dev, generator=gen)
        d = d / d.norm()
        with torch.no_grad():
            Lp = _loss(R, A, net, ap, xyz, params + eps * d, amp, s, p_star)
            Lm = _loss(R, A, net, ap, xyz, params - eps * d, amp, s, p_star)
        fd = (Lp - Lm).item() / (2 * eps)
        an = (gp * d).sum().item()
        print(f"params dir {k}: fd {fd:.6e} analytic {an:.6e}")
        assert _fd_ok(fd, an, Lv, eps, 2e-2)
    with torch.no_grad():
        e = 1e-3 * amp.item()
        fd = (_loss(R, A, net, ap, xyz, params, amp + e, s, p_star) -
              _loss(R, A, net, ap, xyz, params, amp - e, s, p_star)).item() / (2 * e)
    print(f"amp: fd {fd:.6e} analytic {ga.item():.6e}")
    assert _fd_ok(fd, ga.item(), Lv, e, 1e-2)
    with torch.no_grad():
        e = 1e-3 * s.item()
        fd = (_loss(R, A, net, ap, xyz, params, amp, s + e, p_star) -
              _loss(R, A, net, ap, xyz, params, amp, s - e, p_star)).item() / (2 * e)
    print(f"s: fd {fd:.6e} analytic {gs.item():.6e}")
    assert _fd_ok(fd, gs.item(), Lv, e, 2e-2)
    # per-point fields
    with torch.no_grad():
        f, g, a = R.mlp_forward(net, xyz.view(-1, 3))
    shp = xyz.shape[:2]
    fields = [f.view(shp).clone().requires_grad_(), g.view(*shp, 3).clone().requires_grad_(),
              a.view(shp).clone().requires_grad_()]
    Lf = _field_loss(R, A, ap, xyz, *fields, amp.detach(), s.detach(), p_star)
    Lf.backward()
    # the sdf direction is a smooth random field (a plane wave of 10 cm
    # wavelength over the points): neighbouring samples of a ray move together,
    # as under any change of the network, instead of straddling the kink of the
    # opacity clamp at alpha = 0 independently
    kvec = torch.randn(3, device=dev, generator=gen)
    kvec = 2 * np.pi / 0.10 * kvec / kvec.norm()
    smooth = torch.cos(xyz.view(-1, 3) @ kvec + 0.3).view(shp)
    for name, t in zip(("sdf", "grad", "refl"), fields):
        d = smooth.clone() if name == "sdf" else torch.randn(t.shape, device=dev, generator=gen)
        d = d / d.norm()
        with torch.no_grad():
            args_p = [x.detach() + (eps * d if x is t else 0) for x in fields]
            args_m = [x.detach() - (eps * d if x is t else 0) for x in fields]
            fd = (_field_loss(R, A, ap, xyz, *args_p, amp, s, p_star) -
                  _field_loss(R, A, ap, xyz, *args_m, amp, s, p_star)).item() / (2 * eps)
        an = (t.grad * d).sum().item()
        print(f"{name}: fd {fd:.6e} analytic {an:.6e}")
        assert _fd_ok(fd, an, Lf.item(), eps, 2e-2), name


def test_pipeline_gradient_matches_oracle(dev):
    """Network parameter gradient of the whole pipeline vs the FP64 oracle chain
    (torch float64 network + C render/filter adjoints)."""
    _say("autograd pipeline vs FP64 oracle")
    from paper_2605_29097_amd import autograd as A
    R, spec, p_np, net, ap, xyz_t, tx, xyz, f0, df = _setup(dev, seed=3)
    params = torch.from_numpy(p_np).to(dev).requires_grad_()
    amp = torch.tensor([1.0], device=dev, requires_grad=True)
    s = torch.tensor([64.0], device=dev, requires_grad=True)
    rng = np.random.default_rng(4)
    p_star = (rng.uniform(size=xyz.shape[0] * xyz.shape[1]) * 50).astype(np.float32)
    L = _loss(R, A, net, ap, xyz_t, params, amp, s, torch.from_numpy(p_star).to(dev))
    L.backward()
    # oracle chain in float64
    f, g, a = omlp.forward(p_np.astype(np.float64), spec, xyz.reshape(-1, 3).astype(np.float64))
    shp = xyz.shape[:2]
    F = orc.Fields(sdf=f.reshape(shp), grad=g.reshape(*shp, 3), refl=a.reshape(shp), s=64.0, amp=1.0)
    oap = orc.Aperture(tx=tx.astype(np.float64), f0=f0, df=df, n_freq=24)
    sig = orc.render(oap, xyz.astype(np.float64), F)
    z, P = orc.mf(oap, xyz.reshape(-1, 3).astype(np.float64), sig)
    L_o, gP = orc.loss_l2(P, p_star)
    gsig = orc.mf_adjoint(oap, xyz.reshape(-1, 3).astype(np.float64), z, P, gP)
    gr = orc.render_adjoint(oap, xyz.astype(np.float64), F, gsig)
    g_o = omlp.backward(p_np.astype(np.float64), spec, xyz.reshape(-1, 3).astype(np.float64),
                        gr["sdf"].ravel(), gr["grad"].reshape(-1, 3), gr["refl"].ravel())
    got = params.grad.cpu().numpy()
    cos = float(got @ g_o / (np.linalg.norm(got) * np.linalg.norm(g_o)))
    e = rel_rms(got, g_o)
    print(f"loss gpu {L.item():.6e} oracle {L_o:.6e}; grad rms rel {e:.2e} cosine {cos:.8f}")
    assert abs(L.item() - L_o) / L_o < 1e-4
    assert e < 1e-3 and cos > 0.999999
    assert abs(amp.grad.item() - gr["amp"]) / abs(gr["amp"]) < 1e-3
    assert abs(s.grad.item() - gr["s"]) / abs(gr["s"]) < 1e-3
