"""GPU parity of the render, matched filter, loss, sampler and AdamW entry
points against the FP64 oracle, through the C ABI.

Tolerances: signals and heatmaps within 1e-4 RMS relative error (the FP32
path's target); gradients within 1e-4 RMS relative error per tensor, except
where stated; integer-valued decisions (sample strata) exact."""
import numpy as np
import pytest
import torch

from oracle import render as orc
from oracle import sampling as osmp
from oracle import optim as oopt
from gpu_common import (as_complex, full_box_case, max_rel, ragged_case, rel_rms,
                        small_sphere_case)

pytestmark = pytest.mark.gpu

SPEC = {"clamp": 0, "raw": 1, "off": 2}


def _R():
    from paper_2605_29097_amd import rfvr as R
    R.lib()
    return R


def _say(msg):
    print(f"[case] {msg}", flush=True)


# ------------------------------------------------------------------ forward

@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_render_forward_small_sphere(dev, seed):
    _say(f"render_forward small sphere seed={seed}")
    R = _R()
    c = small_sphere_case(seed)
    ap, sm, fl = c.g(dev)
    sig, alpha, trans = R.render_forward(ap, sm, fl, want_alpha=True)
    torch.cuda.synchronize()
    ref, a_ref, t_ref = orc.render(c.o_ap(), c.xyz, c.o_fields(), spec="clamp", return_parts=True)
    got = as_complex(sig)
    e = rel_rms(got, ref)
    print(f"rms rel {e:.3e} max rel {max_rel(got, ref):.3e}")
    assert e <= 1e-4
    assert np.abs(alpha.cpu().numpy() - a_ref).max() < 2e-6
    assert np.abs(trans.cpu().numpy() - t_ref).max() < 2e-6


@pytest.mark.parametrize("spec", ["clamp", "raw", "off"])
def test_render_forward_ragged(dev, spec):
    _say(f"render_forward ragged spec={spec}")
    R = _R()
    c = ragged_case()
    ap, sm, fl = c.g(dev)
    sig = R.render_forward(ap, sm, fl, flags=SPEC[spec])
    ref = orc.render(c.o_ap(), c.xyz, c.o_fields(), spec=spec, ray_w=c.ray_w)
    e = rel_rms(as_complex(sig), ref)
    print(f"rms rel {e:.3e}")
    assert e <= 1e-4


def test_render_forward_is_bitwise_reproducible(dev):
    _say("render_forward determinism")
    R = _R()
    c = ragged_case(seed=3)
    ap, sm, fl = c.g(dev)
    a = R.render_forward(ap, sm, fl)
    b = R.render_forward(ap, sm, fl)
    assert torch.equal(a, b)


def test_render_forward_full_size_sampled_measurements(dev):
    """2^20 points x 1024 measurements x 128 frequencies, in the benchmark's
    launch configuration; the oracle sums all points for 3 measurements."""
    _say("render_forward full size")
    R = _R()
    c = full_box_case()
    ap, sm, fl = c.g(dev)
    sig = as_complex(R.render_forward(ap, sm, fl))
    sel = np.array([0, 517, 1023])
    ref = orc.render(c.o_ap(sel), c.xyz, c.o_fields(sel=sel))
    e = rel_rms(sig[sel], ref)
    print(f"rms rel {e:.3e}")
    assert e <= 1e-4


# ------------------------------------------------------------------ matched filter

def test_mf_forward_two_signals(dev):
    _say("mf_forward two signals")
    R = _R()
    c = small_sphere_case(2)
    rng = np.random.default_rng(4)
    s1 = orc.render(c.o_ap(), c.xyz, c.o_fields())
    s2 = rng.normal(size=s1.shape) + 1j * rng.normal(size=s1.shape)
    ap, sm, fl = c.g(dev)
    t = lambda s: torch.from_numpy(np.stack([s.real, s.imag], -1).astype(np.float32)).to(dev)
    z, p, z2, p2 = R.mf_forward(ap, sm.xyz, t(s1), t(s2))
    # the oracle filters the float32-rounded signals the GPU received
    s1f = s1.astype(np.complex64).astype(np.complex128)
    s2f = s2.astype(np.complex64).astype(np.complex128)
    zr, pr = orc.mf(c.o_ap(), c.xyz.reshape(-1, 3), s1f)
    zr2, pr2 = orc.mf(c.o_ap(), c.xyz.reshape(-1, 3), s2f)
    e1, e2 = rel_rms(as_complex(z), zr), rel_rms(as_complex(z2), zr2)
    print(f"z rms rel {e1:.3e} / {e2:.3e}")
    assert e1 <= 1e-4 and e2 <= 1e-4
    assert rel_rms(p.cpu().numpy(), pr) <= 1e-4 and rel_rms(p2.cpu().numpy(), pr2) <= 1e-4


def test_mf_forward_full_size_sampled_points(dev):
    _say("mf_forward full size")
    R = _R()
    c = full_box_case()
    rng = np.random.default_rng(5)
    s = (rng.normal(size=(1024, 128)) + 1j * rng.normal(size=(1024, 128))).astype(np.complex64)
    ap, sm, fl = c.g(dev)
    st = torch.from_numpy(np.stack([s.real, s.imag], -1)).to(dev)
    z, p = R.mf_forward(ap, sm.xyz, st)
    q = rng.choice(c.xyz.shape[0] * c.xyz.shape[1], 64, replace=False)
    zr, pr = orc.mf(c.o_ap(), c.xyz.reshape(-1, 3)[q], s.astype(np.complex128))
    e = rel_rms(as_complex(z)[q], zr)
    print(f"rms rel {e:.3e}")
    assert e <= 1e-4


def _mf_bwd_pair(dev, c, s, gP, flags=0):
    R = _R()
    ap, sm, fl = c.g(dev)
    st = torch.from_numpy(np.stack([s.real, s.imag], -1).astype(np.float32)).to(dev)
    z, p = R.mf_forward(ap, sm.xyz, st)
    g = R.mf_backward(ap, sm.xyz, z, p, torch.from_numpy(gP.astype(np.float32)).to(dev), flags=flags)
    zr, pr = orc.mf(c.o_ap(), c.xyz.reshape(-1, 3), s.astype(np.complex64).astype(np.complex128))
    gr = orc.mf_adjoint(c.o_ap(), c.xyz.reshape(-1, 3), zr, pr, gP.astype(np.float32).astype(np.float64))
    return as_complex(g), gr


def test_mf_backward_ragged(dev):
    _say("mf_backward ragged")
    c = ragged_case(seed=6)
    rng = np.random.default_rng(6)
    s = rng.normal(size=(c.tx.shape[0], c.n_freq)) + 1j * rng.normal(size=(c.tx.shape[0], c.n_freq))
    gP = rng.normal(size=c.xyz.shape[0] * c.xyz.shape[1])
    g, gr = _mf_bwd_pair(dev, c, s, gP)
    e = rel_rms(g, gr)
    print(f"rms rel {e:.3e}")
    assert e <= 1e-4


def test_mf_backward_full_size_sampled_measurements(dev):
    """Adjoint over 2^20 query points in the benchmark's launch configuration.
    Its inputs (z, P = |z|, g_P) are synthetic and shared; the oracle sums all
    points for two measurements."""
    _say("mf_backward full size")
    R = _R()
    c = full_box_case()
    rng = np.random.default_rng(7)
    nq = c.xyz.shape[0] * c.xyz.shape[1]
    z = (rng.normal(size=nq) + 1j * rng.normal(size=nq)).astype(np.complex64)
    P = np.abs(z).astype(np.float32)
    gP = rng.normal(size=nq).astype(np.float32)
    ap, sm, fl = c.g(dev)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    g = as_complex(R.mf_backward(ap, sm.xyz, t(np.stack([z.real, z.imag], -1)), t(P), t(gP)))
    sel = np.array([3, 700])
    gr = orc.mf_adjoint(c.o_ap(sel), c.xyz.reshape(-1, 3), z.astype(np.complex128), P.astype(np.float64),
                        gP.astype(np.float64))
    e = rel_rms(g[sel], gr)
    print(f"rms rel {e:.3e}")
    assert e <= 1e-4


# ------------------------------------------------------------------ backward

def _render_bwd(dev, c, gs, spec="clamp"):
    R = _R()
    ap, sm, fl = c.g(dev)
    gt = torch.from_numpy(np.stack([gs.real, gs.imag], -1).astype(np.float32)).to(dev)
    out = R.render_backward(ap, sm, fl, gt, flags=SPEC[spec])
    ref = orc.render_adjoint(c.o_ap(), c.xyz, c.o_fields(), gs.astype(np.complex64).astype(np.complex128),
                             spec=spec, ray_w=c.ray_w)
    return {k: v.cpu().numpy() for k, v in out.items()}, ref


@pytest.mark.parametrize("spec", ["clamp", "raw", "off"])
def test_render_backward_ragged(dev, spec):
    _say(f"render_backward ragged spec={spec}")
    c = ragged_case(seed=9)
    rng = np.random.default_rng(9)
    gs = rng.normal(size=(c.tx.shape[0], c.n_freq)) + 1j * rng.normal(size=(c.tx.shape[0], c.n_freq))
    got, ref = _render_bwd(dev, c, gs, spec)
    for k in ("sdf", "grad", "refl"):
        e = rel_rms(got[k], ref[k])
        print(f"{k}: rms rel {e:.3e}")
        assert e <= 1e-4, k
    for k in ("amp", "s"):
        e = abs(got[k][0] - ref[k]) / abs(ref[k])
        print(f"{k}: rel {e:.3e}")
        assert e <= 1e-4, k


def test_render_backward_small_sphere(dev):
    _say("render_backward small sphere")
    c = small_sphere_case(1)
    rng = np.random.default_rng(10)
    gs = rng.normal(size=(64, 32)) + 1j * rng.normal(size=(64, 32))
    got, ref = _render_bwd(dev, c, gs)
    for k in ("sdf", "grad", "refl"):
        e = rel_rms(got[k], ref[k])
        print(f"{k}: rms rel {e:.3e}")
        assert e <= 1e-4, k


def test_render_backward_full_size_sampled_rays(dev):
    """Full 2^20-point adjoint; the oracle recomputes 6 whole rays exactly
    (per-ray quantities depend only on that ray)."""
    _say("render_backward full size")
    R = _R()
    c = full_box_case()
    rng = np.random.default_rng(11)
    gs = (rng.normal(size=(1024, 128)) + 1j * rng.normal(size=(1024, 128))).astype(np.complex64)
    ap, sm, fl = c.g(dev)
    out = R.render_backward(ap, sm, fl, torch.from_numpy(np.stack([gs.real, gs.imag], -1)).to(dev))
    rays = np.array([0, 1000, 2080, 2100, 2111, 4095])       # include rays through the box
    ref = orc.render_adjoint(c.o_ap(), c.xyz[rays], c.o_fields(rays=rays), gs.astype(np.complex128))
    for k in ("sdf", "grad", "refl"):
        e = rel_rms(out[k].cpu().numpy()[rays], ref[k])
        print(f"{k}: rms rel {e:.3e}")
        assert e <= 1e-4, k


def test_end_to_end_gradient_small(dev):
    """render -> MF at the samples -> loss vs a target heatmap -> adjoints."""
    _say("end to end small")
    R = _R()
    c = small_sphere_case(3)
    ap, sm, fl = c.g(dev)
    rng = np.random.default_rng(12)
    Pstar = rng.uniform(0, 1, c.xyz.shape[0] * c.xyz.shape[1]).astype(np.float32) * 3.0
    sig = R.render_forward(ap, sm, fl)
    z, p = R.mf_forward(ap, sm.xyz, sig)
    loss, gP = R.loss_l2(p, torch.from_numpy(Pstar).to(dev))
    gsig = R.mf_backward(ap, sm.xyz, z, p, gP)
    out = R.render_backward(ap, sm, fl, gsig)
    s_o = orc.render(c.o_ap(), c.xyz, c.o_fields())
    z_o, P_o = orc.mf(c.o_ap(), c.xyz.reshape(-1, 3), s_o)
    L_o, gP_o = orc.loss_l2(P_o, Pstar)
    gs_o = orc.mf_adjoint(c.o_ap(), c.xyz.reshape(-1, 3), z_o, P_o, gP_o)
    g_o = orc.render_adjoint(c.o_ap(), c.xyz, c.o_fields(), gs_o)
    assert abs(loss.item() - L_o) / L_o < 1e-4
    assert rel_rms(p.cpu().numpy(), P_o) < 1e-4
    for k in ("sdf", "grad", "refl"):
        e = rel_rms(out[k].cpu().numpy(), g_o[k])
        print(f"{k}: rms rel {e:.3e}")
        assert e <= 2e-4, k


# ------------------------------------------------------------------ small kernels

def test_loss_matches_oracle(dev):
    _say("loss")
    R = _R()
    rng = np.random.default_rng(13)
    n = 100003
    p, ps, m = (rng.uniform(size=n).astype(np.float32), rng.uniform(size=n).astype(np.float32),
                (rng.uniform(size=n) > 0.3).astype(np.float32))
    t = lambda a: torch.from_numpy(a).to(dev)
    loss, g = R.loss_l2(t(p), t(ps), t(m))
    L, gr = orc.loss_l2(p, ps, m)
    assert abs(loss.item() - L) / L < 1e-6
    np.testing.assert_allclose(g.cpu().numpy(), gr, rtol=1e-6, atol=1e-12)


@pytest.mark.parametrize("mode", ["grid", "stratified"])
def test_sample_points_matches_oracle(dev, mode):
    _say(f"sample_points {mode}")
    R = _R()
    w = (0.1, -0.05, 1.0)
    xyz, u, o = R.sample_points((0.01, 0.0, 0.3), 0.1, w, 33, 17, 70,
                                mode=R.SAMPLE_GRID if mode == "grid" else R.SAMPLE_STRATIFIED,
                                seed=123456789012, step=77, device=dev)
    xr, ur, orr = osmp.sample_points(np.float32([0.01, 0.0, 0.3]), np.float32(0.1), np.float32(w),
                                     33, 17, 70, mode, seed=123456789012, step=77)
    np.testing.assert_allclose(u.cpu().numpy(), ur, rtol=0, atol=1e-7)
    np.testing.assert_allclose(xyz.cpu().numpy(), xr, rtol=0, atol=2e-7)
    np.testing.assert_allclose(o.cpu().numpy(), orr, rtol=0, atol=2e-7)
    # the stratum of every sample is an exact integer decision
    h = 0.1
    lo = np.dot(np.float32([0.01, 0.0, 0.3]).astype(np.float64), np.float32(w) / np.linalg.norm(np.float32(w))) - h
    strata = np.floor((u.cpu().numpy().astype(np.float64) - lo) / (2 * h / 70) + 1e-9)
    assert np.array_equal(strata, np.broadcast_to(np.arange(70), strata.shape))


def test_adamw_matches_oracle(dev):
    _say("adamw")
    R = _R()
    rng = np.random.default_rng(14)
    n = 5000
    p, g = rng.normal(size=n).astype(np.float32), rng.normal(size=n).astype(np.float32)
    m, v = (rng.normal(size=n) * 0.1).astype(np.float32), rng.uniform(size=n).astype(np.float32) * 0.01
    t = lambda a: torch.from_numpy(a.copy()).to(dev)
    P, G, M, V = t(p), t(g), t(m), t(v)
    R.adamw(P, G, M, V, 7, 1e-3, wd=0.01)
    # the kernel receives float32 hyper-parameters; give the oracle the same values
    f = lambda x: float(np.float32(x))
    pr, mr, vr = oopt.adamw_step(p, g, m, v, 7, f(1e-3), b1=f(0.9), b2=f(0.999), eps=f(1e-8), wd=f(0.01))
    # float32 arithmetic on O(0.1..3) operands: a few ulp absolute
    np.testing.assert_allclose(P.cpu().numpy(), pr, rtol=1e-6, atol=2e-7)
    np.testing.assert_allclose(M.cpu().numpy(), mr, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(V.cpu().numpy(), vr, rtol=1e-6, atol=1e-9)
