"""GPU parity of bistatic apertures (a receiver apart from each transmitter)
against the FP64 oracle, through the C ABI: render forward and adjoint, matched
filter forward and adjoint, on the moment kernels (default) and on the
per-frequency kernels (RFVR_TERMS_DIRECT), with the lensless shift of both
antennas' transmittances on; swapping transmitters and receivers; rx = tx
against the monostatic render; the 2^20-point workload with a 1 cm baseline.

Tolerances as for monostatic apertures: 1e-4 RMS relative error per output
tensor (the FP32 path's target)."""
import numpy as np
import pytest
import torch

from oracle import render as orc
from gpu_common import Case, as_complex, full_box_case, ragged_case, rel_rms

pytestmark = pytest.mark.gpu

SPEC = {"clamp": 0, "raw": 1, "off": 2}


def _R():
    from paper_2605_29097_amd import rfvr as R
    R.lib()
    return R


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _bistatic(c: Case, seed: int, baseline=(0.011, -0.006, 0.0005), phi=True) -> Case:
    """The case with receivers `baseline` away from the transmitters (jittered
    by 1 mm) and, when the shift is on, their own origin occupancies."""
    rng = np.random.default_rng(100 + seed)
    c.rx = (c.tx + np.asarray(baseline, np.float32) +
            rng.uniform(-1e-3, 1e-3, c.tx.shape).astype(np.float32)).astype(np.float32)
    if phi and c.phi_tx is not None:
        c.phi_rx = rng.uniform(0.97, 1.0, c.tx.shape[0]).astype(np.float32)
    return c


def _flags(spec, direct):
    R = _R()
    return SPEC[spec] | (R.TERMS_DIRECT if direct else 0)


@pytest.mark.parametrize("direct", [False, True], ids=["moments", "per_freq"])
@pytest.mark.parametrize("spec", ["clamp", "raw", "off"])
def test_bistatic_render_forward_ragged(dev, spec, direct):
    _say(f"bistatic render_forward ragged spec={spec} direct={direct}")
    R = _R()
    c = _bistatic(ragged_case(seed=2), 2)
    ap, sm, fl = c.g(dev)
    K = R.term_order(ap, sm.xyz)
    assert K > 0                                   # the moment kernels serve this geometry
    sig = R.render_forward(ap, sm, fl, flags=_flags(spec, direct))
    ref = orc.render(c.o_ap(), c.xyz, c.o_fields(), spec=spec, ray_w=c.ray_w)
    e = rel_rms(as_complex(sig), ref)
    print(f"K = {K}: rms rel {e:.3e}")
    assert e <= 1e-4


@pytest.mark.parametrize("direct", [False, True], ids=["moments", "per_freq"])
@pytest.mark.parametrize("spec", ["clamp", "raw", "off"])
def test_bistatic_render_backward_ragged(dev, spec, direct):
    _say(f"bistatic render_backward ragged spec={spec} direct={direct}")
    R = _R()
    c = _bistatic(ragged_case(seed=9), 9)
    rng = np.random.default_rng(19)
    gs = rng.normal(size=(c.tx.shape[0], c.n_freq)) + 1j * rng.normal(size=(c.tx.shape[0], c.n_freq))
    ap, sm, fl = c.g(dev)
    gt = torch.from_numpy(np.stack([gs.real, gs.imag], -1).astype(np.float32)).to(dev)
    out = R.render_backward(ap, sm, fl, gt, flags=_flags(spec, direct))
    ref = orc.render_adjoint(c.o_ap(), c.xyz, c.o_fields(), gs.astype(np.complex64).astype(np.complex128),
                             spec=spec, ray_w=c.ray_w)
    for k in ("sdf", "grad", "refl"):
        e = rel_rms(out[k].cpu().numpy(), ref[k])
        print(f"{k}: rms rel {e:.3e}")
        assert e <= 1e-4, k
    for k in ("amp", "s"):
        e = abs(out[k].item() - ref[k]) / abs(ref[k])
        print(f"{k}: rel {e:.3e}")
        assert e <= 1e-4, k


def test_bistatic_render_forward_naive_phase(dev):
    """FP32 radians for the phase (RFVR_PHASE_NAIVE32, which runs the
    per-frequency kernels) on a bistatic aperture: the same sum, within the
    naive phase's own rounding at these ranges."""
    _say("bistatic render_forward naive phase")
    R = _R()
    c = _bistatic(ragged_case(seed=4), 4)
    ap, sm, fl = c.g(dev)
    ref = orc.render(c.o_ap(), c.xyz, c.o_fields(), ray_w=c.ray_w)
    sig = R.render_forward(ap, sm, fl, flags=R.PHASE_NAIVE32)
    e = rel_rms(as_complex(sig), ref)
    print(f"rms rel {e:.3e}")
    assert e <= 1e-3


@pytest.mark.parametrize("direct", [False, True], ids=["moments", "per_freq"])
def test_bistatic_mf_forward_and_backward_ragged(dev, direct):
    _say(f"bistatic mf forward/backward ragged direct={direct}")
    R = _R()
    c = _bistatic(ragged_case(seed=6), 6)
    rng = np.random.default_rng(26)
    s = rng.normal(size=(c.tx.shape[0], c.n_freq)) + 1j * rng.normal(size=(c.tx.shape[0], c.n_freq))
    s32 = s.astype(np.complex64)
    ap, sm, fl = c.g(dev)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    flags = R.TERMS_DIRECT if direct else 0
    z, p = R.mf_forward(ap, sm.xyz, t(np.stack([s32.real, s32.imag], -1)), flags=flags)
    xq = c.xyz.reshape(-1, 3)
    zr, pr = orc.mf(c.o_ap(), xq, s32.astype(np.complex128))
    ez = rel_rms(as_complex(z), zr)
    print(f"z rms rel {ez:.3e}")
    assert ez <= 1e-4
    gP = rng.normal(size=xq.shape[0]).astype(np.float32)
    g = R.mf_backward(ap, sm.xyz, z, p, t(gP), flags=flags)
    gr = orc.mf_adjoint(c.o_ap(), xq, zr, pr, gP.astype(np.float64))
    eg = rel_rms(as_complex(g), gr)
    print(f"g_signal rms rel {eg:.3e}")
    assert eg <= 1e-4


def test_bistatic_reciprocity(dev):
    """Swapping every transmitter with its receiver (and their occupancies)
    leaves the rendered signal unchanged: path, 1/(rt rr), T_tx T_rx and
    w_o . w_r are symmetric."""
    _say("bistatic reciprocity")
    R = _R()
    c = _bistatic(ragged_case(seed=3), 3)
    ap, sm, fl = c.g(dev)
    a = as_complex(R.render_forward(ap, sm, fl, flags=SPEC["raw"]))
    ap.tx, ap.rx = ap.rx, ap.tx
    fl.phi_tx, fl.phi_rx = fl.phi_rx, fl.phi_tx
    b = as_complex(R.render_forward(ap, sm, fl, flags=SPEC["raw"]))
    e = rel_rms(b, a)
    print(f"swapped vs original: rms rel {e:.3e}, bitwise equal {np.array_equal(a, b)}")
    assert e <= 1e-6


def test_bistatic_with_rx_equal_tx_matches_monostatic(dev):
    _say("bistatic rx = tx vs monostatic")
    R = _R()
    c = ragged_case(seed=5)
    ap, sm, fl = c.g(dev)
    mono = as_complex(R.render_forward(ap, sm, fl))
    ap.rx = ap.tx.clone()
    fl.phi_rx = fl.phi_tx.clone()
    bi = as_complex(R.render_forward(ap, sm, fl))
    e = rel_rms(bi, mono)
    print(f"rms rel {e:.3e}")
    assert e <= 1e-5


def test_bistatic_argument_errors(dev):
    """The segment weight is monostatic only; a bistatic shift needs phi_rx
    with phi_ray and phi_tx; a monostatic aperture takes no phi_rx."""
    _say("bistatic argument errors")
    R = _R()
    c = _bistatic(ragged_case(seed=7), 7)
    ap, sm, fl = c.g(dev)
    with pytest.raises(R.RfvrError, match="RFVR_E_UNSUPPORTED"):
        R.render_forward(ap, sm, fl, flags=R.WEIGHT_SEGMENT)
    fl.phi_rx = None
    with pytest.raises(R.RfvrError, match="RFVR_E_INVALID"):
        R.render_forward(ap, sm, fl)
    ap.rx = None
    fl.phi_rx = fl.phi_tx.clone()
    with pytest.raises(R.RfvrError, match="RFVR_E_INVALID"):
        R.render_forward(ap, sm, fl)


# ------------------------------------------------------------------ full size

def _full_bistatic():
    """The 2^20-point workload (32 x 32 transmitters, 128 frequencies, 64 x 64
    lines x 256 depths) with every receiver 1 cm from its transmitter along x."""
    c = full_box_case()
    c.rx = (c.tx + np.array([0.01, 0.0, 0.0], np.float32)).astype(np.float32)
    return c


def test_bistatic_render_forward_full_size_sampled_measurements(dev):
    _say("bistatic render_forward full size")
    R = _R()
    c = _full_bistatic()
    ap, sm, fl = c.g(dev)
    sig = as_complex(R.render_forward(ap, sm, fl))
    sel = np.array([0, 517, 1023])
    ref = orc.render(c.o_ap(sel), c.xyz, c.o_fields(sel=sel))
    e = rel_rms(sig[sel], ref)
    print(f"rms rel {e:.3e}")
    assert e <= 1e-4


def test_bistatic_render_backward_full_size_sampled_rays(dev):
    _say("bistatic render_backward full size")
    R = _R()
    c = _full_bistatic()
    rng = np.random.default_rng(31)
    gs = (rng.normal(size=(1024, 128)) + 1j * rng.normal(size=(1024, 128))).astype(np.complex64)
    ap, sm, fl = c.g(dev)
    out = R.render_backward(ap, sm, fl, torch.from_numpy(np.stack([gs.real, gs.imag], -1)).to(dev))
    rays = np.array([0, 1000, 2080, 2100, 2111, 4095])
    ref = orc.render_adjoint(c.o_ap(), c.xyz[rays], c.o_fields(rays=rays), gs.astype(np.complex128))
    for k in ("sdf", "grad", "refl"):
        e = rel_rms(out[k].cpu().numpy()[rays], ref[k])
        print(f"{k}: rms rel {e:.3e}")
        assert e <= 1e-4, k


def test_bistatic_mf_forward_full_size_sampled_points(dev):
    _say("bistatic mf_forward full size")
    R = _R()
    c = _full_bistatic()
    rng = np.random.default_rng(35)
    s = (rng.normal(size=(1024, 128)) + 1j * rng.normal(size=(1024, 128))).astype(np.complex64)
    ap, sm, fl = c.g(dev)
    z, p = R.mf_forward(ap, sm.xyz, torch.from_numpy(np.stack([s.real, s.imag], -1)).to(dev))
    q = rng.choice(c.xyz.shape[0] * c.xyz.shape[1], 64, replace=False)
    zr, pr = orc.mf(c.o_ap(), c.xyz.reshape(-1, 3)[q], s.astype(np.complex128))
    e = rel_rms(as_complex(z)[q], zr)
    print(f"rms rel {e:.3e}")
    assert e <= 1e-4
