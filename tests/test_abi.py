"""C-ABI contract checks that need no GPU: the library loads, exports every
function include/rfvr.h declares, and rejects bad arguments with the
documented codes before enqueueing anything."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rfvr.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = set(re.findall(r"\b(rfvr_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


@pytest.fixture(scope="module")
def R():
    from paper_2605_29097_amd import rfvr as R
    if not os.path.exists(R.LIB_PATH):
        pytest.fail("librfvr.so is not built (run __graft_entry__.build())")
    R.lib()
    return R


def test_header_declares_the_core_entry_points():
    d = _declared()
    for name in ("rfvr_render_forward", "rfvr_render_backward", "rfvr_sample_points",
                 "rfvr_mlp_forward", "rfvr_mlp_backward", "rfvr_mf_forward", "rfvr_mf_backward"):
        assert name in d


def test_every_declared_symbol_is_exported(R):
    L = ctypes.CDLL(R.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    # and the binding knows each of them with a signature
    assert set(_declared()) <= set(R.exported_symbols())


def test_version(R):
    assert R.lib().rfvr_version() >= 100


def _ap(R, **kw):
    a = dict(n_meas=4, tx=ctypes.c_void_p(0x1000), rx=None, f0_hz=77e9, df_hz=1e8, n_freq=8)
    a.update(kw)
    return R.CAperture(**a)


def _sm(R, **kw):
    a = dict(n_ray=2, n_z=3, xyz=ctypes.c_void_p(0x2000), ray_weight=None)
    a.update(kw)
    return R.CSamples(**a)


def _fl(R, **kw):
    a = dict(sdf=ctypes.c_void_p(0x3000), grad=ctypes.c_void_p(0x3000), refl=ctypes.c_void_p(0x3000),
             phi_ray=None, phi_tx=None, phi_rx=None, s=64.0, amp_tx=1.0)
    a.update(kw)
    return R.CFields(**a)


def _fwd(R, ap, sm, fl, flags=0, ws=None, nb=0):
    return R.lib().rfvr_render_forward(ctypes.byref(ap), ctypes.byref(sm), ctypes.byref(fl), flags,
                                       ctypes.c_void_p(0x4000), None, None, ws, nb, None)


def test_render_forward_rejects_bad_arguments(R):
    L = R.lib()
    assert L.rfvr_render_forward(None, None, None, 0, None, None, None, None, 0, None) == -1
    assert _fwd(R, _ap(R, n_meas=0), _sm(R), _fl(R)) == -1
    assert _fwd(R, _ap(R, n_freq=0), _sm(R), _fl(R)) == -1
    assert _fwd(R, _ap(R, f0_hz=float("nan")), _sm(R), _fl(R)) == -1
    assert _fwd(R, _ap(R, tx=None), _sm(R), _fl(R)) == -1
    assert _fwd(R, _ap(R), _sm(R, n_z=0), _fl(R)) == -1
    assert _fwd(R, _ap(R), _sm(R), _fl(R, s=0.0)) == -1
    assert _fwd(R, _ap(R), _sm(R), _fl(R, amp_tx=float("inf"))) == -1
    assert _fwd(R, _ap(R), _sm(R), _fl(R), flags=0x3) == -1
    assert _fwd(R, _ap(R), _sm(R), _fl(R), flags=0x100) == -1
    assert b"flag" in L.rfvr_last_error()
    # bistatic apertures: accepted up to the workspace check (nothing launched)
    bi = _ap(R, rx=ctypes.c_void_p(0x5000))
    v = ctypes.c_void_p(0x5000)
    assert _fwd(R, bi, _sm(R), _fl(R)) == -2
    assert _fwd(R, bi, _sm(R), _fl(R, phi_ray=v, phi_tx=v, phi_rx=v)) == -2
    assert (L.rfvr_render_forward_ws_bytes(ctypes.byref(bi), ctypes.byref(_sm(R))) >=
            L.rfvr_render_forward_ws_bytes(ctypes.byref(_ap(R)), ctypes.byref(_sm(R))) + 4 * 32)
    # the segment weight is monostatic only
    assert _fwd(R, bi, _sm(R), _fl(R), flags=R.WEIGHT_SEGMENT) == -3
    assert b"bistatic" in L.rfvr_last_error()
    # phi_rx comes with phi_ray and phi_tx on a bistatic aperture, never on a monostatic one
    assert _fwd(R, bi, _sm(R), _fl(R, phi_ray=v, phi_tx=v)) == -1
    assert _fwd(R, bi, _sm(R), _fl(R, phi_rx=v)) == -1
    assert _fwd(R, _ap(R), _sm(R), _fl(R, phi_rx=v)) == -1


def test_workspace_is_checked_before_launch(R):
    L = R.lib()
    ap, sm, fl = _ap(R), _sm(R), _fl(R)
    need = L.rfvr_render_forward_ws_bytes(ctypes.byref(ap), ctypes.byref(sm))
    assert need > 0
    assert _fwd(R, ap, sm, fl, ws=None, nb=0) == -2
    assert _fwd(R, ap, sm, fl, ws=ctypes.c_void_p(0x10000), nb=need - 1) == -2
    assert _fwd(R, ap, sm, fl, ws=ctypes.c_void_p(0x10001), nb=need) == -2    # misaligned
    assert b"workspace" in L.rfvr_last_error()
    nb = L.rfvr_render_backward_ws_bytes(ctypes.byref(ap), ctypes.byref(sm))
    assert nb > need
    assert L.rfvr_render_backward(ctypes.byref(ap), ctypes.byref(sm), ctypes.byref(fl), 0,
                                  ctypes.c_void_p(0x4000), None, None, None, None, None, None, 0,
                                  None) == -2


def test_workspace_queries_scale_with_problem(R):
    L = R.lib()
    ap = _ap(R, n_meas=1024, n_freq=128)
    small = L.rfvr_render_forward_ws_bytes(ctypes.byref(ap), ctypes.byref(_sm(R, n_ray=16, n_z=16)))
    big = L.rfvr_render_forward_ws_bytes(ctypes.byref(ap), ctypes.byref(_sm(R, n_ray=4096, n_z=256)))
    assert big > small > 0
    assert big >= 48 * 4096 * 256          # one 48-byte record per point
    assert L.rfvr_mf_forward_ws_bytes(ctypes.byref(ap), 100, 1) > L.rfvr_mf_forward_ws_bytes(ctypes.byref(ap), 100, 0)
    assert L.rfvr_mf_backward_ws_bytes(ctypes.byref(ap), 1 << 20) >= 32 * (1 << 20)
    assert L.rfvr_loss_ws_bytes(0) == 0 and L.rfvr_loss_ws_bytes(10) >= 8


def test_mf_and_loss_reject_bad_arguments(R):
    L = R.lib()
    ap = _ap(R)
    v = ctypes.c_void_p(0x1000)
    assert L.rfvr_mf_forward(ctypes.byref(ap), v, 0, 0, v, v, v, None, None, None, v, 1 << 20, None) == -1
    assert L.rfvr_mf_forward(ctypes.byref(ap), None, 10, 0, v, v, v, None, None, None, v, 1 << 20, None) == -1
    assert L.rfvr_mf_forward(ctypes.byref(ap), v, 10, 0x8, v, v, v, None, None, None, v, 1 << 20, None) == -1
    assert L.rfvr_mf_backward(ctypes.byref(ap), v, 10, v, v, None, 0, v, v, 1 << 20, None) == -1
    assert L.rfvr_loss_l2(0, v, v, None, v, None, v, 256, None) == -1
    assert L.rfvr_loss_l2(10, v, v, None, v, None, None, 0, None) == -2


def test_size_limits_are_checked_before_launch(R):
    """Counts past RFVR_MAX_POINTS / RFVR_MAX_RAYS / RFVR_MAX_MEAS are rejected
    (and their workspace queries return 0) before anything is enqueued."""
    L = R.lib()
    hdr = open(os.path.join(ROOT, "include", "rfvr.h")).read()
    for name, val in (("MAX_POINTS", R.MAX_POINTS), ("MAX_RAYS", R.MAX_RAYS), ("MAX_MEAS", R.MAX_MEAS),
                      ("MAX_RAY_SAMPLES", R.MAX_RAY_SAMPLES)):
        m = re.search(r"#define RFVR_%s\s+(\d+)" % name, hdr)
        assert m and int(m.group(1)) == val, name
    v = ctypes.c_void_p(0x1000)
    ap = _ap(R)
    big = R.MAX_POINTS + 1
    assert L.rfvr_mf_forward_ws_bytes(ctypes.byref(ap), big, 0) == 0
    assert L.rfvr_mf_forward(ctypes.byref(ap), v, big, 0, v, v, v, None, None, None, v, 1 << 40, None) == -1
    assert L.rfvr_mf_backward(ctypes.byref(ap), v, big, v, v, v, 0, v, v, 1 << 40, None) == -1
    assert L.rfvr_loss_l2(big, v, v, None, v, None, v, 1 << 40, None) == -1
    assert L.rfvr_occupancy(big, 64.0, v, v, None) == -1
    sm = R.CSamples(R.MAX_RAYS + 1, 1, v, None, None)
    assert L.rfvr_render_forward_ws_bytes(ctypes.byref(ap), ctypes.byref(sm)) == 0
    sm = R.CSamples(1 << 24, 1 << 8, v, None, None)                   # 2^32 points
    assert L.rfvr_render_forward_ws_bytes(ctypes.byref(ap), ctypes.byref(sm)) == 0
    ap.n_meas = R.MAX_MEAS + 1
    sm = R.CSamples(4, 4, v, None, None)
    assert L.rfvr_render_forward_ws_bytes(ctypes.byref(ap), ctypes.byref(sm)) == 0
    d = R.CSampleDesc((ctypes.c_float * 3)(0, 0, 0.3), 0.05, (ctypes.c_float * 3)(0, 0, 1), 1 << 13, 1 << 13, 64,
                      0, 0, 0)                                         # 2^26 rays
    assert L.rfvr_sample_points(ctypes.byref(d), v, None, None, None) == -1
    d.n_ray_x = 1 << 12                                                # 2^25 rays x 64 depths
    assert L.rfvr_sample_points(ctypes.byref(d), v, None, None, None) == -1
    assert L.rfvr_proposal_targets(R.MAX_RAYS + 1, 8, v, v, v, 0.2, 0.4, 8, 0, v, None) == -1
    assert L.rfvr_proposal_targets(4, 8, v, v, v, 0.2, 0.4, 8, 8, v, None) == -1          # dilation >= n_bins
    assert L.rfvr_proposal_targets(4, 8, v, v, v, 0.2, 0.4, 8, -1, v, None) == -1
    prop = R.CProposal(4, 64, 2, (ctypes.c_float * 3)(0, 0, 0.3), 0.1, v)
    assert L.rfvr_proposal_ws_bytes(ctypes.byref(prop), 1 << 30) > 0
    assert L.rfvr_proposal_ws_bytes(ctypes.byref(prop), (1 << 30) + 1) == 0
    assert L.rfvr_proposal_forward(ctypes.byref(prop), v, (1 << 30) + 1, v, v, 1 << 40, None) == -1


def test_sampler_and_optimizer_reject_bad_arguments(R):
    L = R.lib()
    d = R.CSampleDesc((ctypes.c_float * 3)(0, 0, 0.3), 0.05, (ctypes.c_float * 3)(0, 0, 0), 4, 4, 4,
                      0, 0, 0)
    v = ctypes.c_void_p(0x1000)
    assert L.rfvr_sample_points(ctypes.byref(d), v, None, None, None) == -1     # zero direction
    d.primary_dir[2] = 1.0
    d.mode = 7
    assert L.rfvr_sample_points(ctypes.byref(d), v, None, None, None) == -1
    assert L.rfvr_sample_importance(ctypes.byref(d), v, 16, 4, 4, v, None, None, None) == -1   # mode 7
    assert b"mode" in L.rfvr_last_error()
    d.mode = 0
    d.half_extent = -1.0
    assert L.rfvr_sample_points(ctypes.byref(d), v, None, None, None) == -1
    assert L.rfvr_adamw(10, v, v, v, v, 0, 1e-3, 0.9, 0.999, 1e-8, 0.0, None) == -1
    assert L.rfvr_adamw(10, v, v, v, v, 1, 1e-3, 1.0, 0.999, 1e-8, 0.0, None) == -1


def test_mlp_param_count_matches_layout(R):
    from synth import MLPSpec, mlp_layout
    spec = MLPSpec()
    net = R.MLP(params=None)
    assert net.param_count() == mlp_layout(spec)["__total__"][0]
    spec2 = MLPSpec(n_layers=3, width=64, pe_octaves=4, head_width=64, head_layers=1)
    net2 = R.MLP(params=None, n_layers=3, width=64, pe_octaves=4, head_width=64, head_layers=1)
    assert net2.param_count() == mlp_layout(spec2)["__total__"][0]


def test_mlp_training_pair_checks_reserve_before_launch(R):
    L = R.lib()
    spec = dict(n_layers=8, width=256, pe_octaves=6, head_width=64, head_layers=2)
    net = R.MLP(params=None, **spec).c()
    net.params = ctypes.c_void_p(0x1000)
    n = 1000
    rb = L.rfvr_mlp_reserve_bytes(ctypes.byref(net), n)
    assert rb == (2 * 8 * 256 + 2 * 64) * n * 4   # H and the sweep adjoint S per trunk layer, the head outputs
    assert 0 < L.rfvr_mlp_forward_train_ws_bytes(ctypes.byref(net), n) < L.rfvr_mlp_forward_ws_bytes(ctypes.byref(net), n)
    assert 0 < L.rfvr_mlp_backward_train_ws_bytes(ctypes.byref(net), n) < L.rfvr_mlp_backward_ws_bytes(ctypes.byref(net), n)
    v, ws, big = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x100000), 1 << 40

    def fwd(res, nb):
        return L.rfvr_mlp_forward_train(ctypes.byref(net), v, n, v, v, v, res, nb, ws, big, None)

    def bwd(res, nb):
        return L.rfvr_mlp_backward_train(ctypes.byref(net), v, n, v, v, v, 0, v, res, nb, ws, big, None)

    for call in (fwd, bwd):
        assert call(None, 0) == -1
        assert call(ctypes.c_void_p(0x200000), rb - 1) == -2
        assert call(ctypes.c_void_p(0x200001), rb) == -2            # misaligned
        assert b"reserve" in L.rfvr_last_error()


def test_batched_calls_check_every_scene_before_launch(R):
    """A bad scene anywhere in the array is reported, with its index, before
    anything is enqueued (nothing here touches a GPU)."""
    L = R.lib()
    tx = ctypes.c_void_p(0x1000)
    good_ap = R.CAperture(4, tx, None, 77e9, 1e8, 16)
    bad_ap = R.CAperture(0, tx, None, 77e9, 1e8, 16)
    sm = R.CSamples(2, 3, ctypes.c_void_p(0x2000), None, None)
    fl = R.CFields(ctypes.c_void_p(0x3000), ctypes.c_void_p(0x3000), ctypes.c_void_p(0x3000), None, None, None,
                   64.0, 1.0, None)
    arr = (R.CScene * 3)()
    for k in range(3):
        arr[k].ap, arr[k].sm, arr[k].fl = (bad_ap if k == 2 else good_ap), sm, fl
    v, ws = ctypes.c_void_p(0x4000), ctypes.c_void_p(0x100000)
    assert L.rfvr_render_forward_batched(3, arr, 0, v, None, None, ws, 1 << 40, None) == -1
    assert b"scene 2" in L.rfvr_last_error()
    assert L.rfvr_mf_backward_batched(3, arr, v, v, v, 0, v, ws, 1 << 40, None) == -1
    assert b"scene 2" in L.rfvr_last_error()
    assert L.rfvr_render_forward_batched(0, arr, 0, v, None, None, ws, 1 << 40, None) == -1
    # what only the single-scene adjoint rejects is checked for every scene too
    pw = R.CSamples(2, 3, ctypes.c_void_p(0x2000), None, ctypes.c_void_p(0x5000))
    arr[2].ap, arr[1].sm = good_ap, pw
    assert L.rfvr_render_backward_batched(3, arr, 0, v, v, v, v, v, v, ws, 1 << 40, None) == -3
    assert b"scene 1" in L.rfvr_last_error()
    arr[1].sm = R.CSamples(1 << 30, 1 << 11, ctypes.c_void_p(0x2000), None, None)
    assert L.rfvr_mf_forward_batched(3, arr, 0, v, v, v, None, None, None, ws, 1 << 40, None) == -1
    assert b"scene 1" in L.rfvr_last_error()
    arr[1].sm = sm
    assert L.rfvr_render_forward_batched_ws_bytes(2, arr) == max(
        L.rfvr_render_forward_ws_bytes(ctypes.byref(arr[0].ap), ctypes.byref(arr[0].sm)),
        L.rfvr_render_forward_ws_bytes(ctypes.byref(arr[1].ap), ctypes.byref(arr[1].sm)))


def test_static_filter_checks_size_before_any_device_work(R):
    """rfvr_mf_forward_static refuses arguments and sizes its static scratch
    cannot hold before touching the device (no GPU here)."""
    L = R.lib()
    v = ctypes.c_void_p(0x1000)
    big = _ap(R, n_meas=16384, n_freq=256)
    assert L.rfvr_mf_forward_ws_bytes(ctypes.byref(big), 64, 0) > R.MF_STATIC_SCRATCH_BYTES
    assert L.rfvr_mf_forward_static(ctypes.byref(big), v, 64, 0, v, v, v, None, None, None, None) == -1
    assert b"RFVR_MF_STATIC_SCRATCH_BYTES" in L.rfvr_last_error()
    ap = _ap(R)
    assert L.rfvr_mf_forward_static(ctypes.byref(ap), v, 0, 0, v, v, v, None, None, None, None) == -1
    big_bi = _ap(R, n_meas=16384, n_freq=256, rx=v)          # receiver records are part of the size
    assert L.rfvr_mf_forward_ws_bytes(ctypes.byref(big_bi), 64, 0) > L.rfvr_mf_forward_ws_bytes(ctypes.byref(big), 64, 0)
    assert L.rfvr_mf_forward_static(ctypes.byref(big_bi), v, 64, 0, v, v, v, None, None, None, None) == -1
    hdr = open(HEADER).read()
    assert f"#define RFVR_MF_STATIC_SCRATCH_BYTES (32u << 20)" in hdr and R.MF_STATIC_SCRATCH_BYTES == 32 << 20


def test_mlp_precision_is_checked_before_launch(R):
    """Every RFVR_PREC_* value is accepted; anything else is rejected with
    RFVR_E_INVALID before any device work (a too-small workspace then reports
    -2 for the accepted values, so the precision check ran first)."""
    L = R.lib()
    v, ws = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x100000)
    for prec in (R.PREC_FP32, R.PREC_BF16, R.PREC_BF16X3, R.PREC_F16):
        net = R.MLP(params=None, precision=prec).c()
        net.params = v
        assert L.rfvr_mlp_forward(ctypes.byref(net), v, 1000, v, v, v, ws, 1, None) == -2
    for prec in (-1, 4, 7):
        net = R.MLP(params=None, precision=prec).c()
        net.params = v
        assert L.rfvr_mlp_forward(ctypes.byref(net), v, 1000, v, v, v, ws, 1 << 40, None) == -1
        assert b"precision" in L.rfvr_last_error()
