"""Several scenes (scan planes) or networks per call: each batched or grouped
entry point equals the single-scene calls on the same inputs bit for bit
(the same kernels run scene by scene; packing is by scene order).  The
single-scene calls are themselves held to the FP64 oracle by the other GPU
tests.  Scenes differ in aperture size, sweep, rays, depths and scene."""
import numpy as np
import pytest
import torch

from gpu_common import Case
from synth import MLPSpec, Sphere, line_points, mlp_init, planar_aperture, scene_fields

pytestmark = pytest.mark.gpu


def _R():
    from paper_2605_29097_amd import rfvr as R
    R.lib()
    return R


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _scenes(dev):
    out = []
    specs = [((6, 5), 24, 77e9, 4e9 / 23, (12, 9, 20), (0.0, 0.0, 0.30)),
             ((4, 4), 40, 78e9, 3e9 / 39, (8, 8, 33), (0.01, -0.02, 0.28)),
             ((7, 3), 17, 77.5e9, 2e9 / 16, (5, 11, 16), (-0.01, 0.01, 0.32))]
    for k, ((nx, ny), nf, f0, df, (lx, ly, nz), c) in enumerate(specs):
        tx = planar_aperture(nx, ny, 2e-3)
        xyz, _ = line_points(c, 0.08, lx, ly, nz, jitter_seed=k)
        sdf, grad, refl = scene_fields(Sphere((c[0] + 0.004, c[1], c[2] + 0.003), 0.025, 0.7), xyz)
        case = Case(tx, f0, df, nf, xyz, sdf, grad, refl, s=50.0 + 10 * k, amp=1.0 + 0.2 * k)
        out.append(case.g(dev))
    return out


def _same(a, b):
    return torch.equal(a, b)


def test_render_and_filter_batched_equal_single_scene_calls(dev):
    _say("batched render / filter, 3 scenes")
    R = _R()
    scenes = _scenes(dev)
    sig_b = R.render_forward_batched(scenes)
    sig_1 = [R.render_forward(ap, sm, fl) for ap, sm, fl in scenes]
    assert all(_same(a, b) for a, b in zip(sig_b, sig_1))
    rng = np.random.default_rng(3)
    g_sig = [torch.from_numpy(rng.normal(size=s.shape).astype(np.float32)).to(dev) for s in sig_1]
    gb = R.render_backward_batched(scenes, g_sig)
    g1 = [R.render_backward(ap, sm, fl, g) for (ap, sm, fl), g in zip(scenes, g_sig)]
    for a, b in zip(gb, g1):
        for k in ("sdf", "grad", "refl", "amp", "s"):
            assert _same(a[k], b[k]), k
    zp_b = R.mf_forward_batched(scenes, sig_1)
    zp_1 = [R.mf_forward(ap, sm.xyz, s) for (ap, sm, _), s in zip(scenes, sig_1)]
    for (zb, pb), (z1, p1) in zip(zp_b, zp_1):
        assert _same(zb, z1) and _same(pb, p1)
    g_pow = [torch.from_numpy(rng.normal(size=p.shape).astype(np.float32)).to(dev) for _, p in zp_1]
    ga_b = R.mf_backward_batched(scenes, [z for z, _ in zp_1], [p for _, p in zp_1], g_pow)
    ga_1 = [R.mf_backward(ap, sm.xyz, z, p, g) for (ap, sm, _), (z, p), g in zip(scenes, zp_1, g_pow)]
    assert all(_same(a, b) for a, b in zip(ga_b, ga_1))


def test_batched_optional_outputs_equal_single_scene_calls(dev):
    """The optional outputs: alpha / T of the render, the filter's second signal."""
    _say("batched render alpha / T, filter with two signals, 3 scenes")
    R = _R()
    scenes = _scenes(dev)
    out_b = R.render_forward_batched(scenes, want_alpha=True)
    out_1 = [R.render_forward(ap, sm, fl, want_alpha=True) for ap, sm, fl in scenes]
    for tb, t1 in zip(out_b, out_1):
        assert all(_same(a, b) for a, b in zip(tb, t1))
    rng = np.random.default_rng(8)
    sig1 = [s for s, _, _ in out_1]
    sig2 = [torch.from_numpy(rng.normal(size=s.shape).astype(np.float32)).to(dev) for s in sig1]
    zp_b = R.mf_forward_batched(scenes, sig1, sig2)
    zp_1 = [R.mf_forward(ap, sm.xyz, a, b) for (ap, sm, _), a, b in zip(scenes, sig1, sig2)]
    for tb, t1 in zip(zp_b, zp_1):
        assert len(tb) == 4 and all(_same(a, b) for a, b in zip(tb, t1))


def test_mlp_grouped_equals_single_network_calls(dev):
    _say("grouped network calls, 2 nets")
    R = _R()
    specs = [MLPSpec(n_layers=3, width=64, pe_octaves=2, head_width=64, head_layers=1), MLPSpec()]
    nets, xyzs = [], []
    for k, spec in enumerate(specs):
        p = torch.from_numpy(mlp_init(spec, 10 + k).astype(np.float32)).to(dev)
        nets.append(R.MLP(params=p, n_layers=spec.n_layers, width=spec.width, pe_octaves=spec.pe_octaves,
                          head_width=spec.head_width, head_layers=spec.head_layers, beta=spec.beta,
                          centre=spec.centre, half_size=spec.half_size))
        rng = np.random.default_rng(20 + k)
        c = np.array(spec.centre)
        xyzs.append(torch.from_numpy((c + rng.uniform(-spec.half_size, spec.half_size, (700 + 333 * k, 3)))
                                     .astype(np.float32)).to(dev))
    out_b = R.mlp_forward_grouped(nets, xyzs)
    out_1 = [R.mlp_forward(n, x) for n, x in zip(nets, xyzs)]
    for tb, t1 in zip(out_b, out_1):
        assert all(_same(a, b.reshape(a.shape)) for a, b in zip(tb, t1))
    rng = np.random.default_rng(5)
    up = [[torch.from_numpy(rng.normal(size=s).astype(np.float32)).to(dev) for s in ((x.shape[0],), (x.shape[0], 3),
                                                                                       (x.shape[0],))] for x in xyzs]
    gb = R.mlp_backward_grouped(nets, xyzs, [u[0] for u in up], [u[1] for u in up], [u[2] for u in up])
    g1 = [R.mlp_backward(n, x, *u) for n, x, u in zip(nets, xyzs, up)]
    assert all(_same(a, b) for a, b in zip(gb, g1))


def test_trainers_sharing_a_reserve_match_trainers_with_their_own(dev):
    """Two scenes stepped in turn on one shared network reserve end with the
    same parameters, bit for bit, as with a reserve each."""
    _say("two trainers, shared reserve vs own reserves")
    R = _R()
    from paper_2605_29097_amd.train import StepConfig, Trainer
    rng = np.random.default_rng(31)
    cfgs = [StepConfig(ap=(6, 6), n_freq=16, cube_centre=(0.0, 0.0, 0.30), cube_side=0.10, lines=(8, 8), n_z=16,
                       n_layers=3, width=64, pe_octaves=2, head_width=64, head_layers=1, lr_sdf=1e-3),
            StepConfig(ap=(5, 7), n_freq=16, cube_centre=(0.01, 0.0, 0.32), cube_side=0.10, lines=(8, 8), n_z=16,
                       n_layers=3, width=64, pe_octaves=2, head_width=64, head_layers=1, lr_sdf=1e-3)]
    targets = [torch.from_numpy((rng.normal(size=(c.n_meas, 16, 2)) * 1e-2).astype(np.float32)) for c in cfgs]

    def make(k):
        c = cfgs[k]
        spec = MLPSpec(n_layers=3, width=64, pe_octaves=2, head_width=64, head_layers=1,
                       centre=c.cube_centre, half_size=c.cube_side / 2)
        return Trainer(c, torch.from_numpy(mlp_init(spec, 40 + k)), targets[k], device=dev)

    own = [make(0), make(1)]
    shared = [make(0), make(1)]
    res = R.mlp_reserve(shared[0].net, cfgs[0].n_pts, dev)
    for tr in shared:
        tr.shared_reserve = res
    for _ in range(3):
        for a, b in zip(own, shared):
            la, lb = a.step(), b.step()
            assert _same(la, lb)
    for a, b in zip(own, shared):
        assert _same(a.net.params, b.net.params)
