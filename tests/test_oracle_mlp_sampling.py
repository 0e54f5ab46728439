"""Pins of the oracle's SDF network, sampler and optimiser."""
import json
import os

import numpy as np
import pytest
import torch

from oracle import mlp as omlp
from oracle import optim as oopt
from oracle import sampling as osmp
from synth import MLPSpec, mlp_init, mlp_layout

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SMALL = MLPSpec(n_layers=3, width=16, pe_octaves=2, head_width=8, head_layers=2, beta=100.0,
                centre=(0.0, 0.0, 0.30), half_size=0.10)


def _perturbed(spec, seed, scale=0.3):
    """Initial weights plus dense noise, so every weight and bias matters."""
    p = mlp_init(spec, seed).astype(np.float64)
    rng = np.random.default_rng(seed + 100)
    return p + scale * rng.normal(size=p.shape) / np.sqrt(spec.width)


def _pts(n, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform([-0.1, -0.1, 0.2], [0.1, 0.1, 0.4], (n, 3))


# ------------------------------------------------------------------ network

def test_positional_encoding_closed_form():
    x = torch.tensor([[0.25, 0.5, -0.5]], dtype=torch.float64)
    g = omlp.positional_encoding(x, 2).numpy()[0]
    s2 = np.sqrt(0.5)
    expect = [0.25, 0.5, -0.5, s2, 1.0, -1.0, s2, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, -1.0, -1.0]
    np.testing.assert_allclose(g, expect, atol=1e-15)


def test_softplus_closed_forms():
    z = torch.tensor([0.0, 1.0, -1.0, 0.003], dtype=torch.float64)
    sp = omlp.softplus(z, 100.0).numpy()
    assert abs(sp[0] - np.log(2) / 100) < 1e-16
    assert abs(sp[1] - (1.0 + np.log1p(np.exp(-100.0)) / 100)) < 1e-15
    assert abs(sp[2] - np.log1p(np.exp(-100.0)) / 100) < 1e-50
    assert abs(sp[3] - np.log1p(np.exp(0.3)) / 100) < 1e-16


def test_geometric_init_is_close_to_a_sphere():
    """The seeded geometric initialisation makes f close to the SDF of a sphere
    of radius 0.5 half_size about the cube centre (a property of that
    initialisation that breaks under transposed weights or a wrong layer order)."""
    spec = MLPSpec()
    p = mlp_init(spec, 0)
    x = _pts(400, 1)
    f, g, a = omlp.forward(p, spec, x)
    r = np.linalg.norm(x - np.array(spec.centre), axis=1)
    target = r - 0.5 * spec.half_size
    err = np.abs(f - target)
    assert np.median(err) < 0.1 * spec.half_size, np.median(err)
    nrm = np.linalg.norm(g, axis=1)
    assert 0.7 < np.median(nrm) < 1.3
    radial = (x - np.array(spec.centre)) / r[:, None]
    assert np.median(np.sum(g / nrm[:, None] * radial, 1)) > 0.9
    assert np.all((a > 0) & (a < 1))


def test_head_with_zero_weights_returns_sigmoid_of_bias():
    spec = SMALL
    p = _perturbed(spec, 3)
    lay = mlp_layout(spec)
    for k in range(spec.head_layers):
        o, shp = lay[f"Wh{k}"]
        p[o:o + int(np.prod(shp))] = 0.0
    o, shp = lay["wh_out"]
    p[o:o + int(np.prod(shp))] = 0.0
    p[lay["bh_out"][0]] = 0.7
    _, _, a = omlp.forward(p, spec, _pts(5, 2))
    np.testing.assert_allclose(a, 1.0 / (1.0 + np.exp(-0.7)), rtol=1e-14)


def test_gradient_matches_finite_differences():
    spec = SMALL
    p = _perturbed(spec, 5)
    x = _pts(7, 3)
    _, g, _ = omlp.forward(p, spec, x)
    h = 1e-7
    for c in range(3):
        xp, xm = x.copy(), x.copy()
        xp[:, c] += h
        xm[:, c] -= h
        fd = (omlp.forward(p, spec, xp)[0] - omlp.forward(p, spec, xm)[0]) / (2 * h)
        np.testing.assert_allclose(g[:, c], fd, rtol=2e-6, atol=1e-8)


def test_parameter_gradient_with_normals_matches_finite_differences():
    """The double backward (through grad_x f) against central differences of J."""
    spec = SMALL
    p = _perturbed(spec, 7)
    x = _pts(6, 4)
    rng = np.random.default_rng(8)
    gf, gg, ga = rng.normal(size=6), rng.normal(size=(6, 3)), rng.normal(size=6)
    gp = omlp.backward(p, spec, x, gf, gg, ga)
    lay = mlp_layout(spec)
    idx = [lay["W0"][0] + 1, lay["W0"][0] + 20, lay["b0"][0] + 3, lay["W1"][0] + 17,
           lay["b2"][0] + 5, lay["w_out"][0] + 2, lay["b_out"][0], lay["Wh0"][0] + 9,
           lay["bh1"][0] + 1, lay["wh_out"][0] + 4, lay["bh_out"][0]]
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (omlp.objective(pp, spec, x, gf, gg, ga) - omlp.objective(pm, spec, x, gf, gg, ga)) / (2 * h)
        assert abs(fd - gp[i]) <= 1e-5 * max(abs(fd), 1e-2 * np.abs(gp).max()), (i, fd, gp[i])
    d = rng.normal(size=p.shape)
    fd = (omlp.objective(p + h * d, spec, x, gf, gg, ga) - omlp.objective(p - h * d, spec, x, gf, gg, ga)) / (2 * h)
    assert abs(fd - gp @ d) <= 1e-5 * abs(fd)


# ------------------------------------------------------------------ sampler

def test_splitmix64_reference_outputs():
    with open(os.path.join(GOLDEN, "splitmix64_seed0.json")) as fh:
        g = json.load(fh)
    got = [int(osmp.splitmix64_output(np.uint64(0), np.uint64(k))) for k in range(len(g["outputs"]))]
    assert got == [int(h, 16) for h in g["outputs"]]


def test_grid_sampling_closed_form_small_workload():
    """16x16 rays x 16 depths in a 10 cm cube at 0.30 m: depths 0.25 + (k+1/2) 6.25 mm,
    lateral cell centres, origins on the aperture plane z = 0."""
    xyz, u, o = osmp.sample_points((0, 0, 0.30), 0.05, (0, 0, 1), 16, 16, 16, "grid")
    np.testing.assert_allclose(u[0], 0.25 + (np.arange(16) + 0.5) * 0.00625, atol=1e-15)
    np.testing.assert_allclose(xyz[:, :, 2], u, atol=1e-15)
    lat = -0.05 + (np.arange(16) + 0.5) * 0.00625
    np.testing.assert_allclose(o[:16, 0], lat, atol=1e-15)       # x fastest
    np.testing.assert_allclose(o[::16, 1], lat, atol=1e-15)
    assert np.all(o[:, 2] == 0)


def test_stratified_sampling_strata_and_uniformity():
    xyz, u, o = osmp.sample_points((0.01, -0.02, 0.30), 0.1, (0, 0, 1), 8, 8, 64, "stratified", seed=3, step=5)
    lo = 0.20 + np.arange(64) * (0.2 / 64)
    assert np.all(u >= lo[None] - 1e-15) and np.all(u < lo[None] + 0.2 / 64)
    frac = (u - lo[None]) / (0.2 / 64)
    from scipy.stats import kstest
    assert kstest(frac.ravel(), "uniform").pvalue > 1e-3
    xyz2, u2, _ = osmp.sample_points((0.01, -0.02, 0.30), 0.1, (0, 0, 1), 8, 8, 64, "stratified", seed=3, step=6)
    assert not np.allclose(u, u2)


def test_slanted_primary_direction():
    w = np.array([0.2, -0.1, 1.0])
    w /= np.linalg.norm(w)
    xyz, u, o = osmp.sample_points((0.0, 0.0, 0.3), 0.05, w, 4, 3, 5, "grid")
    assert np.allclose(o @ w, 0.0, atol=1e-15)                  # origins on the aperture plane
    d = xyz - o[:, None, :]
    np.testing.assert_allclose(d / np.linalg.norm(d, axis=-1, keepdims=True),
                               np.broadcast_to(w, d.shape), atol=1e-12)
    assert np.all(np.diff(u, axis=1) > 0)


# ------------------------------------------------------------------ optimiser

def test_adamw_first_step_and_decay():
    rng = np.random.default_rng(0)
    p0, g = rng.normal(size=10), rng.normal(size=10)
    p1, m, v = oopt.adamw_step(p0, g, np.zeros(10), np.zeros(10), 1, 1e-3, wd=0.0)
    np.testing.assert_allclose(p1, p0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    p2, _, _ = oopt.adamw_step(p0, np.zeros(10), np.zeros(10), np.zeros(10), 1, 1e-3, wd=0.1)
    np.testing.assert_allclose(p2, p0 * (1 - 1e-4), rtol=1e-14)


def test_cosine_schedule_endpoints():
    assert oopt.cosine_lr(0, 100, 1e-3) == pytest.approx(1e-3)
    assert oopt.cosine_lr(50, 100, 1e-3) == pytest.approx(5e-4)
    assert oopt.cosine_lr(100, 100, 1e-3, 1e-5) == pytest.approx(1e-5)


def test_ring_apertures_geometry():
    """Each scanning plane faces the ring centre at the given distance, its
    antennas lie in the plane x . w = offset, and plane 0 is the standard
    aperture in z = 0."""
    from synth import planar_aperture, ring_apertures
    c = np.array([0.0, 0.0, 0.30])
    planes = ring_apertures(6, 0.30, 5, 4, 2e-3, centre=c)
    np.testing.assert_allclose(planes[0]["tx"], planar_aperture(5, 4, 2e-3), atol=1e-7)
    for k, pl in enumerate(planes):
        w, tx = pl["w"], pl["tx"].astype(np.float64)
        assert abs(np.linalg.norm(w) - 1.0) < 1e-12
        np.testing.assert_allclose(tx @ w, pl["offset"], atol=1e-7)
        np.testing.assert_allclose(tx.mean(0), c - 0.30 * w, atol=1e-7)
        phi = 2 * np.pi * k / 6
        np.testing.assert_allclose(w, [-np.sin(phi), 0.0, np.cos(phi)], atol=1e-12)


def test_sampling_origins_on_the_aperture_plane():
    """With a plane offset the ray origins lie on x . w = offset and every
    sample lies on its ray; the samples themselves do not depend on it."""
    from oracle.sampling import sample_points
    w = np.array([-1.0, 0.0, 1.0]) / np.sqrt(2.0)
    a = sample_points((0.0, 0.0, 0.3), 0.05, w, 5, 3, 7)
    b = sample_points((0.0, 0.0, 0.3), 0.05, w, 5, 3, 7, plane_offset=-0.1)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_allclose(b[2] @ w, -0.1, atol=1e-14)
    d = b[0] - b[2][:, None, :]
    cross = np.cross(d, w[None, None, :])
    assert np.abs(cross).max() < 1e-14


def test_naive_samples_on_antenna_rays_and_volume_jacobian():
    """Per-antenna samples lie on the ray from the antenna through their grid
    point, inside the cube's slab; for an on-axis antenna the Jacobian-weighted
    cell volumes add up to the volume of the pyramid frustum the rays fill
    (closed form), within the midpoint rule's error."""
    from oracle.sampling import sample_naive
    c, h = (0.0, 0.0, 0.30), 0.05
    tx = np.array([[0.0, 0.0, 0.0], [0.004, -0.002, 0.0]])
    n = (8, 6, 40)
    xyz, jac = sample_naive(tx, c, h, (0, 0, 1), *n)
    assert xyz.shape == (2, 48, 40, 3) and jac.shape == (2, 48, 40)
    assert xyz[..., 2].min() > 0.25 and xyz[..., 2].max() < 0.35
    d = xyz - tx[:, None, None, :]
    cross = np.cross(d[:, :, :1, :], d)                      # all samples of a ray are collinear
    assert np.abs(cross).max() < 1e-15
    # on-axis antenna: frustum of the pyramid through the 10 cm square at z = 0.30
    dV = (2 * h / n[0]) * (2 * h / n[1]) * (2 * h / n[2])
    D, V_exact = 0.30, 4 * h * h / 0.30 ** 2 * ((0.30 + h) ** 3 - (0.30 - h) ** 3) / 3.0
    V = jac[0].sum() * dV
    assert abs(V - V_exact) / V_exact < 1e-3
    # a distant antenna gives parallel rays: the lensless grid, unit Jacobian
    far = np.array([[0.0, 0.0, -1e5]])
    xf, jf = sample_naive(far, c, h, (0, 0, 1), 4, 4, 5)
    from oracle.sampling import sample_points
    xs, _, _ = sample_points(c, h, (0, 0, 1), 4, 4, 5)
    assert np.abs(xf[0] - xs).max() < 1e-6 and np.abs(jf - 1).max() < 1e-5


def test_network_closed_form_with_trunk_biases():
    """Hand-set two-unit network whose every bias matters: layer 0 reads
    x_hat_x (plus half of its first sine feature) and 2 x_hat_y, layer 1 mixes
    the two units, the output layer and the head read known units.  f, grad_x f
    and a are written out with math.exp / math.log1p from the definitions of
    softplus_beta, the encoding and the sigmoid (dropped or mis-indexed biases,
    a transposed matrix or a missing half_size change the values)."""
    import math
    spec = MLPSpec(n_layers=2, width=2, pe_octaves=1, head_width=2, head_layers=1, beta=100.0,
                   centre=(0.01, -0.02, 0.30), half_size=0.1)
    lay = mlp_layout(spec)
    p = np.zeros(lay["__total__"][0])

    def put(name, idx, v):
        off, shp = lay[name]
        p[off + (idx if isinstance(idx, int) else idx[0] * shp[1] + idx[1])] = v

    put("W0", (0, 0), 1.0)          # x_hat_x
    put("W0", (0, 3), 0.5)          # sin(pi x_hat_x)
    put("W0", (1, 1), 2.0)          # x_hat_y
    put("b0", 0, 0.3)
    put("b0", 1, -0.1)
    put("W1", (0, 0), 1.0)
    put("W1", (0, 1), -0.5)
    put("W1", (1, 1), 0.25)
    put("b1", 0, -0.2)
    put("b1", 1, 0.05)
    put("w_out", 0, 1.0)
    put("w_out", 1, 2.0)
    put("b_out", 0, 0.05)
    put("Wh0", (0, 0), 1.0)
    put("Wh0", (1, 1), 1.0)
    put("bh0", 0, -0.1)
    put("bh0", 1, 0.2)
    put("wh_out", 0, 1.0)
    put("wh_out", 1, -1.0)
    put("bh_out", 0, 0.3)

    beta = 100.0
    sp = lambda z: max(z, 0.0) + math.log1p(math.exp(-abs(beta * z))) / beta
    dsp = lambda z: 1.0 / (1.0 + math.exp(-beta * z))
    pts = np.array([[0.05, 0.03, 0.31], [-0.02, 0.06, 0.27], [0.03, -0.01, 0.35], [0.0, 0.09, 0.30]])
    f, g, a = omlp.forward(p, spec, pts)
    for q, x in enumerate(pts):
        xh = [(x[0] - 0.01) / 0.1, (x[1] + 0.02) / 0.1]
        z00 = xh[0] + 0.5 * math.sin(math.pi * xh[0]) + 0.3
        z01 = 2.0 * xh[1] - 0.1
        h00, h01 = sp(z00), sp(z01)
        z10 = h00 - 0.5 * h01 - 0.2
        z11 = 0.25 * h01 + 0.05
        h10, h11 = sp(z10), sp(z11)
        f_h = 0.1 * (h10 + 2.0 * h11 + 0.05)
        # d/dx: chain through both units; d x_hat / dx = 1 / half_size
        dz00 = (1.0 + 0.5 * math.pi * math.cos(math.pi * xh[0])) / 0.1
        dz01 = 2.0 / 0.1
        dh00, dh01 = dsp(z00) * dz00, dsp(z01) * dz01           # d/dx and d/dy
        gx = 0.1 * (dsp(z10) * dh00)
        gy = 0.1 * (dsp(z10) * (-0.5) * dh01 + 2.0 * dsp(z11) * 0.25 * dh01)
        g0, g1 = max(h10 - 0.1, 0.0), max(h11 + 0.2, 0.0)
        a_h = 1.0 / (1.0 + math.exp(-(g0 - g1 + 0.3)))
        assert abs(f[q] - f_h) < 1e-14, (q, f[q], f_h)
        np.testing.assert_allclose(g[q], [gx, gy, 0.0], rtol=1e-12, atol=1e-15)
        assert abs(a[q] - a_h) < 1e-14
