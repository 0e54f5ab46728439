"""Pins of the proposal-sampler oracle against closed forms, brute force, a
library routine and finite differences (none of them re-types the oracle)."""
import numpy as np
import pytest
import torch

from oracle import proposal as op
from oracle.sampling import lateral_basis, uniform24
from synth import ProposalSpec, proposal_init, proposal_layout


def _spec():
    return ProposalSpec(pe_octaves=2, width=8, layers=2, centre=(0.0, 0.0, 0.3), half_size=0.1)


def test_network_output_bias_only():
    """All weights zero except b_out: every logit equals b_out."""
    spec = _spec()
    lay = proposal_layout(spec)
    p = np.zeros(lay["__total__"][0])
    p[lay["b_out"][0]] = -1.75
    xyz = np.random.default_rng(0).normal(size=(9, 3))
    np.testing.assert_array_equal(op.forward(p, spec, xyz), np.full(9, -1.75))


def test_network_closed_form_single_unit():
    """Hand-set weights: unit 0 of layer 0 reads x_hat, layer 1 copies it, the
    output reads it; so z = relu(x_hat) (both relus act on the same value)."""
    spec = _spec()
    lay = proposal_layout(spec)
    p = np.zeros(lay["__total__"][0])
    o, _ = lay["W0"]
    p[o + 0] = 1.0                               # W0[0][0]: x_hat component
    o, (w, fin) = lay["W1"]
    p[o + 0] = 1.0                               # W1[0][0]
    p[lay["w_out"][0]] = 1.0                     # w_out[0]
    xyz = np.array([[0.05, 0.0, 0.3], [-0.02, 0.1, 0.3], [0.0, 0.0, 0.0]])
    xh = (xyz[:, 0] - 0.0) / 0.1
    np.testing.assert_allclose(op.forward(p, spec, xyz), np.maximum(xh, 0.0), rtol=0, atol=1e-15)


def test_network_gradient_finite_differences():
    spec = _spec()
    p = proposal_init(spec, 3).astype(np.float64)
    p += 0.05 * np.random.default_rng(1).normal(size=p.shape)
    rng = np.random.default_rng(2)
    xyz = np.array(spec.centre) + 0.08 * rng.uniform(-1, 1, (40, 3))
    g = rng.normal(size=40)
    gp = op.backward(p, spec, xyz, g)
    for k in range(4):
        d = rng.normal(size=p.shape)
        eps = 1e-6
        fd = (g @ op.forward(p + eps * d, spec, xyz) - g @ op.forward(p - eps * d, spec, xyz)) / (2 * eps)
        assert abs(fd - gp @ d) <= 1e-6 * (abs(fd) + 1e-3)


def test_uniform_logits_give_linear_inverse_cdf():
    """Equal logits -> uniform pdf -> importance depth u = lo + v (hi - lo)."""
    n_ray, n_bins, n_imp, n_uni = 5, 16, 8, 3
    lo, hi = 0.2, 0.4
    u, slot = op.importance_depths(np.zeros((n_ray, n_bins)), lo, hi, n_imp, n_uni, seed=7, step=2)
    K = n_imp + n_uni
    xi = uniform24(7, 2, np.arange(n_ray)[:, None] * K + np.arange(K)[None])
    want = np.empty((n_ray, K))
    want[:, :n_uni] = lo + (np.arange(n_uni) + xi[:, :n_uni]) / n_uni * (hi - lo)
    want[:, n_uni:] = lo + (np.arange(n_imp) + xi[:, n_uni:]) / n_imp * (hi - lo)
    got = np.empty_like(u)
    np.put_along_axis(got, slot, u, 1)           # back to slot order
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13)


def test_fixed_levels_are_the_stratum_midpoints():
    """Without jitter every slot sits at the middle of its stratum: equal logits
    give importance depths lo + (k + 1/2)(hi - lo)/n_imp and uniform depths
    lo + (k + 1/2)(hi - lo)/n_uni, the same for every ray and seed; a single hot
    bin puts the importance levels that fall in its CDF interval at the
    interval's linear map into the bin."""
    n_ray, n_bins, n_imp, n_uni = 4, 16, 8, 3
    lo, hi = 0.2, 0.4
    u, slot = op.importance_depths(np.zeros((n_ray, n_bins)), lo, hi, n_imp, n_uni, seed=7, step=2, jitter=False)
    u2, _ = op.importance_depths(np.zeros((n_ray, n_bins)), lo, hi, n_imp, n_uni, seed=99, step=5, jitter=False)
    np.testing.assert_array_equal(u, u2)
    got = np.empty_like(u)
    np.put_along_axis(got, slot, u, 1)
    want_uni = lo + (np.arange(n_uni) + 0.5) / n_uni * (hi - lo)
    want_imp = lo + (np.arange(n_imp) + 0.5) / n_imp * (hi - lo)
    np.testing.assert_allclose(got[:, :n_uni], np.broadcast_to(want_uni, (n_ray, n_uni)), rtol=0, atol=1e-14)
    np.testing.assert_allclose(got[:, n_uni:], np.broadcast_to(want_imp, (n_ray, n_imp)), rtol=0, atol=1e-14)
    # one hot bin b: CDF interval [c0, c1) with c0 = b q_floor / Z, width p_hot;
    # level v in it lands at lo + (b + (v - c0) / p_hot) (hi - lo) / n_bins
    b = 5
    z = np.full((1, n_bins), -60.0)
    z[0, b] = 60.0
    uh, sh = op.importance_depths(z, lo, hi, n_imp, 0, seed=0, step=0, jitter=False)
    q = 1.0 / (1.0 + np.exp(-z[0])) + 1e-3
    pz = q / q.sum()
    c0, p_hot = pz[:b].sum(), pz[b]
    v = (np.arange(n_imp) + 0.5) / n_imp
    inside = (v >= c0) & (v < c0 + p_hot)
    want = lo + (b + (v[inside] - c0) / p_hot) * (hi - lo) / n_bins
    gotb = np.empty_like(uh)
    np.put_along_axis(gotb, sh, uh, 1)
    np.testing.assert_allclose(gotb[0, inside], want, rtol=0, atol=1e-12)


def test_inverse_cdf_matches_piecewise_linear_interpolation():
    """The importance depths equal the piecewise-linear inverse of the binned CDF,
    evaluated with numpy.interp over the bin edges."""
    rng = np.random.default_rng(4)
    n_ray, n_bins, n_imp = 6, 24, 20
    lo, hi = -0.1, 0.3
    z = rng.normal(0, 3, (n_ray, n_bins))
    u, slot = op.importance_depths(z, lo, hi, n_imp, 0, seed=1, step=0)
    xi = uniform24(1, 0, np.arange(n_ray)[:, None] * n_imp + np.arange(n_imp)[None])
    v = (np.arange(n_imp)[None] + xi) / n_imp
    q = 1.0 / (1.0 + np.exp(-z)) + 1e-3
    edges = lo + np.arange(n_bins + 1) * (hi - lo) / n_bins
    for r in range(n_ray):
        cdf = np.concatenate([[0.0], np.cumsum(q[r]) / q[r].sum()])
        want = np.sort(np.interp(v[r], cdf, edges))
        np.testing.assert_allclose(u[r], want, rtol=0, atol=1e-12)


def test_concentrated_pdf_mass_and_sorting():
    """A single hot bin draws its closed-form share of the samples; depths are
    sorted and inside [lo, hi]; the uniform slots hit one stratum each."""
    n_ray, n_bins, n_imp, n_uni = 400, 32, 16, 4
    lo, hi = 0.0, 1.0
    z = np.full((n_ray, n_bins), -40.0)
    z[:, 11] = 40.0
    u, slot = op.importance_depths(z, lo, hi, n_imp, n_uni, seed=3, step=5)
    assert np.all(np.diff(u, axis=1) >= 0) and u.min() >= lo and u.max() <= hi
    p_hot = (1.0 + 1e-3) / (1.0 + 1e-3 + (n_bins - 1) * 1e-3)
    imp = slot >= n_uni
    in_hot = (np.floor(u * n_bins) == 11) & imp
    share = in_hot.sum() / imp.sum()
    # one level per stratum of width 1/n_imp: the hot bin's CDF interval of
    # length p_hot overlaps fewer than n_imp p_hot + 2 strata, so per ray the
    # count is within 2 of n_imp p_hot
    per_ray = in_hot.sum(1)
    assert np.all(np.abs(per_ray - n_imp * p_hot) < 2.0)
    assert abs(share - p_hot) < 0.01
    uni = np.where(slot < n_uni, u, np.nan)
    for r in range(0, n_ray, 37):
        vals = uni[r][~np.isnan(uni[r])]
        np.testing.assert_array_equal(np.sort(np.floor(vals * n_uni)), np.arange(n_uni))


def test_importance_histogram_follows_pdf():
    """Chi-square test of the importance samples' bin histogram against the pdf."""
    n_ray, n_bins, n_imp = 2000, 16, 8
    rng = np.random.default_rng(9)
    z0 = rng.normal(0, 2, n_bins)
    z = np.broadcast_to(z0, (n_ray, n_bins))
    u, _ = op.importance_depths(z, 0.0, 1.0, n_imp, 0, seed=11, step=0)
    h = np.bincount(np.minimum((u * n_bins).astype(int), n_bins - 1).ravel(), minlength=n_bins)
    q = 1.0 / (1.0 + np.exp(-z0)) + 1e-3
    exp = q / q.sum() * h.sum()
    chi2 = ((h - exp) ** 2 / exp).sum()
    assert chi2 < 40.0                          # 15 dof; stratification keeps it far below


def test_bin_weights_and_targets_brute_force():
    """Spreading a segment's weight over the bins it overlaps, against brute
    force: every segment cut into 20000 equal pieces, each piece's share put
    into the bin of its centre (error below one piece per bin edge); the sum
    over bins keeps each ray's total weight."""
    rng = np.random.default_rng(5)
    n_ray, n_k, n_bins = 7, 30, 10
    lo, hi = 0.1, 0.5
    u = np.sort(rng.uniform(lo, hi, (n_ray, n_k)), 1)
    u[0, 0], u[0, -1] = lo, hi                  # the range's ends land in the end bins
    u[1, 5] = u[1, 4]                           # a zero-length segment
    w = rng.uniform(0, 0.2, (n_ray, n_k))
    w[3] = 1e-5                                  # tiny weights: the 1e-3 floor holds
    W = op.bin_weights(u, w, lo, hi, n_bins)
    Wb = np.zeros((n_ray, n_bins))
    pieces = 20000
    width = (hi - lo) / n_bins
    for r in range(n_ray):
        for k in range(n_k):
            a = u[r, k]
            e = u[r, k + 1] if k + 1 < n_k else a
            if e > a:
                x = a + (np.arange(pieces) + 0.5) * (e - a) / pieces
                b = np.minimum(((x - lo) // width).astype(int), n_bins - 1)
                np.add.at(Wb[r], b, w[r, k] / pieces)
            else:
                Wb[r, min(int((a - lo) // width), n_bins - 1)] += w[r, k]
    np.testing.assert_allclose(W, Wb, rtol=0, atol=2.0 * w.max() / pieces)
    np.testing.assert_allclose(W.sum(1), w.sum(1), rtol=1e-12)
    # a segment inside one bin stays there; one across an edge splits by length
    Wh = op.bin_weights(np.array([[0.12, 0.13, 0.19, 0.24]]), np.array([[0.5, 0.3, 0.2, 0.0]]), lo, hi, n_bins)
    # bins of 4 cm from 0.10: [0.12, 0.13] in bin 0; [0.13, 0.19] overlaps bins
    # 0, 1, 2 by 1, 4, 1 cm; [0.19, 0.24] overlaps bins 2, 3 by 3, 2 cm
    np.testing.assert_allclose(Wh[0, :4], [0.5 + 0.3 / 6, 0.3 * 4 / 6, 0.3 / 6 + 0.2 * 0.6, 0.2 * 0.4],
                               rtol=1e-12)
    t = op.targets(W)
    np.testing.assert_allclose(t.max(1)[[0, 1, 2, 4, 5, 6]], 1.0)
    np.testing.assert_allclose(t[3], W[3] / 1e-3, rtol=1e-12)
    assert np.all((t >= 0) & (t <= 1))


def test_target_depth_dilation():
    """Dilation over d bins: a hand case (a peak spreads to the d bins behind
    it, never in front, and not past the range's end), d = 0 leaves t alone,
    and the result is the running maximum over each window of d + 1 bins
    (brute force over windows)."""
    W = np.array([[0.0, 1.0, 0.0, 0.0, 0.5, 0.0, 0.0, 0.25]])
    np.testing.assert_array_equal(op.targets(W, 0), W)
    np.testing.assert_array_equal(op.targets(W, 2), [[0.0, 1.0, 1.0, 1.0, 0.5, 0.5, 0.5, 0.25]])
    np.testing.assert_array_equal(op.targets(W, 7), [[0.0] + [1.0] * 7])
    rng = np.random.default_rng(3)
    W = rng.uniform(0, 1, (5, 13)) ** 4
    t0 = op.targets(W)
    for d in (1, 3, 12):
        brute = np.array([[t0[r, max(0, b - d): b + 1].max() for b in range(13)] for r in range(5)])
        np.testing.assert_array_equal(op.targets(W, d), brute)


def test_bce_matches_library_and_gradient():
    rng = np.random.default_rng(6)
    z = rng.normal(0, 4, 300)
    z[:3] = [60.0, -60.0, 0.0]
    t = rng.uniform(size=300)
    L, g = op.bce(z, t)
    ref = torch.nn.functional.binary_cross_entropy_with_logits(torch.tensor(z), torch.tensor(t)).item()
    assert abs(L - ref) <= 1e-12 * abs(ref)
    eps = 1e-6
    for i in [0, 5, 77]:
        zp, zm = z.copy(), z.copy()
        zp[i] += eps
        zm[i] -= eps
        fd = (op.bce(zp, t)[0] - op.bce(zm, t)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-7 * abs(g[i]) + 1e-12


def test_bin_centres_on_primary_rays():
    c, h = (0.01, -0.02, 0.3), 0.1
    xyz, origin, lo, hi = op.bin_centres(c, h, (0.0, 0.0, 1.0), 4, 3, 8)
    assert xyz.shape == (12, 8, 3)
    e1, e2, w = lateral_basis((0.0, 0.0, 1.0))
    np.testing.assert_allclose(lo, 0.2) and np.testing.assert_allclose(hi, 0.4)
    np.testing.assert_allclose(xyz[:, :, 2], np.broadcast_to(0.2 + (np.arange(8) + 0.5) * 0.025, (12, 8)))
    # every ray's lateral position is constant along depth
    np.testing.assert_allclose(xyz[:, :, :2], np.broadcast_to(origin[:, None, :2], (12, 8, 2)))
