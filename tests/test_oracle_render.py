"""Pins of the FP64 oracle's render / matched filter / loss against facts that do
not come from the oracle itself: closed forms, the paper's printed radar
numbers, invariants proved in the paper's appendix, finite differences,
adjoint identities and automatic differentiation."""
import json
import os

import numpy as np
import pytest

from oracle import render as orc
from synth import planar_aperture, freq_grid, line_points, Sphere, scene_fields

C0 = 299792458.0
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _ap(nx=4, ny=3, n_freq=5, pitch=2e-3, rx=None):
    f0, df = freq_grid(n_freq)
    return orc.Aperture(tx=planar_aperture(nx, ny, pitch).astype(np.float64), f0=f0, df=df,
                        n_freq=n_freq, rx=rx)


def _single_scatterer(n_ray=3, n_z=6, hit_ray=1, hit_k=2, s=64.0, seed=0):
    """Every sample sits in free space (f = +1 m) except that one ray steps
    to f = -2 m after sample ``hit_k``: exactly one sample has alpha != 0."""
    rng = np.random.default_rng(seed)
    xyz = np.zeros((n_ray, n_z, 3))
    xyz[:, :, 0] = rng.uniform(-0.02, 0.02, (n_ray, 1))
    xyz[:, :, 1] = rng.uniform(-0.02, 0.02, (n_ray, 1))
    xyz[:, :, 2] = 0.25 + 0.004 * np.arange(n_z)[None, :]
    sdf = np.ones((n_ray, n_z))
    sdf[hit_ray, hit_k + 1:] = -2.0
    grad = rng.normal(size=(n_ray, n_z, 3))
    refl = rng.uniform(0.2, 0.9, (n_ray, n_z))
    return xyz, orc.Fields(sdf=sdf, grad=grad, refl=refl, s=s, amp=1.7)


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("spec", ["clamp", "raw", "off"])
def test_point_scatterer_closed_form(spec):
    """Eq. ref_sim with one reflector: s = c e^{-j 4 pi f_n r / c} with
    c = A' a alpha spec / r^2, spec = 2 (n.w_i)^2 - 1 in the monostatic case."""
    ap = _ap()
    xyz, F = _single_scatterer()
    s = orc.render(ap, xyz, F, spec=spec)
    x = xyz[1, 2]
    n = F.grad[1, 2] / np.linalg.norm(F.grad[1, 2])
    alpha = (1.0 / (1.0 + np.exp(-64.0)) - 1.0 / (1.0 + np.exp(128.0))) / (1.0 / (1.0 + np.exp(-64.0)) + 1e-5)
    fn = ap.f0 + ap.df * np.arange(ap.n_freq)
    for i in range(ap.n_meas):
        d = x - ap.tx[i]
        r = np.linalg.norm(d)
        cos_i = np.dot(n, d / r)
        sp = {"clamp": max(0.0, 2 * cos_i ** 2 - 1), "raw": 2 * cos_i ** 2 - 1, "off": 1.0}[spec]
        c = F.amp * F.refl[1, 2] * alpha * sp / r ** 2
        expect = c * np.exp(-1j * 4 * np.pi * fn * r / C0)
        np.testing.assert_allclose(s[i], expect, rtol=1e-10, atol=1e-14 * abs(F.amp / r ** 2))


def test_matched_filter_point_scatterer_dirichlet():
    """At the scatterer the filter adds all N_f N_ant terms coherently; elsewhere
    each antenna contributes a Dirichlet kernel in the range difference."""
    ap = _ap(n_freq=16)
    xyz, F = _single_scatterer()
    s = orc.render(ap, xyz, F, spec="off")
    x0 = xyz[1, 2]
    r0 = np.linalg.norm(x0[None] - ap.tx, axis=1)
    amp_i = np.abs(s[:, 0])                         # c_i (real, positive here)
    q = np.stack([x0, x0 + [0.003, -0.001, 0.004], x0 + [0.0, 0.0, 0.02]])
    z, P = orc.mf(ap, q, s)
    assert abs(z[0] - ap.n_freq * amp_i.sum()) < 1e-9 * abs(z[0])
    N = ap.n_freq
    for k in (1, 2):
        rq = np.linalg.norm(q[k][None] - ap.tx, axis=1)
        delta = 2.0 * (r0 - rq) / C0
        xk = ap.df * delta
        dirich = np.exp(-1j * np.pi * (N - 1) * xk) * np.sin(np.pi * N * xk) / np.sin(np.pi * xk)
        expect = np.sum(amp_i * np.exp(-2j * np.pi * ap.f0 * delta) * dirich)
        assert abs(z[k] - expect) < 1e-9 * np.abs(z[0])


def test_frequency_shift_single_scatterer():
    """Moving the band by D multiplies each antenna's signal by e^{-j 4 pi D r / c}."""
    xyz, F = _single_scatterer()
    a1 = _ap()
    a2 = _ap()
    a2.f0 = a1.f0 + 0.37e9
    s1 = orc.render(a1, xyz, F, spec="raw")
    s2 = orc.render(a2, xyz, F, spec="raw")
    r = np.linalg.norm(xyz[1, 2][None] - a1.tx, axis=1)
    np.testing.assert_allclose(s2, s1 * np.exp(-4j * np.pi * 0.37e9 * r / C0)[:, None], rtol=1e-9)


def test_range_resolution_matches_paper_radar():
    """App. C: 77 GHz start, 64 samples at 1250 ksps, slope 70.15 MHz/us, which the
    paper states gives about 0.04 m range resolution.  The matched filter's
    range profile of one scatterer must have its first null at c / (2 B)."""
    with open(os.path.join(GOLDEN, "radar_params.json")) as fh:
        g = json.load(fh)
    df = g["slope_hz_per_s"] / g["sample_rate_hz"]
    ap = orc.Aperture(tx=np.zeros((1, 3)), f0=g["f_start_hz"], df=df, n_freq=g["n_samples"])
    xyz = np.zeros((1, 3, 3))
    xyz[0, :, 2] = [0.39, 0.40, 0.41]
    F = orc.Fields(sdf=np.array([[1.0, 1.0, -2.0]]), grad=np.tile([0, 0, -1.0], (1, 3, 1)),
                   refl=np.ones((1, 3)), s=64.0)
    s = orc.render(ap, xyz, F, spec="off")
    zs = np.linspace(0.40, 0.50, 4001)
    q = np.stack([np.zeros_like(zs), np.zeros_like(zs), zs], 1)
    _, P = orc.mf(ap, q, s)
    # first local minimum beyond the peak
    k = 1
    while not (P[k] < P[k - 1] and P[k] <= P[k + 1]):
        k += 1
    null = zs[k] - 0.40
    bw = df * g["n_samples"]
    assert abs(null - C0 / (2 * bw)) < 2.5e-5 * 4
    assert abs(null - g["range_resolution_m"]) < g["range_resolution_tol_m"]


# ---------------------------------------------------------------- alpha / T

def test_neus_telescoping_on_sphere():
    """App. B / NeuS: for Phi non-increasing along a ray, 1 - alpha_k =
    (Phi_{k+1} + eps) / (Phi_k + eps), so T_k = (Phi_k + eps)/(Phi_0 + eps) and
    sum_k T_k alpha_k = 1 - T_{N-1}."""
    sph = Sphere((0.0, 0.0, 0.30), 0.03)
    xyz, _ = line_points((0.0, 0.0, 0.265), 0.07, 6, 6, 40)   # front half of the sphere
    sdf, _, _ = scene_fields(sph, xyz)
    sdf = sdf.astype(np.float64)
    assert np.all(np.diff(sdf, axis=1) <= 0)
    phi, alpha, T, _ = orc.alpha_trans(sdf, 64.0)
    eps = orc.ALPHA_EPS
    np.testing.assert_allclose(T, (phi + eps) / (phi[:, :1] + eps), rtol=1e-12)
    np.testing.assert_allclose((T * alpha).sum(1), 1.0 - T[:, -1], rtol=1e-12, atol=1e-15)


def test_transmittance_invariants_random():
    rng = np.random.default_rng(3)
    sdf = rng.normal(0, 0.05, (50, 33))
    phi, alpha, T, _ = orc.alpha_trans(sdf, 64.0)
    assert np.all(alpha >= 0) and np.all(alpha <= 1) and np.all(alpha[:, -1] == 0)
    assert np.all(np.diff(T, axis=1) <= 0) and np.all(T <= 1) and np.all(T >= 0)
    w = (T * alpha).sum(1)
    T_end = T[:, -1] * (1 - alpha[:, -1])
    np.testing.assert_allclose(w, 1 - T_end, atol=1e-13)
    assert np.all(w <= 1 + 1e-15)


@pytest.mark.parametrize("direction", [(0, 0, 1), (0.3, 0.1, 0.95), (-0.5, 0.4, 0.77)])
def test_alpha_invariance_quadrature(direction):
    """App. B.1: 1 - exp(-int rho du) over an interval does not depend on the
    direction of the ray crossing a monotone SDF.  Quadrature of
    rho = max(-(dPhi/du)/Phi, 0) along the slanted segment is compared with the
    discrete alpha of the segment's end points."""
    s = 64.0
    nrm = np.array([0.2, -0.1, 1.0]) / np.linalg.norm([0.2, -0.1, 1.0])  # plane normal
    f = lambda x: -(x @ nrm - 0.30)                                      # decreasing along +z
    d = np.asarray(direction, float) / np.linalg.norm(direction)
    a = np.array([0.0, 0.0, 0.29])
    b = a + d * 0.02 / (d @ nrm)           # both end points at the same pair of SDF levels
    u = np.linspace(0.0, 1.0, 200001)
    pts = a[None] + u[:, None] * (b - a)[None]
    Phi = orc.logistic(s * f(pts))
    dPhi = np.gradient(Phi, u)
    rho = np.maximum(-dPhi / Phi, 0.0)
    integral = np.sum(0.5 * (rho[1:] + rho[:-1]) * np.diff(u))
    alpha_cont = 1.0 - np.exp(-integral)
    _, alpha, _, _ = orc.alpha_trans(np.array([[f(a), f(b)]]), s)
    assert abs(alpha_cont - (1 - Phi[-1] / Phi[0])) < 1e-6
    assert abs(alpha[0, 0] - alpha_cont) < 3e-5


# ---------------------------------------------------------------- structure

def _small_scene(seed=1, n_lx=3, n_ly=2, n_z=7):
    """Soft surface crossing: the SDF falls from +3 cm to -3 cm along every line
    (with seeded wiggles) and s = 40 / m, so every sample has a nonzero opacity
    and the transmittance varies along the whole line; normals lean towards the
    aperture so the clamped specular factor stays positive."""
    xyz, orig = line_points((0.0, 0.0, 0.30), 0.06, n_lx, n_ly, n_z, jitter_seed=seed)
    rng = np.random.default_rng(seed)
    n_line = xyz.shape[0]
    base = np.linspace(0.03, -0.03, n_z)[None, :] + rng.uniform(-0.004, 0.004, (n_line, 1))
    sdf = base + rng.uniform(-0.002, 0.002, (n_line, n_z))
    sdf = np.minimum.accumulate(sdf, axis=1)                  # keep it non-increasing
    grad = np.tile([0.0, 0.0, -1.0], (n_line, n_z, 1)) + rng.normal(0, 0.25, (n_line, n_z, 3))
    refl = rng.uniform(0.3, 0.9, (n_line, n_z))
    F = orc.Fields(sdf=sdf, grad=grad, refl=refl, s=40.0, amp=1.3)
    return xyz.astype(np.float64), F


def test_reciprocity_bistatic():
    """Swapping transmitter and receiver leaves the rendered signal unchanged:
    path length, 1/(r_t r_r), T_tx T_rx and w_o . w_r are all symmetric."""
    xyz, F = _small_scene()
    rng = np.random.default_rng(5)
    A = planar_aperture(3, 2, 3e-3).astype(np.float64)
    B = A + rng.uniform(-0.01, 0.01, A.shape)
    F.phi_ray = rng.uniform(0.9, 1.0, xyz.shape[0])
    pa, pb = rng.uniform(0.9, 1.0, 6), rng.uniform(0.9, 1.0, 6)
    f0, df = freq_grid(4)
    s_ab = orc.render(orc.Aperture(tx=A, rx=B, f0=f0, df=df, n_freq=4),
                      xyz, orc.Fields(**{**F.__dict__, "phi_tx": pa, "phi_rx": pb}), spec="raw")
    s_ba = orc.render(orc.Aperture(tx=B, rx=A, f0=f0, df=df, n_freq=4),
                      xyz, orc.Fields(**{**F.__dict__, "phi_tx": pb, "phi_rx": pa}), spec="raw")
    np.testing.assert_allclose(s_ab, s_ba, rtol=1e-12, atol=1e-12 * np.abs(s_ab).max())


def test_monostatic_equals_bistatic_with_rx_equal_tx():
    xyz, F = _small_scene()
    ap = _ap()
    s_m = orc.render(ap, xyz, F)
    ap_b = _ap(rx=ap.tx.copy())
    s_b = orc.render(ap_b, xyz, F)
    np.testing.assert_allclose(s_m, s_b, rtol=1e-12, atol=1e-14 * np.abs(s_m).max())


def test_linearity_and_superposition():
    xyz, F = _small_scene()
    ap = _ap()
    s = orc.render(ap, xyz, F)
    F2 = orc.Fields(**{**F.__dict__, "amp": 2 * F.amp})
    np.testing.assert_allclose(orc.render(ap, xyz, F2), 2 * s, rtol=1e-12)
    k = 2
    Fa = orc.Fields(**{**F.__dict__, "sdf": F.sdf[:k], "grad": F.grad[:k], "refl": F.refl[:k]})
    Fb = orc.Fields(**{**F.__dict__, "sdf": F.sdf[k:], "grad": F.grad[k:], "refl": F.refl[k:]})
    np.testing.assert_allclose(orc.render(ap, xyz[:k], Fa) + orc.render(ap, xyz[k:], Fb), s,
                               rtol=1e-10, atol=1e-13 * np.abs(s).max())


def test_mirror_symmetry_of_on_axis_sphere():
    """Sphere on the boresight axis, square symmetric aperture and point grid:
    mirroring the aperture in x (index ix -> nx-1-ix) leaves s unchanged."""
    sph = Sphere((0.0, 0.0, 0.30), 0.02)
    xyz, _ = line_points((0.0, 0.0, 0.30), 0.06, 4, 4, 8)
    sdf, grad, refl = scene_fields(sph, xyz)
    F = orc.Fields(sdf=sdf.astype(np.float64), grad=grad.astype(np.float64), refl=refl.astype(np.float64))
    nx = ny = 4
    ap = _ap(nx, ny)
    s = orc.render(ap, xyz.astype(np.float64), F).reshape(ny, nx, -1)
    np.testing.assert_allclose(s, s[:, ::-1], rtol=1e-9, atol=1e-12 * np.abs(s).max())
    np.testing.assert_allclose(s, s[::-1, :], rtol=1e-9, atol=1e-12 * np.abs(s).max())
    np.testing.assert_allclose(s, s.transpose(1, 0, 2), rtol=1e-9, atol=1e-12 * np.abs(s).max())


# ---------------------------------------------------------------- adjoints

def test_mf_adjoint_dot_product():
    rng = np.random.default_rng(7)
    ap = _ap()
    q = rng.uniform([-0.03, -0.03, 0.26], [0.03, 0.03, 0.34], (23, 3))
    s = rng.normal(size=(ap.n_meas, ap.n_freq)) + 1j * rng.normal(size=(ap.n_meas, ap.n_freq))
    gz = rng.normal(size=23) + 1j * rng.normal(size=23)
    z, _ = orc.mf(ap, q, s)
    gs = orc.mf_adjoint_linear(ap, q, gz)
    lhs = np.sum(np.real(np.conj(gz) * z))
    rhs = np.sum(np.real(np.conj(gs) * s))
    assert abs(lhs - rhs) < 1e-11 * (abs(lhs) + 1)


def test_render_adjoint_dot_product_in_reflectance():
    """With the specular factor off, s is linear in the reflectance; the adjoint
    returned for refl must satisfy <s', K refl> = <K^H s', refl>."""
    xyz, F = _small_scene()
    ap = _ap()
    rng = np.random.default_rng(9)
    gs = rng.normal(size=(ap.n_meas, ap.n_freq)) + 1j * rng.normal(size=(ap.n_meas, ap.n_freq))
    s = orc.render(ap, xyz, F, spec="off")
    g = orc.render_adjoint(ap, xyz, F, gs, spec="off")
    lhs = np.sum(np.real(np.conj(gs) * s))
    rhs = np.sum(g["refl"] * F.refl)
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)


def _pipeline_loss(ap, xyz, F, Pstar, spec):
    s = orc.render(ap, xyz, F, spec=spec)
    z, P = orc.mf(ap, xyz.reshape(-1, 3), s)
    return orc.loss_l2(P, Pstar)[0]


def _pipeline_grad(ap, xyz, F, Pstar, spec):
    s = orc.render(ap, xyz, F, spec=spec)
    z, P = orc.mf(ap, xyz.reshape(-1, 3), s)
    _, gP = orc.loss_l2(P, Pstar)
    gs = orc.mf_adjoint(ap, xyz.reshape(-1, 3), z, P, gP)
    return orc.render_adjoint(ap, xyz, F, gs, spec=spec)


@pytest.mark.parametrize("spec", ["raw", "clamp"])
def test_end_to_end_gradient_finite_differences(spec):
    """Loss(MF(render(fields))) gradients vs FP64 central differences."""
    xyz, F = _small_scene(seed=4, n_z=6)
    ap = _ap(3, 2, 4)
    rng = np.random.default_rng(11)
    Pstar = rng.uniform(0, 1, xyz.shape[0] * xyz.shape[1]) * 50
    g = _pipeline_grad(ap, xyz, F, Pstar, spec)
    _, _, _, raw = orc.alpha_trans(F.sdf, F.s)

    def fd(setter, h):
        Fp = orc.Fields(**{k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in F.__dict__.items()})
        Fm = orc.Fields(**{k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in F.__dict__.items()})
        setter(Fp, +h)
        setter(Fm, -h)
        return (_pipeline_loss(ap, xyz, Fp, Pstar, spec) - _pipeline_loss(ap, xyz, Fm, Pstar, spec)) / (2 * h)

    checked = 0
    for (r, k) in [(0, 2), (1, 3), (3, 1), (4, 4), (5, 0)]:
        if k < F.sdf.shape[1] - 1 and (abs(raw[r, k]) < 1e-4 or (k > 0 and abs(raw[r, k - 1]) < 1e-4)):
            continue

        def set_sdf(Fx, h, r=r, k=k):
            Fx.sdf[r, k] += h

        num = fd(set_sdf, 1e-6)
        assert abs(num - g["sdf"][r, k]) <= 1e-5 * max(abs(num), 1e-3 * np.abs(g["sdf"]).max()), (r, k)
        for c in range(3):
            def set_grad(Fx, h, r=r, k=k, c=c):
                Fx.grad[r, k, c] += h
            num = fd(set_grad, 1e-6)
            assert abs(num - g["grad"][r, k, c]) <= 1e-5 * max(abs(num), 1e-3 * np.abs(g["grad"]).max())

        def set_refl(Fx, h, r=r, k=k):
            Fx.refl[r, k] += h
        num = fd(set_refl, 1e-6)
        assert abs(num - g["refl"][r, k]) <= 1e-5 * max(abs(num), 1e-3 * np.abs(g["refl"]).max())
        checked += 1
    assert checked >= 3

    def set_amp(Fx, h):
        Fx.amp += h
    num = fd(set_amp, 1e-6)
    assert abs(num - g["amp"]) <= 1e-6 * abs(num)

    def set_s(Fx, h):
        Fx.s += h
    num = fd(set_s, 1e-4)
    assert abs(num - g["s"]) <= 1e-5 * abs(num)


def test_render_adjoint_matches_torch_autograd():
    """The hand-written adjoint (scan recurrence without division by 1-alpha,
    clamps, normalisation) against torch float64 autograd of the forward."""
    torch = pytest.importorskip("torch")
    xyz, F = _small_scene(seed=2, n_z=5)
    ap = _ap(3, 2, 3)
    rng = np.random.default_rng(13)
    gs = rng.normal(size=(ap.n_meas, ap.n_freq)) + 1j * rng.normal(size=(ap.n_meas, ap.n_freq))
    F.phi_ray = rng.uniform(0.95, 1.0, xyz.shape[0])
    F.phi_tx = rng.uniform(0.95, 1.0, ap.n_meas)
    g = orc.render_adjoint(ap, xyz, F, gs, spec="clamp")

    t = lambda a: torch.tensor(np.asarray(a, np.float64))
    sdf = t(F.sdf).requires_grad_()
    grad = t(F.grad).requires_grad_()
    refl = t(F.refl).requires_grad_()
    amp = torch.tensor(F.amp, dtype=torch.float64, requires_grad=True)
    s_ = torch.tensor(F.s, dtype=torch.float64, requires_grad=True)
    phi = torch.sigmoid(s_ * sdf)
    raw = torch.cat([(phi[:, :-1] - phi[:, 1:]) / (phi[:, :-1] + 1e-5), torch.zeros_like(phi[:, :1])], 1)
    alpha = torch.clamp(raw, 0, 1)
    T = torch.cumprod(torch.cat([torch.ones_like(alpha[:, :1]), 1 - alpha[:, :-1]], 1), 1)
    nh = grad / torch.clamp(grad.norm(dim=-1, keepdim=True), min=1e-12)
    X = t(xyz)[None]                       # [1, R, Z, 3]
    TX = t(ap.tx)[:, None, None, :]        # [I, 1, 1, 3]
    dvec = X - TX
    r = dvec.norm(dim=-1)
    wi = dvec / r[..., None]
    ni = (nh[None] * wi).sum(-1)
    spec = torch.clamp(2 * ni * ni - 1, min=0)
    Tl = torch.clamp(T[None] + t(F.phi_tx)[:, None, None] - t(F.phi_ray)[None, :, None], 0, 1)
    c = amp * refl[None] * alpha[None] * spec * Tl * Tl / (r * r)
    fn = t(ap.f0 + ap.df * np.arange(ap.n_freq))
    ph = 2 * np.pi * ((fn[:, None, None, None] * (2 * r)[None] / 299792458.0) % 1.0)  # [N, I, R, Z]
    s_re = (c[None] * torch.cos(ph)).sum((2, 3)).T
    s_im = -(c[None] * torch.sin(ph)).sum((2, 3)).T
    L = (t(gs.real) * s_re + t(gs.imag) * s_im).sum()
    L.backward()
    np.testing.assert_allclose(g["sdf"], sdf.grad.numpy(), rtol=1e-9, atol=1e-12 * np.abs(g["sdf"]).max())
    np.testing.assert_allclose(g["grad"], grad.grad.numpy(), rtol=1e-9, atol=1e-12 * np.abs(g["grad"]).max())
    np.testing.assert_allclose(g["refl"], refl.grad.numpy(), rtol=1e-9, atol=1e-12 * np.abs(g["refl"]).max())
    assert abs(g["amp"] - amp.grad.item()) < 1e-9 * abs(g["amp"])
    assert abs(g["s"] - s_.grad.item()) < 1e-8 * abs(g["s"]) + 1e-12


def test_loss_gradient_closed_form():
    rng = np.random.default_rng(1)
    P, Ps, m = rng.uniform(size=9), rng.uniform(size=9), rng.integers(0, 2, 9)
    L, g = orc.loss_l2(P, Ps, m)
    assert abs(L - np.sum(m * (P - Ps) ** 2) / 9) < 1e-15
    np.testing.assert_allclose(g, 2 * m * (P - Ps) / 9)


# ---------------------------------------------------------------- lensless shift

def _two_scatterer_ray(n_ray=3, n_z=6, hit_ray=1, s=64.0, f_mid=0.01, seed=0):
    """One ray crosses a soft step: f = +1 m for samples 0..1, f_mid at sample 2
    and -2 m from sample 3 on; every other ray stays at f = +1 m.  Exactly two
    samples carry opacity, the second behind the first (transmittance < 1)."""
    rng = np.random.default_rng(seed)
    xyz = np.zeros((n_ray, n_z, 3))
    xyz[:, :, 0] = rng.uniform(-0.02, 0.02, (n_ray, 1))
    xyz[:, :, 1] = rng.uniform(-0.02, 0.02, (n_ray, 1))
    xyz[:, :, 2] = 0.25 + 0.004 * np.arange(n_z)[None, :]
    sdf = np.ones((n_ray, n_z))
    sdf[hit_ray, 2] = f_mid
    sdf[hit_ray, 3:] = -2.0
    grad = rng.normal(size=(n_ray, n_z, 3))
    grad[..., 2] = -np.abs(grad[..., 2]) - 1.0          # normals lean towards the aperture
    refl = rng.uniform(0.2, 0.9, (n_ray, n_z))
    return xyz, sdf, grad, refl


def _hand_alpha_T(s, f_mid):
    """Opacity and transmittance of the two live samples, from the logistic CDF
    written out with math.exp (samples 1 and 2 of the hit ray)."""
    import math
    Phi = lambda x: 1.0 / (1.0 + math.exp(-x))
    p1, p2, p3 = Phi(s * 1.0), Phi(s * f_mid), Phi(s * -2.0)
    a1 = (p1 - p2) / (p1 + 1e-5)
    a2 = (p2 - p3) / (p2 + 1e-5)
    return (a1, 1.0), (a2, 1.0 - a1)


@pytest.mark.parametrize("bistatic", [False, True])
def test_transmittance_shift_closed_form_with_clamps(bistatic):
    """Eq. lens-less-transmittance with injected origin occupancies: the real-ray
    transmittance is T + Phi(real origin) - Phi(primary origin), clamped to
    [0, 1] after the shift, once for the transmitter and once for the receiver.
    The measurements' occupancies are chosen so that, over the two live samples
    (T = 1 and T = 0.655), the shifted value lies inside [0, 1], above 1 and
    below 0.  Each term is written out by hand: a swapped sign of the shift, a
    clamp taken before the shift or a missing clamp each change the sum."""
    s, f_mid = 64.0, 0.01
    xyz, sdf, grad, refl = _two_scatterer_ray(s=s, f_mid=f_mid)
    nx, ny = 4, 3
    tx = planar_aperture(nx, ny, 2e-3).astype(np.float64)
    f0, df = freq_grid(5)
    phi_ray = np.array([0.90, 0.95, 0.60])
    d_tx = np.array([-0.30, 0.04, -0.80, -0.50, 0.02, -0.10, -0.70, 0.05, -0.95, -0.40, 0.0, -0.20])
    phi_tx = phi_ray[1] + d_tx
    rx, phi_rx = None, None
    if bistatic:
        rx = tx + np.array([0.004, -0.003, 0.0])
        d_rx = np.roll(d_tx, 5)
        phi_rx = phi_ray[1] + d_rx
    ap = orc.Aperture(tx=tx, rx=rx, f0=f0, df=df, n_freq=5)
    F = orc.Fields(sdf=sdf, grad=grad, refl=refl, s=s, amp=1.3, phi_ray=phi_ray, phi_tx=phi_tx,
                   phi_rx=phi_rx)
    got = orc.render(ap, xyz, F, spec="raw")

    clamp = lambda v: min(1.0, max(0.0, v))
    fn = f0 + df * np.arange(5)
    expect = np.zeros((tx.shape[0], 5), complex)
    seen = set()
    for k, (alpha, T) in zip((1, 2), _hand_alpha_T(s, f_mid)):
        x = xyz[1, k]
        nrm = grad[1, k] / np.linalg.norm(grad[1, k])
        for i in range(tx.shape[0]):
            t_at = tx[i]
            r_at = tx[i] if rx is None else rx[i]
            dt = x - t_at
            rt = np.linalg.norm(dt)
            wi = dt / rt
            er = r_at - x
            rr = np.linalg.norm(er)
            wr = er / rr
            wo = wi - 2.0 * np.dot(nrm, wi) * nrm
            spec_f = float(np.dot(wo, wr))
            sh_t = T + phi_tx[i] - phi_ray[1]
            sh_r = T + (phi_tx[i] if rx is None else phi_rx[i]) - phi_ray[1]
            for v in (sh_t, sh_r):
                seen.add("low" if v < 0 else ("high" if v > 1 else "in"))
            c = 1.3 * refl[1, k] * alpha * spec_f * clamp(sh_t) * clamp(sh_r) / (rt * rr)
            expect[i] += c * np.exp(-2j * np.pi * fn * (rt + rr) / C0)
    assert seen == {"low", "high", "in"}
    np.testing.assert_allclose(got, expect, rtol=1e-10, atol=1e-12 * np.abs(expect).max())


@pytest.mark.parametrize("bistatic", [False, True])
def test_gradient_through_shift_and_clamps_finite_differences(bistatic):
    """Adjoint of the render with origin occupancies that push the shifted
    transmittance past both clamps for some (measurement, point) pairs: the
    oracle's gradients in sdf, grad, refl and A' against FP64 central
    differences of its own forward, at entries whose perturbation crosses no
    clamp kink.  Bistatic: receivers 1-2 cm from their transmitters with their
    own occupancies (the gradient of w_o . w_r in the normal, -2 (n.w_r w_i +
    n.w_i w_r), and of T_tx T_rx)."""
    xyz, F = _small_scene(seed=6, n_z=6)
    ap = _ap(3, 2, 4)
    rng = np.random.default_rng(21)
    F.phi_ray = rng.uniform(0.35, 0.65, xyz.shape[0])
    F.phi_tx = np.array([0.05, 0.95, 0.5, 0.2, 0.8, 0.6])
    shifts = [F.phi_tx]
    if bistatic:
        ap = _ap(3, 2, 4, rx=_ap(3, 2, 4).tx + rng.uniform(-0.02, 0.02, (6, 3)))
        F.phi_rx = np.array([0.7, 0.1, 0.9, 0.45, 0.3, 0.98])
        shifts.append(F.phi_rx)
    gs = rng.normal(size=(ap.n_meas, ap.n_freq)) + 1j * rng.normal(size=(ap.n_meas, ap.n_freq))
    g = orc.render_adjoint(ap, xyz, F, gs, spec="raw")
    _, alpha, T, raw = orc.alpha_trans(F.sdf, F.s)
    shifted = np.concatenate([T[None] + p[:, None, None] - F.phi_ray[None, :, None] for p in shifts])
    assert (shifted < 0).any() and (shifted > 1).any() and ((shifted > 0) & (shifted < 1)).any()

    def J(Fx):
        s = orc.render(ap, xyz, Fx, spec="raw")
        return float(np.sum(np.real(np.conj(gs) * s)))

    def copy(Fx):
        return orc.Fields(**{k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in Fx.__dict__.items()})

    def fd(setter, h):
        Fp, Fm = copy(F), copy(F)
        setter(Fp, +h)
        setter(Fm, -h)
        return (J(Fp) - J(Fm)) / (2 * h)

    checked = 0
    for r in range(xyz.shape[0]):
        for k in range(xyz.shape[1] - 1):
            # the entry moves alpha_{k-1}, alpha_k and every later T of the ray
            if abs(raw[r, k]) < 1e-3 or (k > 0 and abs(raw[r, k - 1]) < 1e-3):
                continue
            near = np.abs(shifted[:, r, k:]) < 1e-3
            near |= np.abs(shifted[:, r, k:] - 1.0) < 1e-3
            if near.any():
                continue

            def set_sdf(Fx, h, r=r, k=k):
                Fx.sdf[r, k] += h

            num = fd(set_sdf, 1e-7)
            assert abs(num - g["sdf"][r, k]) <= 1e-5 * max(abs(num), 1e-3 * np.abs(g["sdf"]).max()), (r, k)
            checked += 1
    assert checked >= 6
    for (r, k) in [(0, 1), (2, 3), (4, 2)]:
        for c in range(3):
            def set_grad(Fx, h, r=r, k=k, c=c):
                Fx.grad[r, k, c] += h
            num = fd(set_grad, 1e-6)
            assert abs(num - g["grad"][r, k, c]) <= 1e-6 * max(abs(num), 1e-3 * np.abs(g["grad"]).max())

        def set_refl(Fx, h, r=r, k=k):
            Fx.refl[r, k] += h
        num = fd(set_refl, 1e-6)
        assert abs(num - g["refl"][r, k]) <= 1e-6 * max(abs(num), 1e-3 * np.abs(g["refl"]).max())

    def set_amp(Fx, h):
        Fx.amp += h
    num = fd(set_amp, 1e-6)
    assert abs(num - g["amp"]) <= 1e-7 * abs(num)


def _real_ray_T(sdf_fn, start, end, s, n=4001):
    """Transmittance at ``end`` accumulated along the straight segment from
    ``start`` by the discrete alpha product of the oracle on n samples."""
    t = np.linspace(0.0, 1.0, n)
    pts = start[None] + t[:, None] * (end - start)[None]
    _, _, T, _ = orc.alpha_trans(sdf_fn(pts)[None], s)
    return float(T[0, -1])


def _sphere_sdf(c, R):
    c = np.asarray(c, np.float64)
    return lambda p: np.linalg.norm(p - c, axis=-1) - R


def _union_sdf(*fns):
    return lambda p: np.minimum.reduce([f(p) for f in fns])


def _lensless_vs_real(sdf_fn, s, tx, origins_xy, depths):
    """Per (antenna, point): the shifted primary-ray transmittance of Eq.
    lens-less-transmittance against the real ray's own dense alpha product
    (App. B.2 brute force).  Primary rays run along +z from their foot on the
    aperture plane z = 0."""
    Phi = lambda p: float(orc.logistic(s * sdf_fn(np.asarray(p)[None]))[0])
    out = []
    for (ox, oy) in origins_xy:
        o = np.array([ox, oy, 0.0])
        for d in depths:
            x = o + np.array([0.0, 0.0, d])
            T_prim = _real_ray_T(sdf_fn, o, x, s)
            for t in tx:
                T_lens = min(1.0, max(0.0, T_prim + Phi(t) - Phi(o)))
                out.append((T_lens, _real_ray_T(sdf_fn, t, x, s), Phi(t) - Phi(o)))
    return np.array(out)


def test_lensless_transmittance_against_real_rays():
    """App. B.2 / Eq. lens-less-transmittance against brute force.

    (a) Both origins in air (Phi = 1 at the aperture): along any ray that meets
    the sphere's near side, the SDF falls monotonically, so both the primary and
    the real ray telescope to Phi(x) / Phi(origin); the shift is 0 and the
    lensless value must equal the real ray's (to the 1e-5 of the opacity's
    denominator).
    (b) A soft sphere centred on the aperture plane makes Phi vary over it, so
    the shift is nonzero.  The paper's derivation assumes equal occupancy at
    corresponding points of the two rays; the discrepancy it leaves here is
    printed (reported, not asserted)."""
    s = 64.0
    target = _sphere_sdf((0.0, 0.0, 0.30), 0.04)
    tx = planar_aperture(3, 3, 0.01).astype(np.float64)
    origins = [(0.0, 0.0), (0.01, -0.005), (-0.012, 0.008)]
    res = _lensless_vs_real(target, s, tx, origins, depths=[0.20, 0.255, 0.262])
    assert np.all(np.abs(res[:, 2]) < 1e-6)
    assert np.max(np.abs(res[:, 0] - res[:, 1])) < 2e-5, np.max(np.abs(res[:, 0] - res[:, 1]))

    soft = _union_sdf(target, _sphere_sdf((0.004, -0.003, 0.0), 0.015))
    res = _lensless_vs_real(soft, s, tx, origins, depths=[0.05, 0.20, 0.262])
    shift = res[:, 2]
    err = res[:, 0] - res[:, 1]
    assert np.all(np.isfinite(err)) and np.abs(shift).max() > 0.05
    print(f"\n[report] shift |dPhi| mean {np.abs(shift).mean():.3f} max {np.abs(shift).max():.3f}; "
          f"lensless - real T: rms {np.sqrt(np.mean(err ** 2)):.3e}, max {np.abs(err).max():.3e}; "
          f"without the shift: rms {np.sqrt(np.mean((res[:, 0] - shift - res[:, 1]) ** 2)):.3e}")


# ---------------------------------------------------------------- segment weight

@pytest.mark.parametrize("n_z", [3, 7, 60])
def test_segment_weight_sum_is_independent_of_the_samples(n_z):
    """With weight="segment" every segment carries the exact integral of the
    round-trip weight T^2 rho, (T_k^2 - T_{k+1}^2) / 2, so the weights of a ray
    add up to (1 - T_end^2) / 2 whatever its samples.  All samples of the ray
    sit at one point (so every contribution has the same phase, range and
    specular factor), the SDF falls monotonically from +2 cm to -1.5 cm through
    randomly spaced levels, and NeuS telescoping gives T_end = (Phi_end + eps) /
    (Phi_0 + eps): the signal is A' a spec (1 - T_end^2) / 2 e^{-j4 pi f r/c} /
    r^2 for every sample count."""
    s, eps = 64.0, 1e-5
    rng = np.random.default_rng(n_z)
    levels = np.sort(rng.uniform(-0.015, 0.02, n_z - 2))[::-1]
    sdf = np.concatenate([[0.02], levels, [-0.015]])[None]
    x = np.array([0.003, -0.002, 0.29])
    xyz = np.tile(x, (1, n_z, 1))
    nrm = np.array([0.1, 0.05, -1.0])
    grad = np.tile(nrm, (1, n_z, 1))
    refl = np.full((1, n_z), 0.7)
    ap = _ap(3, 2, 6)
    F = orc.Fields(sdf=sdf, grad=grad, refl=refl, s=s, amp=1.4)
    got = orc.render(ap, xyz, F, spec="raw", weight="segment")
    Phi = lambda f: 1.0 / (1.0 + np.exp(-s * f))
    T_end = (Phi(-0.015) + eps) / (Phi(0.02) + eps)
    fn = ap.f0 + ap.df * np.arange(ap.n_freq)
    nh = nrm / np.linalg.norm(nrm)
    for i in range(ap.n_meas):
        d = x - ap.tx[i]
        r = np.linalg.norm(d)
        spec_f = 2.0 * np.dot(nh, d / r) ** 2 - 1.0
        expect = 1.4 * 0.7 * spec_f * 0.5 * (1.0 - T_end ** 2) * np.exp(-4j * np.pi * fn * r / C0) / r ** 2
        np.testing.assert_allclose(got[i], expect, rtol=1e-11)
    # the sample weight instead depends on the spacing (the three sample
    # counts give different sums), which is what the segment weight removes
    w_sample = orc.render(ap, xyz, F, spec="raw")[0, 0] / got[0, 0] * 0.5 * (1 - T_end ** 2)
    assert abs(w_sample - 0.5 * (1 - T_end ** 2)) > 1e-3


def test_segment_weight_closed_form_with_midpoints_and_shift():
    """The two-scatterer ray of the transmittance-shift pin, with the segment
    weight: each live segment contributes A' a spec alpha T clamp(T (1 -
    alpha/2) + dPhi, 0, 1) / r^2 at the midpoint of its two samples (range,
    phase and specular factor taken there, normal and reflectiveness from its
    first sample), written out by hand; the occupancies make the clamp act at
    both ends for some measurements."""
    s, f_mid = 64.0, 0.01
    xyz, sdf, grad, refl = _two_scatterer_ray(s=s, f_mid=f_mid)
    tx = planar_aperture(4, 3, 2e-3).astype(np.float64)
    f0, df = freq_grid(5)
    phi_ray = np.array([0.90, 0.70, 0.60])
    d_tx = np.array([-0.30, 0.25, -0.50, -0.45, 0.20, -0.10, -0.65, 0.28, -0.70, -0.40, 0.0, -0.60])
    phi_tx = phi_ray[1] + d_tx
    ap = orc.Aperture(tx=tx, f0=f0, df=df, n_freq=5)
    F = orc.Fields(sdf=sdf, grad=grad, refl=refl, s=s, amp=1.3, phi_ray=phi_ray, phi_tx=phi_tx)
    got = orc.render(ap, xyz, F, spec="raw", weight="segment")
    clamp = lambda v: min(1.0, max(0.0, v))
    fn = f0 + df * np.arange(5)
    expect = np.zeros((tx.shape[0], 5), complex)
    seen = set()
    for k, (alpha, T) in zip((1, 2), _hand_alpha_T(s, f_mid)):
        m = 0.5 * (xyz[1, k] + xyz[1, k + 1])
        nrm = grad[1, k] / np.linalg.norm(grad[1, k])
        Tbar = T * (1.0 - 0.5 * alpha)
        for i in range(tx.shape[0]):
            d = m - tx[i]
            r = np.linalg.norm(d)
            spec_f = 2.0 * np.dot(nrm, d / r) ** 2 - 1.0
            sh = Tbar + d_tx[i]
            seen.add("low" if sh < 0 else ("high" if sh > 1 else "in"))
            c = 1.3 * refl[1, k] * alpha * T * spec_f * clamp(sh) / r ** 2
            expect[i] += c * np.exp(-4j * np.pi * fn * r / C0)
    assert seen == {"low", "high", "in"}
    np.testing.assert_allclose(got, expect, rtol=1e-10, atol=1e-12 * np.abs(expect).max())


def test_segment_weight_gradient_finite_differences():
    """Adjoint of the segment-weight render (midpoints, shift past both clamps)
    in sdf, grad, refl, A' and s against FP64 central differences."""
    xyz, F = _small_scene(seed=8, n_z=6)
    ap = _ap(3, 2, 4)
    rng = np.random.default_rng(23)
    F.phi_ray = rng.uniform(0.35, 0.65, xyz.shape[0])
    F.phi_tx = np.array([0.05, 0.95, 0.5, 0.2, 0.8, 0.6])
    gs = rng.normal(size=(ap.n_meas, ap.n_freq)) + 1j * rng.normal(size=(ap.n_meas, ap.n_freq))
    g = orc.render_adjoint(ap, xyz, F, gs, spec="raw", weight="segment")
    _, alpha, T, raw = orc.alpha_trans(F.sdf, F.s)
    shifted = (T * (1 - 0.5 * alpha))[None] + F.phi_tx[:, None, None] - F.phi_ray[None, :, None]
    assert (shifted < 0).any() and (shifted > 1).any()

    def J(Fx):
        s = orc.render(ap, xyz, Fx, spec="raw", weight="segment")
        return float(np.sum(np.real(np.conj(gs) * s)))

    def copy(Fx):
        return orc.Fields(**{k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in Fx.__dict__.items()})

    def fd(setter, h):
        Fp, Fm = copy(F), copy(F)
        setter(Fp, +h)
        setter(Fm, -h)
        return (J(Fp) - J(Fm)) / (2 * h)

    checked = 0
    for r in range(xyz.shape[0]):
        for k in range(xyz.shape[1] - 1):
            if abs(raw[r, k]) < 1e-3 or (k > 0 and abs(raw[r, k - 1]) < 1e-3):
                continue
            lo = max(k - 1, 0)
            near = (np.abs(shifted[:, r, lo:]) < 1e-3) | (np.abs(shifted[:, r, lo:] - 1.0) < 1e-3)
            if near.any():
                continue

            def set_sdf(Fx, h, r=r, k=k):
                Fx.sdf[r, k] += h

            num = fd(set_sdf, 1e-7)
            assert abs(num - g["sdf"][r, k]) <= 1e-5 * max(abs(num), 1e-3 * np.abs(g["sdf"]).max()), (r, k)
            checked += 1
    assert checked >= 6
    for (r, k) in [(0, 1), (2, 3), (4, 2)]:
        for c in range(3):
            def set_grad(Fx, h, r=r, k=k, c=c):
                Fx.grad[r, k, c] += h
            num = fd(set_grad, 1e-6)
            assert abs(num - g["grad"][r, k, c]) <= 1e-6 * max(abs(num), 1e-3 * np.abs(g["grad"]).max())

        def set_refl(Fx, h, r=r, k=k):
            Fx.refl[r, k] += h
        num = fd(set_refl, 1e-6)
        assert abs(num - g["refl"][r, k]) <= 1e-6 * max(abs(num), 1e-3 * np.abs(g["refl"]).max())

    def set_amp(Fx, h):
        Fx.amp += h
    num = fd(set_amp, 1e-6)
    assert abs(num - g["amp"]) <= 1e-7 * abs(num)

    def set_s(Fx, h):
        Fx.s += h
    num = fd(set_s, 1e-4)
    assert abs(num - g["s"]) <= 1e-5 * abs(num)
