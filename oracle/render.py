"""FP64 CPU oracle of the lensless RF render, matched filter and loss.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the product package.  It shares no
code with the HIP library; the O(points x measurements x frequencies) sums run
in the plain C core (``orc_core.c``), everything per-ray or per-point runs
here in numpy float64.

Inputs are taken as given (float32 arrays are promoted to float64), so input
quantisation is common to both sides and is not counted as error.

Definitions followed (GeRaF, arXiv 2605.29097):
* occupancy Phi = logistic CDF of s*f (Sec. "Opaque density representation");
* discrete opacity from consecutive samples of the NeuS discretisation
  (Sec. "Discretization", App. B.1) -- reading: alpha_k =
  clamp((Phi_k - Phi_{k+1}) / (Phi_k + 1e-5), 0, 1), alpha of the last sample 0;
* transmittance T_k = prod_{m<k} (1 - alpha_m) (Sec. "Signal Amplitude Tracing");
* lensless shift T' = clamp(T + Phi(origin of real ray) - Phi(origin of
  primary ray), 0, 1), origins detached (Eq. lens-less-transmittance);
* amplitude amp * w * refl * alpha * T_tx * T_rx * (w_o . w_r) / (r_t r_r)
  (Eq. signal_amp_tracing, Eq. reflection_angle);
* or, with weight="segment" (monostatic): the exact integral of the round-trip
  weight T(u)^2 rho(u) over the segment [u_k, u_{k+1}] that alpha_k covers.
  Along the primary ray T rho du = -dT, so the integral is
  (T_k^2 - T_{k+1}^2) / 2 = alpha_k T_k Tbar_k with the segment's mean
  transmittance Tbar_k = T_k (1 - alpha_k / 2), whatever the spacing; on a real
  ray (Eq. lens-less-transmittance, App. B.2) T' rho' du' = T rho du as well,
  so the integral of T'^2 rho' is alpha_k T_k (Tbar_k + dPhi), clamped to
  [0, 1] like T'.  The segment's contribution sits at its midpoint
  (x_k + x_{k+1}) / 2 (the last sample, alpha = 0, at itself), with the
  sample's normal and reflectiveness;
* signal tracing Eq. ref_sim and matched filter Eq. mf-sm, with
  f_n = f0 + n df and round-trip delay d/c; P = |z| (magnitude, as printed);
* loss L = (1/Q) sum_q m_q (P_q - P*_q)^2 (Sec. "Overview", step 5).
Gradients use the PyTorch complex convention g = dL/dRe + j dL/dIm.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

SPEC_MODES = {"clamp": 0, "raw": 1, "off": 2}
ALPHA_EPS = 1e-5


def _lib():
    global _LIB
    if _LIB is None:
        from . import build as _b
        path = _b.build(force=False)
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.orc_render.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_int, ctypes.c_int, dp, dp, dp, dp, dp, dp, dp, dp, dp,
                                   ctypes.c_double, ctypes.c_int, ctypes.c_int, dp, dp]
        lib.orc_render_adjoint.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_int, ctypes.c_int, dp, dp, dp, dp,
                                           dp, dp, dp, dp, dp, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                           dp, dp, dp, dp, dp]
        lib.orc_mf.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                               ctypes.c_long, dp, dp, dp, dp, dp]
        lib.orc_mf_adjoint.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_long, dp, dp, dp, dp, dp]
        _LIB = lib
    return _LIB


def _d(a):
    """float64 C-contiguous copy (or None) and its ctypes pointer."""
    if a is None:
        return None, None
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return arr, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Aperture:
    tx: np.ndarray                 # [n_meas, 3]
    f0: float
    df: float
    n_freq: int
    rx: Optional[np.ndarray] = None  # None -> monostatic (rx = tx)

    @property
    def n_meas(self) -> int:
        return int(np.asarray(self.tx).shape[0])


@dataclass
class Fields:
    sdf: np.ndarray                # [n_ray, n_z]  (metres)
    grad: np.ndarray               # [n_ray, n_z, 3]
    refl: np.ndarray               # [n_ray, n_z]
    s: float = 64.0                # logistic sharpness (1/m)
    amp: float = 1.0               # learnt global amplitude A'_tx
    phi_ray: Optional[np.ndarray] = None   # [n_ray] Phi at primary-ray origins (detached)
    phi_tx: Optional[np.ndarray] = None    # [n_meas] Phi at transmitters (detached)
    phi_rx: Optional[np.ndarray] = None    # [n_meas] Phi at receivers (bistatic only)


# --------------------------------------------------------------------------
# per-ray quantities
# --------------------------------------------------------------------------

def logistic(x):
    """Phi(x) = 1 / (1 + exp(-x)), evaluated without overflow."""
    x = np.asarray(x, np.float64)
    e = np.exp(-np.abs(x))
    return np.where(x >= 0, 1.0 / (1.0 + e), e / (1.0 + e))


def logistic_pdf(x):
    """Phi'(x) = Phi(x) (1 - Phi(x)) = exp(-|x|) / (1 + exp(-|x|))^2."""
    e = np.exp(-np.abs(np.asarray(x, np.float64)))
    return e / (1.0 + e) ** 2


def alpha_trans(sdf, s, eps=ALPHA_EPS):
    """(Phi, alpha, T, raw) per ray for samples ordered by increasing depth.

    raw_k = (Phi_k - Phi_{k+1}) / (Phi_k + eps) for k < n_z-1 (0 for the last);
    alpha = clamp(raw, 0, 1); T_k = prod_{m<k} (1 - alpha_m), T_0 = 1.
    """
    sdf = np.asarray(sdf, np.float64)
    phi = logistic(s * sdf)
    raw = np.zeros_like(phi)
    raw[:, :-1] = (phi[:, :-1] - phi[:, 1:]) / (phi[:, :-1] + eps)
    alpha = np.clip(raw, 0.0, 1.0)
    trans = np.ones_like(phi)
    for k in range(1, phi.shape[1]):
        trans[:, k] = trans[:, k - 1] * (1.0 - alpha[:, k - 1])
    return phi, alpha, trans, raw


def unit_normal(grad):
    g = np.asarray(grad, np.float64)
    nrm = np.linalg.norm(g, axis=-1)
    return g / np.maximum(nrm, 1e-12)[..., None], nrm


# --------------------------------------------------------------------------
# forward
# --------------------------------------------------------------------------

WEIGHTS = {"sample": 0, "segment": 1}


def segment_midpoints(xyz):
    """(x_k + x_{k+1}) / 2 along each ray; the last sample stays where it is."""
    xyz = np.asarray(xyz, np.float64)
    mid = xyz.copy()
    mid[:, :-1] = 0.5 * (xyz[:, :-1] + xyz[:, 1:])
    return mid


def _scene_args(ap: Aperture, xyz, fields: Fields, ray_w, weight="sample"):
    xyz = np.asarray(xyz)
    n_ray, n_z = xyz.shape[0], xyz.shape[1]
    _, alpha, trans, _ = alpha_trans(fields.sdf, fields.s)
    nhat, _ = unit_normal(fields.grad)
    keep = []

    def P(a):
        arr, ptr = _d(a)
        keep.append(arr)
        return ptr

    if weight == "segment":
        if ap.rx is not None:
            raise ValueError("the segment weight is defined for monostatic apertures")
        pos, a_in, t_in = segment_midpoints(xyz), alpha * trans, trans * (1.0 - 0.5 * alpha)
    else:
        pos, a_in, t_in = xyz, alpha, trans
    args = [ap.n_meas, P(ap.tx), P(ap.rx), ap.n_freq, ap.f0, ap.df, n_ray, n_z, P(pos),
            P(ray_w), P(nhat), P(fields.refl), P(a_in), P(t_in), P(fields.phi_ray),
            P(fields.phi_tx), P(fields.phi_rx), float(fields.amp)]
    return args, keep, alpha, trans


def render(ap: Aperture, xyz, fields: Fields, spec: str = "clamp", ray_w=None,
           return_parts: bool = False, weight: str = "sample"):
    """Rendered signal s [n_meas, n_freq] complex128 (Eq. ref_sim); weight
    "sample" (T^2 alpha at the sample) or "segment" (see the module notes)."""
    args, keep, alpha, trans = _scene_args(ap, xyz, fields, ray_w, weight)
    s_re = np.zeros((ap.n_meas, ap.n_freq))
    s_im = np.zeros((ap.n_meas, ap.n_freq))
    dp = ctypes.POINTER(ctypes.c_double)
    _lib().orc_render(*args, SPEC_MODES[spec], WEIGHTS[weight], s_re.ctypes.data_as(dp),
                      s_im.ctypes.data_as(dp))
    s = s_re + 1j * s_im
    if return_parts:
        return s, alpha, trans
    return s


def mf(ap: Aperture, xq, s):
    """Matched filter at query points: (z [Q] complex128, P = |z| [Q])."""
    xq = np.asarray(xq).reshape(-1, 3)
    sr, psr = _d(np.real(s))
    si, psi = _d(np.imag(s))
    tx, ptx = _d(ap.tx)
    rx, prx = _d(ap.rx)
    xx, pxq = _d(xq)
    z_re = np.zeros(xq.shape[0])
    z_im = np.zeros(xq.shape[0])
    dp = ctypes.POINTER(ctypes.c_double)
    _lib().orc_mf(ap.n_meas, ptx, prx, ap.n_freq, ap.f0, ap.df, xq.shape[0], pxq, psr, psi,
                  z_re.ctypes.data_as(dp), z_im.ctypes.data_as(dp))
    z = z_re + 1j * z_im
    return z, np.abs(z)


def loss_l2(P, Pstar, mask=None):
    """L = (1/Q) sum m (P - P*)^2 and dL/dP."""
    P = np.asarray(P, np.float64).ravel()
    Pstar = np.asarray(Pstar, np.float64).ravel()
    m = np.ones_like(P) if mask is None else np.asarray(mask, np.float64).ravel()
    Q = P.size
    diff = P - Pstar
    return float(np.sum(m * diff * diff) / Q), 2.0 * m * diff / Q


# --------------------------------------------------------------------------
# adjoints
# --------------------------------------------------------------------------

def mf_adjoint(ap: Aperture, xq, z, P, g_P):
    """dL/ds [n_meas, n_freq] from dL/dP through P = |z| and the matched filter.

    dL/dz = g_P z / P (zero where P == 0); then the adjoint of the linear map
    s -> z, which carries exp(-j phase).  (The printed backward formula of
    App. A (Differentiable Matched Filter & Signal Tracing) omits the factor z;
    the factor follows from differentiating |z|.)
    """
    xq = np.asarray(xq).reshape(-1, 3)
    z = np.asarray(z).ravel()
    P = np.asarray(P, np.float64).ravel()
    g_P = np.asarray(g_P, np.float64).ravel()
    scale = np.where(P > 0, g_P / np.where(P > 0, P, 1.0), 0.0)
    gz = scale * z
    gzr, pgr = _d(np.real(gz))
    gzi, pgi = _d(np.imag(gz))
    tx, ptx = _d(ap.tx)
    rx, prx = _d(ap.rx)
    xx, pxq = _d(xq)
    gs_re = np.zeros((ap.n_meas, ap.n_freq))
    gs_im = np.zeros((ap.n_meas, ap.n_freq))
    dp = ctypes.POINTER(ctypes.c_double)
    _lib().orc_mf_adjoint(ap.n_meas, ptx, prx, ap.n_freq, ap.f0, ap.df, xq.shape[0], pxq, pgr, pgi,
                          gs_re.ctypes.data_as(dp), gs_im.ctypes.data_as(dp))
    return gs_re + 1j * gs_im


def mf_adjoint_linear(ap: Aperture, xq, gz):
    """Adjoint of the linear map s -> z alone (used by the dot-product pin)."""
    xq = np.asarray(xq).reshape(-1, 3)
    gz = np.asarray(gz).ravel()
    gzr, pgr = _d(np.real(gz))
    gzi, pgi = _d(np.imag(gz))
    tx, ptx = _d(ap.tx)
    rx, prx = _d(ap.rx)
    xx, pxq = _d(xq)
    gs_re = np.zeros((ap.n_meas, ap.n_freq))
    gs_im = np.zeros((ap.n_meas, ap.n_freq))
    dp = ctypes.POINTER(ctypes.c_double)
    _lib().orc_mf_adjoint(ap.n_meas, ptx, prx, ap.n_freq, ap.f0, ap.df, xq.shape[0], pxq, pgr, pgi,
                          gs_re.ctypes.data_as(dp), gs_im.ctypes.data_as(dp))
    return gs_re + 1j * gs_im


def render_adjoint_parts(ap: Aperture, xyz, fields: Fields, g_s, spec="clamp", ray_w=None, weight="sample"):
    """Per-point partials before the scan: dL/d(base), dL/dT, dL/dn_hat, where
    base and T are the C core's per-point inputs (see _scene_args)."""
    args, keep, alpha, trans = _scene_args(ap, xyz, fields, ray_w, weight)
    gr, pgr = _d(np.real(g_s))
    gi, pgi = _d(np.imag(g_s))
    xyz = np.asarray(xyz)
    n_pts = xyz.shape[0] * xyz.shape[1]
    g_base = np.zeros(n_pts)
    g_trans = np.zeros(n_pts)
    g_nhat = np.zeros((n_pts, 3))
    dp = ctypes.POINTER(ctypes.c_double)
    _lib().orc_render_adjoint(*args, SPEC_MODES[spec], WEIGHTS[weight], pgr, pgi, g_base.ctypes.data_as(dp),
                              g_trans.ctypes.data_as(dp), g_nhat.ctypes.data_as(dp))
    shp = xyz.shape[:2]
    return g_base.reshape(shp), g_trans.reshape(shp), g_nhat.reshape(shp + (3,)), alpha, trans


def render_adjoint(ap: Aperture, xyz, fields: Fields, g_s, spec="clamp", ray_w=None, weight="sample"):
    """Gradients of L (through s) w.r.t. the per-point fields, A' and s.

    Returns dict(sdf [n_ray,n_z], grad [n_ray,n_z,3], refl [n_ray,n_z],
    amp (scalar), s (scalar)).  The origin occupancies are detached.
    """
    g_base, g_Tin, g_nhat, alpha, trans = render_adjoint_parts(ap, xyz, fields, g_s, spec, ray_w, weight)
    n_ray, n_z = g_base.shape
    w = np.ones(n_ray) if ray_w is None else np.asarray(ray_w, np.float64)
    refl = np.asarray(fields.refl, np.float64)
    amp = float(fields.amp)
    if weight == "segment":
        # base = amp w refl alpha T and Tbar = T (1 - alpha/2)
        g_alpha = g_base * amp * w[:, None] * refl * trans - 0.5 * g_Tin * trans
        g_T = g_base * amp * w[:, None] * refl * alpha + g_Tin * (1.0 - 0.5 * alpha)
        ta = alpha * trans
    else:
        g_alpha = g_base * amp * w[:, None] * refl
        g_T = g_Tin
        ta = alpha
    g_refl = g_base * amp * w[:, None] * ta
    g_amp = float(np.sum(g_base * w[:, None] * refl * ta))

    # transmittance product scan, reverse: R_k = g_T[k+1] + (1-alpha[k+1]) R_{k+1}
    R = np.zeros((n_ray, n_z))
    for k in range(n_z - 2, -1, -1):
        R[:, k] = g_T[:, k + 1] + (1.0 - alpha[:, k + 1]) * R[:, k + 1]
    g_alpha = g_alpha - trans * R

    # alpha_k(Phi_k, Phi_{k+1}) with the clamp's pass-through on [0, 1]
    sdf = np.asarray(fields.sdf, np.float64)
    phi, _, _, raw = alpha_trans(sdf, fields.s)
    live = (raw >= 0.0) & (raw <= 1.0)
    live[:, -1] = False
    D = phi[:, :-1] + ALPHA_EPS
    da_dphi_k = np.zeros_like(phi)
    da_dphi_next = np.zeros_like(phi)
    da_dphi_k[:, :-1] = (phi[:, 1:] + ALPHA_EPS) / (D * D)
    da_dphi_next[:, :-1] = -1.0 / D
    ga = np.where(live, g_alpha, 0.0)
    g_phi = ga * da_dphi_k
    g_phi[:, 1:] += ga[:, :-1] * da_dphi_next[:, :-1]
    dens = logistic_pdf(fields.s * sdf)
    g_sdf = g_phi * fields.s * dens
    g_sharp = float(np.sum(g_phi * sdf * dens))

    # n_hat = g / max(|g|, 1e-12)
    nhat, nrm = unit_normal(fields.grad)
    big = nrm >= 1e-12
    proj = g_nhat - nhat * np.sum(nhat * g_nhat, axis=-1, keepdims=True)
    g_grad = np.where(big[..., None], proj / np.maximum(nrm, 1e-12)[..., None], g_nhat / 1e-12)
    return dict(sdf=g_sdf, grad=g_grad, refl=g_refl, amp=g_amp, s=g_sharp)
