"""Thin Python binding of librfvr (include/rfvr.h).

Argument marshalling only: every step runs in the HIP library.  Tensors are
torch CUDA tensors (device memory on the MI355X); the stream is torch's
current stream unless one is given.  Workspaces are allocated with torch's
caching allocator at the size the library's query returns.  If the shared
library is missing or fails to load, every call raises -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# RFVR_LIBRARY may point at another build of the same library (kernel tuning)
LIB_PATH = os.environ.get("RFVR_LIBRARY") or os.path.join(_HERE, "librfvr.so")

SPEC_CLAMP, SPEC_RAW, SPEC_OFF = 0x0, 0x1, 0x2
PHASE_FP64RR, PHASE_NAIVE32 = 0x0, 0x4
ACCUMULATE = 0x8
TERMS_DIRECT = 0x10      # per-frequency evaluation of the term sums
WEIGHT_SEGMENT = 0x20    # render: exact segment integral of T^2 rho, placed at the segment midpoint
SAMPLE_GRID, SAMPLE_STRATIFIED = 0, 1
PREC_FP32, PREC_BF16, PREC_BF16X3, PREC_F16 = 0, 1, 2, 3
# size limits of one call (RFVR_MAX_* in rfvr.h)
MAX_POINTS, MAX_RAYS, MAX_MEAS, MAX_RAY_SAMPLES = (1 << 31) - 1, 1 << 25, 1 << 20, 1024
ERRORS = {-1: "RFVR_E_INVALID", -2: "RFVR_E_WORKSPACE", -3: "RFVR_E_UNSUPPORTED", -4: "RFVR_E_HIP"}

_c_i32, _c_i64, _c_u32, _c_u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
_c_f, _c_d, _vp, _sz = ctypes.c_float, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t


class CAperture(ctypes.Structure):
    _fields_ = [("n_meas", _c_i32), ("tx", _vp), ("rx", _vp), ("f0_hz", _c_d), ("df_hz", _c_d),
                ("n_freq", _c_i32)]


class CSamples(ctypes.Structure):
    _fields_ = [("n_ray", _c_i32), ("n_z", _c_i32), ("xyz", _vp), ("ray_weight", _vp), ("point_weight", _vp)]


class CFields(ctypes.Structure):
    _fields_ = [("sdf", _vp), ("grad", _vp), ("refl", _vp), ("phi_ray", _vp), ("phi_tx", _vp),
                ("phi_rx", _vp), ("s", _c_f), ("amp_tx", _c_f), ("amp_ptr", _vp), ("log_s_ptr", _vp)]


class CSampleDesc(ctypes.Structure):
    _fields_ = [("centre", _c_f * 3), ("half_extent", _c_f), ("primary_dir", _c_f * 3),
                ("n_ray_x", _c_i32), ("n_ray_y", _c_i32), ("n_z", _c_i32), ("mode", _c_i32),
                ("seed", _c_u64), ("step", _c_u64), ("plane_offset", _c_f)]


class CMlp(ctypes.Structure):
    _fields_ = [("n_layers", _c_i32), ("width", _c_i32), ("pe_octaves", _c_i32),
                ("head_width", _c_i32), ("head_layers", _c_i32), ("softplus_beta", _c_f),
                ("centre", _c_f * 3), ("half_size", _c_f), ("precision", _c_i32),
                ("params", _vp)]


class CScene(ctypes.Structure):
    _fields_ = [("ap", CAperture), ("sm", CSamples), ("fl", CFields)]


class CProposal(ctypes.Structure):
    _fields_ = [("pe_octaves", _c_i32), ("width", _c_i32), ("layers", _c_i32), ("centre", _c_f * 3),
                ("half_size", _c_f), ("params", _vp)]


_P = ctypes.POINTER
_SIGS = {
    "rfvr_version": ([], _c_i32),
    "rfvr_last_error": ([], ctypes.c_char_p),
    "rfvr_render_forward_ws_bytes": ([_P(CAperture), _P(CSamples)], _sz),
    "rfvr_render_forward": ([_P(CAperture), _P(CSamples), _P(CFields), _c_u32, _vp, _vp, _vp, _vp,
                             _sz, _vp], _c_i32),
    "rfvr_render_backward_ws_bytes": ([_P(CAperture), _P(CSamples)], _sz),
    "rfvr_render_backward": ([_P(CAperture), _P(CSamples), _P(CFields), _c_u32, _vp, _vp, _vp, _vp,
                              _vp, _vp, _vp, _sz, _vp], _c_i32),
    "rfvr_mf_forward_ws_bytes": ([_P(CAperture), _c_i64, _c_i32], _sz),
    "rfvr_mf_forward": ([_P(CAperture), _vp, _c_i64, _c_u32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp],
                        _c_i32),
    "rfvr_mf_forward_static": ([_P(CAperture), _vp, _c_i64, _c_u32, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
                               _c_i32),
    "rfvr_mf_backward_ws_bytes": ([_P(CAperture), _c_i64], _sz),
    "rfvr_mf_backward": ([_P(CAperture), _vp, _c_i64, _vp, _vp, _vp, _c_u32, _vp, _vp, _sz, _vp],
                         _c_i32),
    "rfvr_loss_ws_bytes": ([_c_i64], _sz),
    "rfvr_loss_l2": ([_c_i64, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp], _c_i32),
    "rfvr_sample_points": ([_P(CSampleDesc), _vp, _vp, _vp, _vp], _c_i32),
    "rfvr_mlp_param_count": ([_P(CMlp)], _c_i64),
    "rfvr_mlp_forward_ws_bytes": ([_P(CMlp), _c_i64], _sz),
    "rfvr_mlp_forward": ([_P(CMlp), _vp, _c_i64, _vp, _vp, _vp, _vp, _sz, _vp], _c_i32),
    "rfvr_mlp_backward_ws_bytes": ([_P(CMlp), _c_i64], _sz),
    "rfvr_mlp_backward": ([_P(CMlp), _vp, _c_i64, _vp, _vp, _vp, _c_u32, _vp, _vp, _sz, _vp],
                          _c_i32),
    "rfvr_mlp_reserve_bytes": ([_P(CMlp), _c_i64], _sz),
    "rfvr_mlp_forward_train_ws_bytes": ([_P(CMlp), _c_i64], _sz),
    "rfvr_mlp_forward_train": ([_P(CMlp), _vp, _c_i64, _vp, _vp, _vp, _vp, _sz, _vp, _sz, _vp], _c_i32),
    "rfvr_mlp_backward_train_ws_bytes": ([_P(CMlp), _c_i64], _sz),
    "rfvr_mlp_backward_train": ([_P(CMlp), _vp, _c_i64, _vp, _vp, _vp, _c_u32, _vp, _vp, _sz, _vp, _sz,
                                 _vp], _c_i32),
    "rfvr_occupancy": ([_c_i64, _c_f, _vp, _vp, _vp], _c_i32),
    "rfvr_occupancy_logs": ([_c_i64, _vp, _vp, _vp, _vp], _c_i32),
    "rfvr_proposal_param_count": ([_P(CProposal)], _c_i64),
    "rfvr_proposal_ws_bytes": ([_P(CProposal), _c_i64], _sz),
    "rfvr_proposal_forward": ([_P(CProposal), _vp, _c_i64, _vp, _vp, _sz, _vp], _c_i32),
    "rfvr_proposal_backward": ([_P(CProposal), _vp, _c_i64, _vp, _c_u32, _vp, _vp, _sz, _vp], _c_i32),
    "rfvr_sample_naive": ([_P(CSampleDesc), _vp, _c_i32, _vp, _vp, _vp], _c_i32),
    "rfvr_sample_importance": ([_P(CSampleDesc), _vp, _c_i32, _c_i32, _c_i32, _vp, _vp, _vp, _vp],
                               _c_i32),
    "rfvr_proposal_targets": ([_c_i32, _c_i32, _vp, _vp, _vp, _c_f, _c_f, _c_i32, _c_i32, _vp, _vp], _c_i32),
    "rfvr_bce_ws_bytes": ([_c_i64], _sz),
    "rfvr_mask_ws_bytes": ([_c_i64], _sz),
    "rfvr_mask_update": ([_c_i64, _vp, _vp, _vp, _c_f, _c_f, _vp, _vp, _sz, _vp], _c_i32),
    "rfvr_bce": ([_c_i64, _vp, _vp, _vp, _vp, _vp, _sz, _vp], _c_i32),
    "rfvr_adamw": ([_c_i64, _vp, _vp, _vp, _vp, _c_i64, _c_f, _c_f, _c_f, _c_f, _c_f, _vp], _c_i32),
    "rfvr_term_order_ws_bytes": ([_P(CAperture), _c_i64], _sz),
    "rfvr_render_forward_batched_ws_bytes": ([_c_i32, _P(CScene)], _sz),
    "rfvr_render_forward_batched": ([_c_i32, _P(CScene), _c_u32, _vp, _vp, _vp, _vp, _sz, _vp], _c_i32),
    "rfvr_render_backward_batched_ws_bytes": ([_c_i32, _P(CScene)], _sz),
    "rfvr_render_backward_batched": ([_c_i32, _P(CScene), _c_u32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp],
                                     _c_i32),
    "rfvr_mf_forward_batched_ws_bytes": ([_c_i32, _P(CScene), _c_i32], _sz),
    "rfvr_mf_forward_batched": ([_c_i32, _P(CScene), _c_u32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp],
                                _c_i32),
    "rfvr_mf_backward_batched_ws_bytes": ([_c_i32, _P(CScene)], _sz),
    "rfvr_mf_backward_batched": ([_c_i32, _P(CScene), _vp, _vp, _vp, _c_u32, _vp, _vp, _sz, _vp], _c_i32),
    "rfvr_mlp_forward_grouped_ws_bytes": ([_c_i32, _P(CMlp), _P(_c_i64)], _sz),
    "rfvr_mlp_forward_grouped": ([_c_i32, _P(CMlp), _vp, _P(_c_i64), _vp, _vp, _vp, _vp, _sz, _vp], _c_i32),
    "rfvr_mlp_backward_grouped_ws_bytes": ([_c_i32, _P(CMlp), _P(_c_i64)], _sz),
    "rfvr_mlp_backward_grouped": ([_c_i32, _P(CMlp), _vp, _P(_c_i64), _vp, _vp, _vp, _c_u32, _vp, _vp, _sz,
                                   _vp], _c_i32),
    "rfvr_term_order": ([_P(CAperture), _vp, _c_i64, _vp, _vp, _sz, _vp], _c_i32),
}

_lib = None


class RfvrError(RuntimeError):
    pass


def lib():
    """The loaded librfvr (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RfvrError(f"librfvr.so not found at {LIB_PATH}; build it with "
                            "`python -m paper_2605_29097_amd.build` (no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def _check(rc: int, what: str):
    if rc != 0:
        msg = lib().rfvr_last_error().decode()
        raise RfvrError(f"{what} failed: {ERRORS.get(rc, rc)}: {msg}")


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensors passed to librfvr must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ws(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _f32(t, device=None):
    if t is None:
        return None
    t = torch.as_tensor(t)
    if device is not None:
        t = t.to(device)
    return t.to(torch.float32).contiguous()


# ----------------------------------------------------------------------------
# descriptors
# ----------------------------------------------------------------------------
@dataclass
class Aperture:
    tx: torch.Tensor          # [n_meas, 3] float32 on the device
    f0: float
    df: float
    n_freq: int
    rx: Optional[torch.Tensor] = None   # [n_meas, 3] receivers (bistatic), or None (rx = tx)

    def c(self) -> CAperture:
        if self.rx is not None and tuple(self.rx.shape) != tuple(self.tx.shape):
            raise ValueError(f"rx {tuple(self.rx.shape)} must have the shape of tx {tuple(self.tx.shape)}")
        return CAperture(self.tx.shape[0], _ptr(self.tx), _ptr(self.rx), float(self.f0), float(self.df),
                         int(self.n_freq))

    @property
    def n_meas(self) -> int:
        return int(self.tx.shape[0])


@dataclass
class Samples:
    xyz: torch.Tensor                      # [n_ray, n_z, 3]
    ray_weight: Optional[torch.Tensor] = None
    point_weight: Optional[torch.Tensor] = None   # [n_ray, n_z], forward render only

    def c(self) -> CSamples:
        return CSamples(self.xyz.shape[0], self.xyz.shape[1], _ptr(self.xyz), _ptr(self.ray_weight),
                        _ptr(self.point_weight))


@dataclass
class Fields:
    sdf: torch.Tensor
    grad: torch.Tensor
    refl: torch.Tensor
    s: float = 64.0
    amp: float = 1.0
    phi_ray: Optional[torch.Tensor] = None
    phi_tx: Optional[torch.Tensor] = None
    amp_dev: Optional[torch.Tensor] = None     # device [1]: overrides amp at kernel time
    log_s_dev: Optional[torch.Tensor] = None   # device [1]: s = exp(log_s) at kernel time; g_s is then
                                               # the gradient in log s
    phi_rx: Optional[torch.Tensor] = None      # [n_meas] Phi at the receivers (bistatic apertures)

    def c(self) -> CFields:
        return CFields(_ptr(self.sdf), _ptr(self.grad), _ptr(self.refl), _ptr(self.phi_ray),
                       _ptr(self.phi_tx), _ptr(self.phi_rx), float(self.s), float(self.amp),
                       _ptr(self.amp_dev), _ptr(self.log_s_dev))


# ----------------------------------------------------------------------------
# entry points (same names as the C ABI, without the prefix)
# ----------------------------------------------------------------------------
def render_forward(ap: Aperture, sm: Samples, fl: Fields, flags: int = 0, want_alpha=False,
                   out=None, stream=None):
    """signal [n_meas, n_freq, 2] float32 (and alpha, trans [n_ray, n_z] if asked).
    out: optional contiguous [n_meas, n_freq, 2] destination (e.g. rows of a bank)."""
    dev = sm.xyz.device
    cap, csm, cfl = ap.c(), sm.c(), fl.c()
    if out is not None:
        assert out.is_contiguous() and out.shape == (ap.n_meas, ap.n_freq, 2) and out.dtype == torch.float32
        sig = out
    else:
        sig = torch.empty(ap.n_meas, ap.n_freq, 2, dtype=torch.float32, device=dev)
    alpha = trans = None
    if want_alpha:
        alpha = torch.empty(sm.xyz.shape[:2], dtype=torch.float32, device=dev)
        trans = torch.empty_like(alpha)
    nb = lib().rfvr_render_forward_ws_bytes(ctypes.byref(cap), ctypes.byref(csm))
    ws = _ws(nb, dev)
    _check(lib().rfvr_render_forward(ctypes.byref(cap), ctypes.byref(csm), ctypes.byref(cfl), flags,
                                     _ptr(sig), _ptr(alpha), _ptr(trans), _ptr(ws), ws.numel(),
                                     _stream(stream)), "rfvr_render_forward")
    return (sig, alpha, trans) if want_alpha else sig


def render_backward(ap: Aperture, sm: Samples, fl: Fields, g_signal: torch.Tensor, flags: int = 0,
                    stream=None):
    """dict(sdf, grad, refl, amp, s) of gradients."""
    dev = sm.xyz.device
    cap, csm, cfl = ap.c(), sm.c(), fl.c()
    shp = tuple(sm.xyz.shape[:2])
    out = dict(sdf=torch.empty(shp, dtype=torch.float32, device=dev),
               grad=torch.empty(shp + (3,), dtype=torch.float32, device=dev),
               refl=torch.empty(shp, dtype=torch.float32, device=dev),
               amp=torch.empty(1, dtype=torch.float32, device=dev),
               s=torch.empty(1, dtype=torch.float32, device=dev))
    nb = lib().rfvr_render_backward_ws_bytes(ctypes.byref(cap), ctypes.byref(csm))
    ws = _ws(nb, dev)
    _check(lib().rfvr_render_backward(ctypes.byref(cap), ctypes.byref(csm), ctypes.byref(cfl), flags,
                                      _ptr(g_signal.contiguous()), _ptr(out["sdf"]), _ptr(out["grad"]),
                                      _ptr(out["refl"]), _ptr(out["amp"]), _ptr(out["s"]), _ptr(ws),
                                      ws.numel(), _stream(stream)), "rfvr_render_backward")
    return out


def mf_forward(ap: Aperture, xyz_q: torch.Tensor, signal: torch.Tensor, signal2=None,
               flags: int = 0, stream=None):
    """(z [Q,2], power [Q]) or, with signal2, (z, power, z2, power2)."""
    dev = xyz_q.device
    cap = ap.c()
    nq = xyz_q.numel() // 3
    z = torch.empty(nq, 2, dtype=torch.float32, device=dev)
    p = torch.empty(nq, dtype=torch.float32, device=dev)
    z2 = p2 = None
    if signal2 is not None:
        z2 = torch.empty_like(z)
        p2 = torch.empty_like(p)
    nb = lib().rfvr_mf_forward_ws_bytes(ctypes.byref(cap), nq, 1 if signal2 is not None else 0)
    ws = _ws(nb, dev)
    _check(lib().rfvr_mf_forward(ctypes.byref(cap), _ptr(xyz_q.contiguous()), nq, int(flags),
                                 _ptr(signal.contiguous()), _ptr(z), _ptr(p),
                                 _ptr(signal2.contiguous() if signal2 is not None else None),
                                 _ptr(z2), _ptr(p2), _ptr(ws), ws.numel(), _stream(stream)),
           "rfvr_mf_forward")
    return (z, p) if signal2 is None else (z, p, z2, p2)


MF_STATIC_SCRATCH_BYTES = 32 << 20     # RFVR_MF_STATIC_SCRATCH_BYTES


def mf_forward_static(ap: Aperture, xyz_q: torch.Tensor, signal: torch.Tensor, signal2=None,
                      flags: int = 0, out=None, stream=None):
    """rfvr_mf_forward_static: the filter forward on the library's static
    scratch.  The library allocates nothing; with ``out`` = (z, power) or
    (z, power, z2, power2) preallocated by the caller this wrapper allocates
    nothing either."""
    dev = xyz_q.device
    cap = ap.c()
    nq = xyz_q.numel() // 3
    if out is None:
        out = [torch.empty(nq, 2, dtype=torch.float32, device=dev), torch.empty(nq, dtype=torch.float32, device=dev)]
        if signal2 is not None:
            out += [torch.empty(nq, 2, dtype=torch.float32, device=dev),
                    torch.empty(nq, dtype=torch.float32, device=dev)]
    z, p = out[0], out[1]
    z2, p2 = (out[2], out[3]) if signal2 is not None else (None, None)
    _check(lib().rfvr_mf_forward_static(ctypes.byref(cap), _ptr(xyz_q), nq, int(flags), _ptr(signal), _ptr(z),
                                        _ptr(p), _ptr(signal2), _ptr(z2), _ptr(p2), _stream(stream)),
           "rfvr_mf_forward_static")
    return tuple(out)


def mf_backward(ap: Aperture, xyz_q: torch.Tensor, z: torch.Tensor, power: torch.Tensor,
                g_power: torch.Tensor, flags: int = 0, out=None, stream=None):
    """dL/dsignal [n_meas, n_freq, 2]."""
    dev = xyz_q.device
    cap = ap.c()
    nq = xyz_q.numel() // 3
    g = out if out is not None else torch.empty(ap.n_meas, ap.n_freq, 2, dtype=torch.float32,
                                                device=dev)
    nb = lib().rfvr_mf_backward_ws_bytes(ctypes.byref(cap), nq)
    ws = _ws(nb, dev)
    _check(lib().rfvr_mf_backward(ctypes.byref(cap), _ptr(xyz_q.contiguous()), nq, _ptr(z.contiguous()),
                                  _ptr(power.contiguous()), _ptr(g_power.contiguous()), flags, _ptr(g),
                                  _ptr(ws), ws.numel(), _stream(stream)), "rfvr_mf_backward")
    return g


def loss_l2(p: torch.Tensor, p_star: torch.Tensor, mask=None, want_grad=True, stream=None):
    n = p.numel()
    dev = p.device
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    g = torch.empty_like(p) if want_grad else None
    ws = _ws(lib().rfvr_loss_ws_bytes(n), dev)
    _check(lib().rfvr_loss_l2(n, _ptr(p.contiguous()), _ptr(p_star.contiguous()), _ptr(mask), _ptr(loss),
                              _ptr(g), _ptr(ws), ws.numel(), _stream(stream)), "rfvr_loss_l2")
    return loss, g


def _sample_desc(centre, half_extent, primary_dir, n_ray_x, n_ray_y, n_z, mode, seed, step, plane_offset=0.0):
    return CSampleDesc((_c_f * 3)(*[float(c) for c in centre]), float(half_extent),
                       (_c_f * 3)(*[float(c) for c in primary_dir]), int(n_ray_x), int(n_ray_y),
                       int(n_z), int(mode), int(seed) & (2 ** 64 - 1), int(step) & (2 ** 64 - 1),
                       float(plane_offset))


def sample_points(centre, half_extent, primary_dir, n_ray_x, n_ray_y, n_z, mode=SAMPLE_GRID,
                  seed=0, step=0, device="cuda", plane_offset=0.0, stream=None):
    """(xyz [n_ray, n_z, 3], u [n_ray, n_z], ray_origin [n_ray, 3])."""
    d = _sample_desc(centre, half_extent, primary_dir, n_ray_x, n_ray_y, n_z, mode, seed, step, plane_offset)
    n_ray = n_ray_x * n_ray_y
    xyz = torch.empty(n_ray, n_z, 3, dtype=torch.float32, device=device)
    u = torch.empty(n_ray, n_z, dtype=torch.float32, device=device)
    o = torch.empty(n_ray, 3, dtype=torch.float32, device=device)
    _check(lib().rfvr_sample_points(ctypes.byref(d), _ptr(xyz), _ptr(u), _ptr(o), _stream(stream)),
           "rfvr_sample_points")
    return xyz, u, o


@dataclass
class MLP:
    params: torch.Tensor
    n_layers: int = 8
    width: int = 256
    pe_octaves: int = 6
    head_width: int = 64
    head_layers: int = 2
    beta: float = 100.0
    centre: tuple = (0.0, 0.0, 0.30)
    half_size: float = 0.10
    precision: int = PREC_FP32

    def c(self, params: Optional[torch.Tensor] = None) -> CMlp:
        p = self.params if params is None else params
        return CMlp(self.n_layers, self.width, self.pe_octaves, self.head_width, self.head_layers,
                    float(self.beta), (_c_f * 3)(*[float(c) for c in self.centre]),
                    float(self.half_size), int(self.precision), _ptr(p))

    def param_count(self) -> int:
        return int(lib().rfvr_mlp_param_count(ctypes.byref(self.c())))


def mlp_reserve(net: MLP, n: int, device) -> torch.Tensor:
    """Reserve of the training pair for n points (every trunk layer's H and
    sweep adjoint S, every head layer's output)."""
    return _ws(lib().rfvr_mlp_reserve_bytes(ctypes.byref(net.c()), int(n)), device)


def mlp_forward(net: MLP, xyz: torch.Tensor, stream=None, reserve: Optional[torch.Tensor] = None):
    """(f [N], grad [N, 3], a [N]); with ``reserve`` (from mlp_reserve) the
    training forward, which also fills the reserve for mlp_backward."""
    dev = xyz.device
    n = xyz.numel() // 3
    cn = net.c()
    f = torch.empty(n, dtype=torch.float32, device=dev)
    g = torch.empty(n, 3, dtype=torch.float32, device=dev)
    a = torch.empty(n, dtype=torch.float32, device=dev)
    if reserve is None:
        ws = _ws(lib().rfvr_mlp_forward_ws_bytes(ctypes.byref(cn), n), dev)
        _check(lib().rfvr_mlp_forward(ctypes.byref(cn), _ptr(xyz.contiguous()), n, _ptr(f), _ptr(g), _ptr(a),
                                      _ptr(ws), ws.numel(), _stream(stream)), "rfvr_mlp_forward")
    else:
        ws = _ws(lib().rfvr_mlp_forward_train_ws_bytes(ctypes.byref(cn), n), dev)
        _check(lib().rfvr_mlp_forward_train(ctypes.byref(cn), _ptr(xyz.contiguous()), n, _ptr(f), _ptr(g),
                                            _ptr(a), _ptr(reserve), reserve.numel(), _ptr(ws), ws.numel(),
                                            _stream(stream)), "rfvr_mlp_forward_train")
    return f, g, a


def mlp_backward(net: MLP, xyz: torch.Tensor, g_sdf=None, g_grad=None, g_refl=None, flags=0,
                 out=None, stream=None, reserve: Optional[torch.Tensor] = None):
    """Parameter gradient; with ``reserve`` the training backward, which reads
    the activations the training forward left there (same net, xyz)."""
    dev = xyz.device
    n = xyz.numel() // 3
    cn = net.c()
    gp = out if out is not None else torch.empty(net.param_count(), dtype=torch.float32, device=dev)
    if reserve is None:
        ws = _ws(lib().rfvr_mlp_backward_ws_bytes(ctypes.byref(cn), n), dev)
        _check(lib().rfvr_mlp_backward(ctypes.byref(cn), _ptr(xyz.contiguous()), n, _ptr(g_sdf), _ptr(g_grad),
                                       _ptr(g_refl), flags, _ptr(gp), _ptr(ws), ws.numel(),
                                       _stream(stream)), "rfvr_mlp_backward")
    else:
        ws = _ws(lib().rfvr_mlp_backward_train_ws_bytes(ctypes.byref(cn), n), dev)
        _check(lib().rfvr_mlp_backward_train(ctypes.byref(cn), _ptr(xyz.contiguous()), n, _ptr(g_sdf),
                                             _ptr(g_grad), _ptr(g_refl), flags, _ptr(gp), _ptr(reserve),
                                             reserve.numel(), _ptr(ws), ws.numel(), _stream(stream)),
               "rfvr_mlp_backward_train")
    return gp


# ----------------------------------------------------------------------------
# several scenes (scan planes) or networks per call: lists in, packed for the
# C ABI, per-scene views out
# ----------------------------------------------------------------------------
def _scenes(scenes):
    """(ctypes array of CScene, keep-alive list) from [(Aperture, Samples, Fields or None)]."""
    arr = (CScene * len(scenes))()
    for k, (ap, sm, fl) in enumerate(scenes):
        arr[k].ap = ap.c()
        arr[k].sm = sm.c()
        if fl is not None:
            arr[k].fl = fl.c()
    return arr


def _split(t: torch.Tensor, sizes, tail=()):
    out, o = [], 0
    for n in sizes:
        out.append(t[o:o + n].view((n,) + tuple(tail)) if tail else t[o:o + n])
        o += n
    return out


def render_forward_batched(scenes, flags: int = 0, want_alpha=False, stream=None):
    """Signals of several scenes [(Aperture, Samples, Fields)]: list of [n_meas, n_freq, 2]
    (with want_alpha, list of (signal, alpha, trans) with alpha, trans [n_ray, n_z])."""
    dev = scenes[0][1].xyz.device
    arr = _scenes(scenes)
    sizes = [ap.n_meas * ap.n_freq for ap, _, _ in scenes]
    npts = [sm.xyz.shape[0] * sm.xyz.shape[1] for _, sm, _ in scenes]
    sig = torch.empty(sum(sizes), 2, dtype=torch.float32, device=dev)
    alpha = trans = None
    if want_alpha:
        alpha = torch.empty(sum(npts), dtype=torch.float32, device=dev)
        trans = torch.empty_like(alpha)
    ws = _ws(lib().rfvr_render_forward_batched_ws_bytes(len(scenes), arr), dev)
    _check(lib().rfvr_render_forward_batched(len(scenes), arr, flags, _ptr(sig), _ptr(alpha), _ptr(trans), _ptr(ws),
                                             ws.numel(), _stream(stream)), "rfvr_render_forward_batched")
    sigs = [v.view(ap.n_meas, ap.n_freq, 2) for v, (ap, _, _) in zip(_split(sig, sizes), scenes)]
    if not want_alpha:
        return sigs
    shp = [tuple(sm.xyz.shape[:2]) for _, sm, _ in scenes]
    return [(s, a.view(h), t.view(h)) for s, a, t, h in zip(sigs, _split(alpha, npts), _split(trans, npts), shp)]


def render_backward_batched(scenes, g_signals, flags: int = 0, stream=None):
    """Per-scene dicts (sdf, grad, refl, amp, s) of gradients, as render_backward."""
    dev = scenes[0][1].xyz.device
    arr = _scenes(scenes)
    npts = [sm.xyz.shape[0] * sm.xyz.shape[1] for _, sm, _ in scenes]
    n = sum(npts)
    g_sig = torch.cat([g.reshape(-1, 2) for g in g_signals]).contiguous()
    sdf = torch.empty(n, dtype=torch.float32, device=dev)
    grad = torch.empty(n, 3, dtype=torch.float32, device=dev)
    refl = torch.empty(n, dtype=torch.float32, device=dev)
    amp = torch.empty(len(scenes), dtype=torch.float32, device=dev)
    gs = torch.empty(len(scenes), dtype=torch.float32, device=dev)
    ws = _ws(lib().rfvr_render_backward_batched_ws_bytes(len(scenes), arr), dev)
    _check(lib().rfvr_render_backward_batched(len(scenes), arr, flags, _ptr(g_sig), _ptr(sdf), _ptr(grad), _ptr(refl),
                                              _ptr(amp), _ptr(gs), _ptr(ws), ws.numel(), _stream(stream)),
           "rfvr_render_backward_batched")
    out = []
    for k, (a, b, c) in enumerate(zip(_split(sdf, npts), _split(grad, npts), _split(refl, npts))):
        shp = tuple(scenes[k][1].xyz.shape[:2])
        out.append(dict(sdf=a.view(shp), grad=b.view(shp + (3,)), refl=c.view(shp), amp=amp[k:k + 1], s=gs[k:k + 1]))
    return out


def mf_forward_batched(scenes, signals, signals2=None, flags: int = 0, stream=None):
    """Matched filter of each scene's signal at its sample points: list of (z [Q, 2], power [Q]);
    with signals2 (a second signal per scene), list of (z, power, z2, power2)."""
    dev = scenes[0][1].xyz.device
    arr = _scenes([(ap, sm, None) for ap, sm, *_ in scenes])
    npts = [sm.xyz.shape[0] * sm.xyz.shape[1] for _, sm, *_ in scenes]
    sig = torch.cat([s.reshape(-1, 2) for s in signals]).contiguous()
    sig2 = None if signals2 is None else torch.cat([s.reshape(-1, 2) for s in signals2]).contiguous()
    z = torch.empty(sum(npts), 2, dtype=torch.float32, device=dev)
    p = torch.empty(sum(npts), dtype=torch.float32, device=dev)
    z2 = p2 = None
    if sig2 is not None:
        z2 = torch.empty_like(z)
        p2 = torch.empty_like(p)
    ws = _ws(lib().rfvr_mf_forward_batched_ws_bytes(len(scenes), arr, 0 if sig2 is None else 1), dev)
    _check(lib().rfvr_mf_forward_batched(len(scenes), arr, flags, _ptr(sig), _ptr(z), _ptr(p), _ptr(sig2), _ptr(z2),
                                         _ptr(p2), _ptr(ws), ws.numel(), _stream(stream)), "rfvr_mf_forward_batched")
    if sig2 is None:
        return list(zip(_split(z, npts), _split(p, npts)))
    return list(zip(_split(z, npts), _split(p, npts), _split(z2, npts), _split(p2, npts)))


def mf_backward_batched(scenes, zs, powers, g_powers, flags: int = 0, stream=None):
    """dL/dsignal of each scene: list of [n_meas, n_freq, 2]."""
    dev = scenes[0][1].xyz.device
    arr = _scenes([(ap, sm, None) for ap, sm, *_ in scenes])
    sizes = [ap.n_meas * ap.n_freq for ap, *_ in scenes]
    z = torch.cat([t.reshape(-1, 2) for t in zs]).contiguous()
    p = torch.cat([t.reshape(-1) for t in powers]).contiguous()
    gp = torch.cat([t.reshape(-1) for t in g_powers]).contiguous()
    g = torch.empty(sum(sizes), 2, dtype=torch.float32, device=dev)
    ws = _ws(lib().rfvr_mf_backward_batched_ws_bytes(len(scenes), arr), dev)
    _check(lib().rfvr_mf_backward_batched(len(scenes), arr, _ptr(z), _ptr(p), _ptr(gp), flags, _ptr(g), _ptr(ws),
                                          ws.numel(), _stream(stream)), "rfvr_mf_backward_batched")
    return [v.view(ap.n_meas, ap.n_freq, 2) for v, (ap, *_) in zip(_split(g, sizes), scenes)]


def _nets(nets, xyzs):
    arr = (CMlp * len(nets))()
    for k, net in enumerate(nets):
        arr[k] = net.c()
    cnt = (_c_i64 * len(nets))(*[x.numel() // 3 for x in xyzs])
    return arr, cnt


def mlp_forward_grouped(nets, xyzs, stream=None):
    """(f, grad, a) of several networks, each at its own points: list of triples."""
    dev = xyzs[0].device
    arr, cnt = _nets(nets, xyzs)
    n = [int(c) for c in cnt]
    x = torch.cat([t.reshape(-1, 3) for t in xyzs]).contiguous()
    f = torch.empty(sum(n), dtype=torch.float32, device=dev)
    g = torch.empty(sum(n), 3, dtype=torch.float32, device=dev)
    a = torch.empty(sum(n), dtype=torch.float32, device=dev)
    ws = _ws(lib().rfvr_mlp_forward_grouped_ws_bytes(len(nets), arr, cnt), dev)
    _check(lib().rfvr_mlp_forward_grouped(len(nets), arr, _ptr(x), cnt, _ptr(f), _ptr(g), _ptr(a), _ptr(ws),
                                          ws.numel(), _stream(stream)), "rfvr_mlp_forward_grouped")
    return list(zip(_split(f, n), _split(g, n), _split(a, n)))


def mlp_backward_grouped(nets, xyzs, g_sdfs, g_grads, g_refls, flags: int = 0, stream=None):
    """Parameter gradients of several networks: list of flat tensors."""
    dev = xyzs[0].device
    arr, cnt = _nets(nets, xyzs)
    x = torch.cat([t.reshape(-1, 3) for t in xyzs]).contiguous()
    cat = lambda ts, w: torch.cat([t.reshape(-1, w) for t in ts]).contiguous()
    gf, gg, ga = cat(g_sdfs, 1), cat(g_grads, 3), cat(g_refls, 1)
    counts = [net.param_count() for net in nets]
    gp = torch.empty(sum(counts), dtype=torch.float32, device=dev)
    ws = _ws(lib().rfvr_mlp_backward_grouped_ws_bytes(len(nets), arr, cnt), dev)
    _check(lib().rfvr_mlp_backward_grouped(len(nets), arr, _ptr(x), cnt, _ptr(gf), _ptr(gg), _ptr(ga), flags,
                                           _ptr(gp), _ptr(ws), ws.numel(), _stream(stream)),
           "rfvr_mlp_backward_grouped")
    return _split(gp, counts)


def term_order(ap: Aperture, xyz: torch.Tensor, stream=None) -> int:
    """Order K of the Chebyshev-moment evaluation the term calls choose for
    these measurements and points (0: per-frequency kernels).  Synchronises."""
    dev = xyz.device
    n = xyz.numel() // 3
    cap = ap.c()
    ws = _ws(lib().rfvr_term_order_ws_bytes(ctypes.byref(cap), n), dev)
    out = torch.zeros(1, dtype=torch.int32, device=dev)
    _check(lib().rfvr_term_order(ctypes.byref(cap), _ptr(xyz.contiguous()), n, _ptr(out), _ptr(ws), ws.numel(),
                                 _stream(stream)), "rfvr_term_order")
    return int(out.item())


def occupancy(s, sdf: torch.Tensor, stream=None):
    """Phi = sigmoid(s * sdf) (detached origin occupancies); s a float, or a
    device tensor [1] holding log s (rfvr_occupancy_logs)."""
    phi = torch.empty_like(sdf)
    if isinstance(s, torch.Tensor):
        _check(lib().rfvr_occupancy_logs(sdf.numel(), _ptr(s), _ptr(sdf.contiguous()), _ptr(phi), _stream(stream)),
               "rfvr_occupancy_logs")
    else:
        _check(lib().rfvr_occupancy(sdf.numel(), float(s), _ptr(sdf.contiguous()), _ptr(phi), _stream(stream)),
               "rfvr_occupancy")
    return phi


def adamw(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8, wd=0.0, stream=None):
    _check(lib().rfvr_adamw(p.numel(), _ptr(p), _ptr(g), _ptr(m), _ptr(v), int(t), float(lr),
                            float(b1), float(b2), float(eps), float(wd), _stream(stream)),
           "rfvr_adamw")


def sample_naive(centre, half_extent, primary_dir, n_ray_x, n_ray_y, n_z, tx: torch.Tensor, stream=None):
    """Per-antenna samples: (xyz [n_ant, n_ray, n_z, 3], jac [n_ant, n_ray, n_z])."""
    n_ant = tx.shape[0]
    d = _sample_desc(centre, half_extent, primary_dir, n_ray_x, n_ray_y, n_z, 0, 0, 0)
    n_ray = n_ray_x * n_ray_y
    xyz = torch.empty(n_ant, n_ray, n_z, 3, dtype=torch.float32, device=tx.device)
    jac = torch.empty(n_ant, n_ray, n_z, dtype=torch.float32, device=tx.device)
    _check(lib().rfvr_sample_naive(ctypes.byref(d), _ptr(tx.contiguous()), int(n_ant), _ptr(xyz), _ptr(jac),
                                   _stream(stream)), "rfvr_sample_naive")
    return xyz, jac


def sample_importance(centre, half_extent, primary_dir, n_ray_x, n_ray_y, logits: torch.Tensor,
                      n_imp, n_uni, seed=0, step=0, plane_offset=0.0, stream=None, jitter=True):
    """Proposal-guided depths: (xyz [n_ray, K, 3], u [n_ray, K], ray_origin [n_ray, 3]),
    K = n_uni + n_imp, from bin logits [n_ray, n_bins]; jitter=False puts every
    slot at the middle of its stratum."""
    n_ray = n_ray_x * n_ray_y
    n_bins = logits.shape[-1]
    assert logits.numel() == n_ray * n_bins
    d = _sample_desc(centre, half_extent, primary_dir, n_ray_x, n_ray_y, n_imp + n_uni,
                     SAMPLE_STRATIFIED if jitter else SAMPLE_GRID, seed, step, plane_offset)
    dev = logits.device
    K = n_imp + n_uni
    xyz = torch.empty(n_ray, K, 3, dtype=torch.float32, device=dev)
    u = torch.empty(n_ray, K, dtype=torch.float32, device=dev)
    o = torch.empty(n_ray, 3, dtype=torch.float32, device=dev)
    _check(lib().rfvr_sample_importance(ctypes.byref(d), _ptr(logits.contiguous()), int(n_bins), int(n_imp),
                                        int(n_uni), _ptr(xyz), _ptr(u), _ptr(o), _stream(stream)),
           "rfvr_sample_importance")
    return xyz, u, o


@dataclass
class Proposal:
    params: torch.Tensor
    pe_octaves: int = 4
    width: int = 64
    layers: int = 2
    centre: tuple = (0.0, 0.0, 0.28)
    half_size: float = 0.10

    def c(self, params: Optional[torch.Tensor] = None) -> CProposal:
        p = self.params if params is None else params
        return CProposal(self.pe_octaves, self.width, self.layers,
                         (_c_f * 3)(*[float(c) for c in self.centre]), float(self.half_size), _ptr(p))

    def param_count(self) -> int:
        return int(lib().rfvr_proposal_param_count(ctypes.byref(self.c())))


def proposal_forward(net: Proposal, xyz: torch.Tensor, stream=None):
    """logits [N] at xyz [N, 3]."""
    dev = xyz.device
    n = xyz.numel() // 3
    cn = net.c()
    z = torch.empty(n, dtype=torch.float32, device=dev)
    ws = _ws(lib().rfvr_proposal_ws_bytes(ctypes.byref(cn), n), dev)
    _check(lib().rfvr_proposal_forward(ctypes.byref(cn), _ptr(xyz.contiguous()), n, _ptr(z), _ptr(ws),
                                       ws.numel(), _stream(stream)), "rfvr_proposal_forward")
    return z


def proposal_backward(net: Proposal, xyz: torch.Tensor, g_logits: torch.Tensor, flags=0, out=None,
                      stream=None):
    dev = xyz.device
    n = xyz.numel() // 3
    cn = net.c()
    gp = out if out is not None else torch.empty(net.param_count(), dtype=torch.float32, device=dev)
    ws = _ws(lib().rfvr_proposal_ws_bytes(ctypes.byref(cn), n), dev)
    _check(lib().rfvr_proposal_backward(ctypes.byref(cn), _ptr(xyz.contiguous()), n,
                                        _ptr(g_logits.contiguous()), flags, _ptr(gp), _ptr(ws), ws.numel(),
                                        _stream(stream)), "rfvr_proposal_backward")
    return gp


def proposal_targets(u: torch.Tensor, alpha: torch.Tensor, trans: torch.Tensor, lo: float, hi: float,
                     n_bins: int, dilate: int = 0, stream=None):
    """Binned, max-normalised blend weights [n_ray, n_bins] of the render at depths u [n_ray, n_k],
    dilated in depth over `dilate` bins."""
    n_ray, n_k = u.shape
    t = torch.empty(n_ray, n_bins, dtype=torch.float32, device=u.device)
    _check(lib().rfvr_proposal_targets(n_ray, n_k, _ptr(u.contiguous()), _ptr(alpha.contiguous()),
                                       _ptr(trans.contiguous()), float(lo), float(hi), int(n_bins), int(dilate),
                                       _ptr(t), _stream(stream)), "rfvr_proposal_targets")
    return t


def bce(logits: torch.Tensor, t: torch.Tensor, want_grad=True, stream=None):
    """(loss [1], g_logits) of the mean binary cross-entropy of sigmoid(logits) vs t."""
    n = logits.numel()
    loss = torch.empty(1, dtype=torch.float32, device=logits.device)
    g = torch.empty_like(logits) if want_grad else None
    ws = _ws(lib().rfvr_bce_ws_bytes(n), logits.device)
    _check(lib().rfvr_bce(n, _ptr(logits.contiguous()), _ptr(t.contiguous()), _ptr(loss), _ptr(g), _ptr(ws),
                          ws.numel(), _stream(stream)), "rfvr_bce")
    return loss, g


def mask_update(power: torch.Tensor, power_ref: torch.Tensor, history: torch.Tensor, tau_hi: float = 0.25,
                tau_lo: float = 0.25, out=None, stream=None):
    """Dynamic loss mask [n] (1 keep, 0 drop); updates history in place."""
    n = power.numel()
    mask = out if out is not None else torch.empty_like(power)
    ws = _ws(lib().rfvr_mask_ws_bytes(n), power.device)
    _check(lib().rfvr_mask_update(n, _ptr(power.contiguous()), _ptr(power_ref.contiguous()), _ptr(history),
                                  float(tau_hi), float(tau_lo), _ptr(mask), _ptr(ws), ws.numel(),
                                  _stream(stream)), "rfvr_mask_update")
    return mask


# C-ABI names
rfvr_render_forward = render_forward
rfvr_render_backward = render_backward
rfvr_mf_forward = mf_forward
rfvr_mf_backward = mf_backward
rfvr_loss_l2 = loss_l2
rfvr_sample_points = sample_points
rfvr_mlp_forward = mlp_forward
rfvr_mlp_backward = mlp_backward
rfvr_mlp_reserve_bytes = mlp_reserve


def rfvr_mlp_forward_train(net: MLP, xyz: torch.Tensor, reserve: torch.Tensor, stream=None):
    return mlp_forward(net, xyz, stream=stream, reserve=reserve)


def rfvr_mlp_backward_train(net: MLP, xyz: torch.Tensor, g_sdf, g_grad, g_refl, reserve: torch.Tensor,
                            flags=0, out=None, stream=None):
    return mlp_backward(net, xyz, g_sdf, g_grad, g_refl, flags=flags, out=out, stream=stream, reserve=reserve)


rfvr_adamw = adamw
rfvr_occupancy = occupancy
rfvr_proposal_forward = proposal_forward
rfvr_proposal_backward = proposal_backward
rfvr_sample_importance = sample_importance
rfvr_sample_naive = sample_naive
rfvr_proposal_targets = proposal_targets
rfvr_bce = bce
rfvr_mask_update = mask_update
rfvr_term_order = term_order
