"""torch.autograd wrappers over the library's forward / adjoint pairs.

Each Function saves only its inputs; backward calls the hand-written adjoint,
which recomputes per-term phases and amplitudes (render, matched filter) or
activations (network) instead of storing them.

    f, grad, a = MLPFn.apply(params, xyz, net)
    sig        = RenderFn.apply(sdf, grad, refl, amp, s, ap, xyz, phi_ray, phi_tx, flags)
    z, p       = MFFn.apply(sig, ap, xyz_q, flags)   (p differentiable)
    loss       = LossFn.apply(p, p_star)
"""
from __future__ import annotations

import torch

from . import rfvr as R


class MLPFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, xyz, net: R.MLP):
        ctx.save_for_backward(params, xyz)
        ctx.net = net
        f, g, a = R.mlp_forward(_with_params(net, params), xyz.contiguous())
        return f, g, a

    @staticmethod
    def backward(ctx, g_f, g_grad, g_a):
        params, xyz = ctx.saved_tensors
        gp = R.mlp_backward(_with_params(ctx.net, params), xyz.contiguous(),
                            None if g_f is None else g_f.contiguous(),
                            None if g_grad is None else g_grad.contiguous(),
                            None if g_a is None else g_a.contiguous())
        return gp, None, None


def _with_params(net: R.MLP, params: torch.Tensor) -> R.MLP:
    return R.MLP(params=params.detach().contiguous(), n_layers=net.n_layers, width=net.width,
                 pe_octaves=net.pe_octaves, head_width=net.head_width, head_layers=net.head_layers,
                 beta=net.beta, centre=net.centre, half_size=net.half_size, precision=net.precision)


class RenderFn(torch.autograd.Function):
    """signal [n_meas, n_freq, 2] from per-point fields [n_ray, n_z(, 3)], A' [1] and s [1]."""

    @staticmethod
    def forward(ctx, sdf, grad, refl, amp, s, ap: R.Aperture, xyz, phi_ray=None, phi_tx=None,
                flags: int = 0):
        ctx.save_for_backward(sdf, grad, refl, amp, s, xyz)
        ctx.ap, ctx.phi_ray, ctx.phi_tx, ctx.flags = ap, phi_ray, phi_tx, flags
        fl = R.Fields(sdf=sdf.detach().contiguous(), grad=grad.detach().contiguous(),
                      refl=refl.detach().contiguous(), s=float(s.item()), amp=1.0,
                      amp_dev=amp.detach().contiguous(), phi_ray=phi_ray, phi_tx=phi_tx)
        return R.render_forward(ap, R.Samples(xyz=xyz.contiguous()), fl, flags=flags)

    @staticmethod
    def backward(ctx, g_sig):
        sdf, grad, refl, amp, s, xyz = ctx.saved_tensors
        fl = R.Fields(sdf=sdf.detach().contiguous(), grad=grad.detach().contiguous(),
                      refl=refl.detach().contiguous(), s=float(s.item()), amp=1.0,
                      amp_dev=amp.detach().contiguous(), phi_ray=ctx.phi_ray, phi_tx=ctx.phi_tx)
        out = R.render_backward(ctx.ap, R.Samples(xyz=xyz.contiguous()), fl, g_sig.contiguous(),
                                flags=ctx.flags)
        return (out["sdf"].view_as(sdf), out["grad"].view_as(grad), out["refl"].view_as(refl),
                out["amp"].view_as(amp), out["s"].view_as(s), None, None, None, None, None)


class MFFn(torch.autograd.Function):
    """(z [Q, 2], p [Q]) = matched filter of signal at xyz_q; only p carries gradient."""

    @staticmethod
    def forward(ctx, signal, ap: R.Aperture, xyz_q, flags: int = 0):
        z, p = R.mf_forward(ap, xyz_q.contiguous(), signal.contiguous(), flags=flags)
        ctx.save_for_backward(xyz_q, z, p)
        ctx.ap, ctx.flags = ap, flags
        ctx.mark_non_differentiable(z)
        return z, p

    @staticmethod
    def backward(ctx, g_z, g_p):
        xyz_q, z, p = ctx.saved_tensors
        g = R.mf_backward(ctx.ap, xyz_q, z, p, g_p.contiguous(), flags=ctx.flags)
        return g, None, None, None


class LossFn(torch.autograd.Function):
    """(1/Q) sum (p - p*)^2 on the library's loss kernel."""

    @staticmethod
    def forward(ctx, p, p_star):
        loss, g = R.loss_l2(p.contiguous(), p_star.contiguous())
        ctx.save_for_backward(g)
        return loss[0]

    @staticmethod
    def backward(ctx, g_loss):
        (g,) = ctx.saved_tensors
        return g * g_loss, None
