"""Oracle of the SDF network and its derivatives (torch float64 on the CPU).

TEST INFRASTRUCTURE ONLY.

Network (Sec. "Opaque density representation", App. C Training Setup; sizes of
the 2^20-point MLP workload):
  x_hat = (x - centre) / half_size
  gamma(x_hat) = [x_hat, sin(2^0 pi x_hat), cos(2^0 pi x_hat), ...,
                  sin(2^{L-1} pi x_hat), cos(2^{L-1} pi x_hat)]   (3 + 6L values;
                  each sin/cos block holds the three coordinates)
  h_0 = gamma ; h_l = softplus_beta(W_{l-1} h_{l-1} + b_{l-1}), l = 1..n_layers
  f = half_size * (w_out . h_L + b_out)                  (SDF in metres)
  head: g_0 = h_L ; g_k = relu(Wh_{k-1} g_{k-1} + bh_{k-1}) ; a = sigmoid(wh_out . g + bh_out)
  softplus_beta(z) = log(1 + exp(beta z)) / beta.
The normal is grad_x f (Sec. "Discretization"); it is not detached, so the
parameter gradient of a loss that depends on grad_x f needs second derivatives.
Parameters follow the flat layout of ``synth.mlp_layout``.
"""
from __future__ import annotations

import numpy as np
import torch

from synth.mlp_init import MLPSpec, mlp_layout


def _unflatten(params: torch.Tensor, spec: MLPSpec):
    lay = mlp_layout(spec)
    out = {}
    for name, (off, shape) in lay.items():
        if name.startswith("__"):
            continue
        n = int(np.prod(shape))
        out[name] = params[off:off + n].view(*shape)
    return out


def positional_encoding(xhat: torch.Tensor, octaves: int) -> torch.Tensor:
    feats = [xhat]
    for k in range(octaves):
        feats.append(torch.sin((2.0 ** k) * np.pi * xhat))
        feats.append(torch.cos((2.0 ** k) * np.pi * xhat))
    return torch.cat(feats, dim=-1)


def softplus(z: torch.Tensor, beta: float) -> torch.Tensor:
    bz = beta * z
    return (torch.clamp(bz, min=0) + torch.log1p(torch.exp(-torch.abs(bz)))) / beta


def network(params: torch.Tensor, spec: MLPSpec, xyz: torch.Tensor):
    """(f, a) at points xyz [N, 3]; differentiable in params and xyz."""
    P = _unflatten(params, spec)
    c = torch.tensor(spec.centre, dtype=xyz.dtype)
    h = positional_encoding((xyz - c) / spec.half_size, spec.pe_octaves)
    for l in range(spec.n_layers):
        h = softplus(h @ P[f"W{l}"].T + P[f"b{l}"], spec.beta)
    f = spec.half_size * (h @ P["w_out"] + P["b_out"][0])
    g = h
    for k in range(spec.head_layers):
        g = torch.relu(g @ P[f"Wh{k}"].T + P[f"bh{k}"])
    a = torch.sigmoid(g @ P["wh_out"] + P["bh_out"][0])
    return f, a


def forward(params, spec: MLPSpec, xyz):
    """numpy in/out: (f [N], grad_x f [N, 3], a [N]) in float64."""
    p = torch.tensor(np.asarray(params, np.float64))
    x = torch.tensor(np.asarray(xyz, np.float64).reshape(-1, 3), requires_grad=True)
    f, a = network(p, spec, x)
    (gx,) = torch.autograd.grad(f.sum(), x)
    return f.detach().numpy(), gx.numpy(), a.detach().numpy()


def backward(params, spec: MLPSpec, xyz, g_f, g_grad, g_a):
    """Gradient w.r.t. the flat parameters of
    J = sum_q [ g_f,q f_q + g_grad,q . grad_x f_q + g_a,q a_q ]  (float64 numpy)."""
    p = torch.tensor(np.asarray(params, np.float64), requires_grad=True)
    x = torch.tensor(np.asarray(xyz, np.float64).reshape(-1, 3), requires_grad=True)
    f, a = network(p, spec, x)
    (gx,) = torch.autograd.grad(f.sum(), x, create_graph=True)
    J = (torch.tensor(np.asarray(g_f, np.float64)) * f).sum() \
        + (torch.tensor(np.asarray(g_grad, np.float64).reshape(-1, 3)) * gx).sum() \
        + (torch.tensor(np.asarray(g_a, np.float64)) * a).sum()
    (gp,) = torch.autograd.grad(J, p)
    return gp.numpy()


def objective(params, spec: MLPSpec, xyz, g_f, g_grad, g_a) -> float:
    """The scalar J above (for finite-difference checks)."""
    p = torch.tensor(np.asarray(params, np.float64))
    x = torch.tensor(np.asarray(xyz, np.float64).reshape(-1, 3), requires_grad=True)
    f, a = network(p, spec, x)
    (gx,) = torch.autograd.grad(f.sum(), x)
    J = (torch.tensor(np.asarray(g_f, np.float64)) * f).sum() \
        + (torch.tensor(np.asarray(g_grad, np.float64).reshape(-1, 3)) * gx).sum() \
        + (torch.tensor(np.asarray(g_a, np.float64)) * a).sum()
    return float(J.detach())
