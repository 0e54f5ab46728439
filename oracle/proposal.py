"""Oracle of the learned proposal sampler (float64 numpy / torch).

TEST INFRASTRUCTURE ONLY.

The paper samples full space uniformly along its primary rays (Sec. Lensless
Sampling).  The proposal sampler concentrates those samples where the method's
own blend weights are: a small ReLU network predicts an occupancy logit z_b
at the centres of n_bins uniform depth bins of every primary ray; the depth
pdf is p_b = (sigmoid(z_b) + 1e-3) / sum_b' (sigmoid(z_b') + 1e-3); n_imp
depths are drawn by inverse-CDF sampling at stratified levels
v_k = (k + xi_k) / n_imp, and n_uni depths stratified uniformly over the whole
range keep coverage (the uniform fallback).  All depths of a ray are sorted
ascending (ties: uniform slots first, then by slot index).  Slot s of ray r
draws xi from the counter-based SplitMix64 stream of the step with counter
r * (n_uni + n_imp) + s; slots 0..n_uni-1 are the uniform ones.

Training signal: the render's blend weights w_k = T_k alpha_k at the sampled
depths.  w_k is the opacity of the segment [u_k, u_{k+1}] that alpha_k covers,
so it is spread over the bins that segment overlaps, in proportion to the
overlap (reading: with sparse samples a long segment says only that the
surface lies somewhere inside it; the last sample, or a segment of zero length,
goes to the bin of u_k).  The per-bin sums W_b are normalised per ray,
t_b = min(1, W_b / max(max_b W_b, 1e-3)), optionally dilated in depth (each
bin takes the largest t of itself and the `dilate` bins in front of it, so that
samples continue into an object behind its front surface; an option of this
implementation, not in the paper), and the mean binary cross-entropy between
sigmoid(z_b) and t_b is the loss.

Network: gamma_4(x_hat) (27 values) -> Linear(64) -> relu -> Linear(64) -> relu
-> Linear(1); flat layout W0 [64][27], b0 [64], W1 [64][64], b1 [64],
w_out [64], b_out [1] (``synth.proposal_layout``).
"""
from __future__ import annotations

import numpy as np
import torch

from synth.mlp_init import proposal_layout
from .mlp import positional_encoding
from .sampling import lateral_basis, uniform24

PDF_FLOOR = 1e-3
TARGET_FLOOR = 1e-3


def _unflatten(params, spec):
    lay = proposal_layout(spec)
    return {k: params[o:o + int(np.prod(s))].view(*s) for k, (o, s) in lay.items() if not k.startswith("__")}


def network(params: torch.Tensor, spec, xyz: torch.Tensor) -> torch.Tensor:
    P = _unflatten(params, spec)
    c = torch.tensor(spec.centre, dtype=xyz.dtype)
    h = positional_encoding((xyz - c) / spec.half_size, spec.pe_octaves)
    for l in range(spec.layers):
        h = torch.relu(h @ P[f"W{l}"].T + P[f"b{l}"])
    return h @ P["w_out"] + P["b_out"][0]


def forward(params, spec, xyz):
    p = torch.tensor(np.asarray(params, np.float64))
    x = torch.tensor(np.asarray(xyz, np.float64).reshape(-1, 3))
    return network(p, spec, x).numpy()


def backward(params, spec, xyz, g_logit):
    p = torch.tensor(np.asarray(params, np.float64), requires_grad=True)
    x = torch.tensor(np.asarray(xyz, np.float64).reshape(-1, 3))
    z = network(p, spec, x)
    (g,) = torch.autograd.grad((z * torch.tensor(np.asarray(g_logit, np.float64))).sum(), p)
    return g.numpy()


def bin_centres(centre, half_extent, w_p, n_rx, n_ry, n_bins):
    """Points at the bin centres of every primary ray: [n_ray, n_bins, 3], lo, hi."""
    c = np.asarray(centre, np.float64)
    e1, e2, w = lateral_basis(w_p)
    h = float(half_extent)
    ax = -h + (np.arange(n_rx) + 0.5) * 2 * h / n_rx
    ay = -h + (np.arange(n_ry) + 0.5) * 2 * h / n_ry
    gx, gy = np.meshgrid(ax, ay, indexing="xy")
    origin = (c - np.dot(c, w) * w)[None] + gx.ravel()[:, None] * e1 + gy.ravel()[:, None] * e2
    lo, hi = np.dot(c, w) - h, np.dot(c, w) + h
    u = lo + (np.arange(n_bins) + 0.5) * (hi - lo) / n_bins
    xyz = origin[:, None, :] + u[None, :, None] * w[None, None, :]
    return xyz, origin, lo, hi


def importance_depths(logits, lo, hi, n_imp, n_uni, seed, step, jitter=True):
    """Sorted depths [n_ray, n_uni + n_imp] and their slot of origin; without
    jitter every slot takes xi = 1/2, the middle of its stratum."""
    z = np.asarray(logits, np.float64)
    n_ray, n_bins = z.shape
    sig = 1.0 / (1.0 + np.exp(-z))
    p = sig + PDF_FLOOR
    p = p / p.sum(1, keepdims=True)
    cdf = np.cumsum(p, 1)
    K = n_uni + n_imp
    cnt = (np.arange(n_ray, dtype=np.uint64)[:, None] * np.uint64(K) + np.arange(K, dtype=np.uint64)[None])
    xi = uniform24(seed, step, cnt) if jitter else np.full(cnt.shape, 0.5)   # [n_ray, K]
    delta = (hi - lo) / n_bins
    u = np.empty((n_ray, K))
    # uniform slots
    ku = np.arange(n_uni)
    u[:, :n_uni] = lo + (ku[None] + xi[:, :n_uni]) * (hi - lo) / n_uni
    # importance slots: inverse CDF at stratified levels
    ki = np.arange(n_imp)
    v = (ki[None] + xi[:, n_uni:]) / n_imp                      # [n_ray, n_imp]
    for r in range(n_ray):
        b = np.minimum(np.searchsorted(cdf[r], v[r], side="right"), n_bins - 1)
        prev = np.where(b > 0, cdf[r][np.maximum(b - 1, 0)], 0.0)
        frac = np.clip((v[r] - prev) / p[r][b], 0.0, 1.0)
        u[r, n_uni:] = lo + (b + frac) * delta
    slot = np.broadcast_to(np.arange(K), u.shape)
    order = np.argsort(u, axis=1, kind="stable")                # ties keep slot order
    return np.take_along_axis(u, order, 1), np.take_along_axis(slot, order, 1)


def bin_of(u, lo, hi, n_bins):
    """Index of the equal depth bin of [lo, hi] holding depth u (clamped)."""
    u = np.asarray(u, np.float64)
    return np.clip(np.floor((u - lo) / (hi - lo) * n_bins).astype(np.int64), 0, n_bins - 1)


def bin_weights(u, w, lo, hi, n_bins):
    """W[r, b]: each blend weight w[r, k] spread over the bins that its segment
    [u[r, k], u[r, k+1]] overlaps, in proportion to the overlap; the last
    sample and zero-length segments put theirs in the bin of u[r, k]."""
    u = np.asarray(u, np.float64)
    w = np.asarray(w, np.float64)
    n_ray, n_k = u.shape
    edges = lo + (hi - lo) * np.arange(n_bins + 1) / n_bins
    W = np.zeros((n_ray, n_bins))
    for r in range(n_ray):
        for k in range(n_k):
            a = u[r, k]
            e = u[r, k + 1] if k + 1 < n_k else a
            if e > a:
                ov = np.clip(np.minimum(e, edges[1:]) - np.maximum(a, edges[:-1]), 0.0, None)
                W[r] += w[r, k] * ov / (e - a)
            else:
                W[r, bin_of(a, lo, hi, n_bins)] += w[r, k]
    return W


def targets(W, dilate=0):
    """t_b = min(1, W_b / max(max_b W_b, floor)), then the largest of t over
    the bin and the `dilate` bins in front of it (depth dilation)."""
    W = np.asarray(W, np.float64)
    t = np.minimum(1.0, W / np.maximum(W.max(1, keepdims=True), TARGET_FLOOR))
    out = t.copy()
    for d in range(1, dilate + 1):
        out[:, d:] = np.maximum(out[:, d:], t[:, :-d])
    return out


def bce(logits, t):
    """Mean binary cross-entropy of sigmoid(z) against t, and its gradient."""
    z = np.asarray(logits, np.float64).ravel()
    t = np.asarray(t, np.float64).ravel()
    # log sigmoid(z) = -softplus(-z), log(1 - sigmoid(z)) = -softplus(z)
    sp = lambda x: np.maximum(x, 0) + np.log1p(np.exp(-np.abs(x)))
    L = np.mean(t * sp(-z) + (1 - t) * sp(z))
    g = (1.0 / (1.0 + np.exp(-z)) - t) / z.size
    return float(L), g
