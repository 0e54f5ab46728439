"""Oracle of lensless primary-ray sampling (Sec. "Lensless Sampling", Primary Ray).

TEST INFRASTRUCTURE ONLY.

Parallel rays leave the aperture plane (through the origin, normal to the
primary direction w_p) and cross the sampling cube; points are x = o_r + u w_p
with u ascending along each ray.

* Lateral layout: an n_rx x n_ry grid of cell centres over the cube's cross
  section, ray index r = iy * n_rx + ix.  Lateral axes: e1 = unit(y_hat x w_p)
  (x_hat x w_p when w_p is nearly parallel to y_hat), e2 = w_p x e1.
* GRID: u_k = (c.w_p - h) + (k + 1/2) * 2h / n_z.
* STRATIFIED: u_k = (c.w_p - h) + (k + xi_{r,k}) * 2h / n_z, xi drawn from the
  counter-based generator below with counter r * n_z + k.

Counter-based generator: SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014).  Its k-th output (k >= 0) from
state ``seed`` is mix(seed + (k + 1) * GAMMA) with
mix(z) = z3 ^ (z3 >> 31), z1 = (z ^ (z >> 30)) * M1, z2 = (z1 ^ (z1 >> 27)) * M2.
A training step gets its own stream: key = output(seed, step); the draw for
counter c is xi = (output(key, c) >> 40) * 2^-24, uniform on [0, 1).
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)


def _mix(z):
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
    return z ^ (z >> np.uint64(31))


def splitmix64_output(seed, k):
    """k-th (0-based) output of SplitMix64 started from state ``seed``."""
    seed = np.asarray(seed, dtype=np.uint64)
    k = np.asarray(k, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(seed + (k + np.uint64(1)) * GAMMA)


def uniform24(seed: int, step: int, counter) -> np.ndarray:
    key = splitmix64_output(np.uint64(seed), np.uint64(step))
    v = splitmix64_output(key, np.asarray(counter, dtype=np.uint64))
    return (v >> np.uint64(40)).astype(np.float64) * (2.0 ** -24)


def lateral_basis(w_p):
    w = np.asarray(w_p, np.float64)
    w = w / np.linalg.norm(w)
    ref = np.array([0.0, 1.0, 0.0]) if abs(w[1]) < 0.9 else np.array([1.0, 0.0, 0.0])
    e1 = np.cross(ref, w)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(w, e1)
    return e1, e2, w


def sample_points(centre, half_extent, w_p, n_rx, n_ry, n_z, mode="grid", seed=0, step=0, plane_offset=0.0):
    """Returns (xyz [n_ray, n_z, 3], u [n_ray, n_z], ray_origin [n_ray, 3]) in float64.
    The ray origins are the rays' feet on the aperture plane x . w = plane_offset;
    u is measured along w from the parallel plane through the world origin."""
    c = np.asarray(centre, np.float64)
    h = float(half_extent)
    e1, e2, w = lateral_basis(w_p)
    ax = -h + (np.arange(n_rx) + 0.5) * 2.0 * h / n_rx
    ay = -h + (np.arange(n_ry) + 0.5) * 2.0 * h / n_ry
    gx, gy = np.meshgrid(ax, ay, indexing="xy")          # [n_ry, n_rx]
    base = c - np.dot(c, w) * w
    origin = base[None, :] + gx.ravel()[:, None] * e1[None] + gy.ravel()[:, None] * e2[None]
    n_ray = n_rx * n_ry
    if mode == "grid":
        frac = np.full((n_ray, n_z), 0.5)
    elif mode == "stratified":
        cnt = np.arange(n_ray * n_z, dtype=np.uint64).reshape(n_ray, n_z)
        frac = uniform24(seed, step, cnt)
    else:
        raise ValueError(mode)
    u = (np.dot(c, w) - h) + (np.arange(n_z)[None, :] + frac) * (2.0 * h / n_z)
    xyz = origin[:, None, :] + u[:, :, None] * w[None, None, :]
    return xyz, u, origin + float(plane_offset) * w[None, :]


def sample_naive(tx, centre, half_extent, w_p, n_rx, n_ry, n_z):
    """Per-antenna Monte Carlo samples of Sec. Integration (the brute force the
    lensless sampling replaces).  Ray r of antenna i runs from tx_i through the
    r-th cell centre g_r of the lateral grid on the plane through the cube
    centre normal to w; its n_z samples are the cell centres of the ray's
    segment between the planes x . w = c . w -+ h.  jac = (|x - tx_i| / |g_r -
    tx_i|)^2 is the sample's volume relative to a lensless grid cell.
    Returns xyz [n_ant, n_ray, n_z, 3], jac [n_ant, n_ray, n_z] (float64)."""
    c = np.asarray(centre, np.float64)
    h = float(half_extent)
    e1, e2, w = lateral_basis(w_p)
    ax = -h + (np.arange(n_rx) + 0.5) * 2.0 * h / n_rx
    ay = -h + (np.arange(n_ry) + 0.5) * 2.0 * h / n_ry
    gx, gy = np.meshgrid(ax, ay, indexing="xy")
    g = c[None] + gx.ravel()[:, None] * e1[None] + gy.ravel()[:, None] * e2[None]      # [n_ray, 3]
    t = np.asarray(tx, np.float64).reshape(-1, 3)
    d = g[None, :, :] - t[:, None, :]                                                 # [n_ant, n_ray, 3]
    rc = np.linalg.norm(d, axis=-1)
    u = d / rc[..., None]
    cos_w = u @ w
    tw = t @ w
    s_in = (np.dot(c, w) - h - tw)[:, None] / cos_w
    s_out = (np.dot(c, w) + h - tw)[:, None] / cos_w
    dist = s_in[..., None] + (np.arange(n_z) + 0.5)[None, None, :] * ((s_out - s_in) / n_z)[..., None]
    xyz = t[:, None, None, :] + dist[..., None] * u[:, :, None, :]
    return xyz, (dist / rc[..., None]) ** 2
