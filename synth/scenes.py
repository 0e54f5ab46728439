"""Synthetic radar scenes: apertures, frequency grids, point sets, analytic SDFs.

Conventions
-----------
* Antennas of a planar aperture sit in the plane z = ``z`` at
  ``((ix - (nx-1)/2) * pitch, (iy - (ny-1)/2) * pitch, z)`` with flat index
  ``i = iy * nx + ix`` (x fastest).
* Frequencies are linearly spaced and inclusive of both ends, like
  ``numpy.linspace(f_lo, f_hi, n)``: ``f_n = f0 + n * df``.
* Point sets are laid out ``[n_line, n_z, 3]`` along lines parallel to +z,
  with depth increasing along the second axis.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np


def planar_aperture(nx: int, ny: int, pitch: float, z: float = 0.0,
                    centre_xy: Tuple[float, float] = (0.0, 0.0)) -> np.ndarray:
    """Monostatic planar array, float32 [nx*ny, 3], index i = iy*nx + ix."""
    ix = (np.arange(nx) - (nx - 1) / 2.0) * pitch + centre_xy[0]
    iy = (np.arange(ny) - (ny - 1) / 2.0) * pitch + centre_xy[1]
    gx, gy = np.meshgrid(ix, iy, indexing="xy")  # gy varies along axis 0
    pos = np.stack([gx.ravel(), gy.ravel(), np.full(nx * ny, z)], axis=1)
    return np.ascontiguousarray(pos, dtype=np.float32)


def ring_apertures(n_planes: int, distance: float, nx: int, ny: int, pitch: float,
                   centre: Sequence[float] = (0.0, 0.0, 0.30), first: float = 0.0,
                   span: float = 2.0 * np.pi):
    """Scanning planes on a ring around a vertical (y) axis through ``centre``.

    Plane k sits at azimuth phi_k = first + span * k / n_planes, its centre at
    centre + distance * (sin phi, 0, -cos phi), facing the centre: unit primary
    direction w = (-sin phi, 0, cos phi).  Its antennas form an nx x ny grid of
    pitch ``pitch`` along e_x = (cos phi, 0, sin phi) and e_y = (0, 1, 0), index
    i = iy * nx + ix.  Plane 0 with centre (0, 0, d) is the standard aperture in
    z = 0.  Returns a list of dicts: tx float32 [nx*ny, 3], w float64 [3],
    offset = plane centre . w (the plane is {x : x . w = offset})."""
    c = np.asarray(centre, np.float64)
    out = []
    for k in range(n_planes):
        phi = first + span * k / n_planes
        w = np.array([-np.sin(phi), 0.0, np.cos(phi)])
        ex = np.array([np.cos(phi), 0.0, np.sin(phi)])
        ey = np.array([0.0, 1.0, 0.0])
        pc = c - distance * w
        ix = (np.arange(nx) - (nx - 1) / 2.0) * pitch
        iy = (np.arange(ny) - (ny - 1) / 2.0) * pitch
        gx, gy = np.meshgrid(ix, iy, indexing="xy")
        tx = pc[None] + gx.ravel()[:, None] * ex[None] + gy.ravel()[:, None] * ey[None]
        out.append({"tx": np.ascontiguousarray(tx, np.float32), "w": w, "offset": float(pc @ w)})
    return out


def freq_grid(n_freq: int, f_lo: float = 77e9, f_hi: float = 81e9) -> Tuple[float, float]:
    """(f0, df) of an inclusive linear grid of ``n_freq`` frequencies."""
    if n_freq < 1:
        raise ValueError("n_freq must be >= 1")
    df = 0.0 if n_freq == 1 else (f_hi - f_lo) / (n_freq - 1)
    return float(f_lo), float(df)


def line_points(centre: Sequence[float], side: float, n_lx: int, n_ly: int, n_z: int,
                jitter_seed: int | None = None) -> Tuple[np.ndarray, np.ndarray]:
    """Points on lines parallel to +z through a cube.

    Lines pass through the centres of an ``n_lx x n_ly`` lateral grid over the
    cube's cross-section; depths are cell centres of ``n_z`` equal slices, or,
    with ``jitter_seed``, one uniform draw inside each slice (still sorted).
    Returns ``xyz`` float32 [n_lx*n_ly, n_z, 3] and the lines' crossing points
    with the plane z = 0, float32 [n_lx*n_ly, 3].
    """
    cx, cy, cz = (float(c) for c in centre)
    h = side / 2.0
    lx = cx - h + (np.arange(n_lx) + 0.5) * side / n_lx
    ly = cy - h + (np.arange(n_ly) + 0.5) * side / n_ly
    gx, gy = np.meshgrid(lx, ly, indexing="xy")
    n_line = n_lx * n_ly
    if jitter_seed is None:
        frac = np.broadcast_to(np.full(n_z, 0.5), (n_line, n_z))
    else:
        frac = np.random.default_rng(jitter_seed).random((n_line, n_z))
    z = cz - h + (np.arange(n_z)[None, :] + frac) * side / n_z
    xyz = np.empty((n_line, n_z, 3), dtype=np.float64)
    xyz[:, :, 0] = gx.ravel()[:, None]
    xyz[:, :, 1] = gy.ravel()[:, None]
    xyz[:, :, 2] = z
    origin = np.stack([gx.ravel(), gy.ravel(), np.zeros(n_line)], axis=1)
    return (np.ascontiguousarray(xyz, dtype=np.float32),
            np.ascontiguousarray(origin, dtype=np.float32))


# ----------------------------------------------------------------------------
# Analytic signed-distance primitives (float64).  ``eval(x)`` takes [..., 3]
# and returns (sdf [...], grad [..., 3]).
# ----------------------------------------------------------------------------

@dataclass
class Sphere:
    centre: Sequence[float]
    radius: float
    refl: float = 0.8

    def eval(self, x):
        d = np.asarray(x, np.float64) - np.asarray(self.centre, np.float64)
        n = np.linalg.norm(d, axis=-1)
        safe = np.maximum(n, 1e-300)
        return n - self.radius, d / safe[..., None]


@dataclass
class Box:
    centre: Sequence[float]
    half: Sequence[float]          # half side lengths (x, y, z)
    refl: float = 0.8

    def eval(self, x):
        d = np.asarray(x, np.float64) - np.asarray(self.centre, np.float64)
        q = np.abs(d) - np.asarray(self.half, np.float64)
        qp = np.maximum(q, 0.0)
        out_n = np.linalg.norm(qp, axis=-1)
        qmax = q.max(axis=-1)
        sdf = out_n + np.minimum(qmax, 0.0)
        sgn = np.where(d >= 0, 1.0, -1.0)
        g_out = qp / np.maximum(out_n, 1e-300)[..., None] * sgn
        axis = q.argmax(axis=-1)
        g_in = np.zeros_like(d)
        np.put_along_axis(g_in, axis[..., None], np.take_along_axis(sgn, axis[..., None], -1), -1)
        grad = np.where((out_n > 0)[..., None], g_out, g_in)
        return sdf, grad


@dataclass
class Torus:
    centre: Sequence[float]
    major: float                   # R
    minor: float                   # r ; axis is +z
    refl: float = 0.8

    def eval(self, x):
        d = np.asarray(x, np.float64) - np.asarray(self.centre, np.float64)
        rho = np.hypot(d[..., 0], d[..., 1])
        a = rho - self.major
        n = np.hypot(a, d[..., 2])
        sdf = n - self.minor
        safe_rho = np.maximum(rho, 1e-300)
        safe_n = np.maximum(n, 1e-300)
        g = np.empty_like(d)
        g[..., 0] = a / safe_n * d[..., 0] / safe_rho
        g[..., 1] = a / safe_n * d[..., 1] / safe_rho
        g[..., 2] = d[..., 2] / safe_n
        return sdf, g


@dataclass
class Slab:
    z0: float                      # mid-plane
    half_thickness: float
    refl: float = 0.1

    def eval(self, x):
        x = np.asarray(x, np.float64)
        dz = x[..., 2] - self.z0
        sdf = np.abs(dz) - self.half_thickness
        g = np.zeros_like(x)
        g[..., 2] = np.where(dz >= 0, 1.0, -1.0)
        return sdf, g


@dataclass
class Union:
    parts: List = field(default_factory=list)

    def eval(self, x):
        vals = [p.eval(x) for p in self.parts]
        sdfs = np.stack([v[0] for v in vals], axis=0)
        k = sdfs.argmin(axis=0)
        sdf = np.take_along_axis(sdfs, k[None], 0)[0]
        grads = np.stack([v[1] for v in vals], axis=0)
        grad = np.take_along_axis(grads, k[None, ..., None], 0)[0]
        return sdf, grad

    def refl_at(self, x):
        sdfs = np.stack([p.eval(x)[0] for p in self.parts], axis=0)
        refls = np.asarray([p.refl for p in self.parts])
        return refls[sdfs.argmin(axis=0)]


def scene_fields(scene, xyz: np.ndarray, chunk: int = 1 << 16):
    """(sdf, grad, refl) of an analytic scene at points ``xyz`` as float32.

    Evaluated in chunks of ``chunk`` points (every operation is per point, so
    the values do not depend on the chunking; small chunks keep the float64
    temporaries in cache, which matters at millions of points)."""
    xyz = np.asarray(xyz)
    shp = xyz.shape[:-1]
    flat = xyz.reshape(-1, 3)
    n = flat.shape[0]
    sdf = np.empty(n, np.float32)
    grad = np.empty((n, 3), np.float32)
    refl = np.empty(n, np.float32)
    for a in range(0, n, chunk):
        x = np.asarray(flat[a:a + chunk], np.float64)
        f, g = scene.eval(x)
        sdf[a:a + chunk] = f
        grad[a:a + chunk] = g
        refl[a:a + chunk] = scene.refl_at(x) if isinstance(scene, Union) else scene.refl
    return sdf.reshape(shp), grad.reshape(shp + (3,)), refl.reshape(shp)


def complex_noise(clean: np.ndarray, snr_db: float, seed: int) -> np.ndarray:
    """Circular complex Gaussian noise with mean |n|^2 = mean |clean|^2 / 10^(snr/10)."""
    p = float(np.mean(np.abs(clean) ** 2))
    var = p / (10.0 ** (snr_db / 10.0))
    rng = np.random.default_rng(seed)
    sd = np.sqrt(var / 2.0)
    n = rng.normal(0.0, sd, clean.shape) + 1j * rng.normal(0.0, sd, clean.shape)
    return n.astype(np.complex128)


def random_union_scene(seed: int, cube_centre: Sequence[float]) -> Union:
    """Seeded union of 1-3 primitives inside a 25 cm cube (large batched workload)."""
    rng = np.random.default_rng(seed)
    c = np.asarray(cube_centre, np.float64)
    parts = []
    for _ in range(int(rng.integers(1, 4))):
        kind = int(rng.integers(0, 3))
        off = rng.uniform(-0.05, 0.05, 3)
        if kind == 0:
            parts.append(Sphere(c + off, float(rng.uniform(0.02, 0.05)), 0.8))
        elif kind == 1:
            parts.append(Box(c + off, rng.uniform(0.015, 0.05, 3), 0.8))
        else:
            parts.append(Torus(c + off, float(rng.uniform(0.03, 0.06)),
                               float(rng.uniform(0.005, 0.015)), 0.8))
    return Union(parts)
