"""The study's surface extraction and Chamfer distance (bench.py) on analytic
shapes: zero crossings of a sphere's SDF on a grid lie on the sphere, and the
Chamfer distance of two concentric spheres is their radius difference."""
import numpy as np

import bench
from synth import Sphere


def test_surface_points_lie_on_the_sphere():
    c, h, n = (0.01, -0.02, 0.30), 0.08, 96
    x = bench.grid_points(c, h, n)
    f, _ = Sphere(c, 0.05).eval(x.astype(np.float64))
    pts = bench.surface_points(f.reshape(n, n, n), c, h)
    r = np.linalg.norm(pts - np.asarray(c), axis=1)
    cell = 2 * h / n
    assert len(pts) > 1000
    # linear interpolation of a smooth SDF: error of order cell^2 / R
    assert np.abs(r - 0.05).max() < 0.2 * cell ** 2 / 0.05 + 1e-9
    # grid order of the axes: a point from each side of the sphere along x
    assert pts[:, 0].min() < c[0] - 0.049 and pts[:, 0].max() > c[0] + 0.049


def test_chamfer_of_concentric_spheres():
    c, h, n = (0.0, 0.0, 0.3), 0.075, 128
    x = bench.grid_points(c, h, n).astype(np.float64)
    a = bench.surface_points(Sphere(c, 0.05).eval(x)[0].reshape(n, n, n), c, h)
    b = bench.surface_points(Sphere(c, 0.06).eval(x)[0].reshape(n, n, n), c, h)
    cd2, cd = bench.chamfer(a, b)
    # 5000 samples on a 5 cm sphere are ~2.5 mm apart: the nearest sample on
    # the other sphere sits up to ~1.3 mm to the side, a few 1e-4 m over 1 cm
    assert abs(cd - 0.01) < 3e-4, cd
    assert abs(cd2 - 2 * 0.01 ** 2) < 1.5e-5, cd2
    assert bench.chamfer(a[:3000], a[:3000])[1] == 0.0        # whole sets, no subsampling
