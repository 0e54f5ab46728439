"""Write the measured signal of the 2^20-point MLP workload with the FP64 oracle.

Scene: analytic box 8 x 6 x 4 cm (a = 0.8) centred at (0, 0, 0.30) m, seen by a
32 x 32 monostatic aperture at 2 mm pitch, 128 frequencies 77-81 GHz, rendered
at the workload's sample grid (64 x 64 lines x 256 depths in a 20 cm cube),
s = 64 / m, A' = 1, clamped specular factor; then circular complex Gaussian
noise at 10 dB SNR (seed 0).  Output: box_target.npz with `clean` and `noisy`
complex128 [1024, 128].  Only the oracle and the seeded generators are used.

With arguments s, "segment" and n_z: the render at that s with the segment
weight (the exact integral of T^2 rho over each segment, placed at its
midpoint) on 64 x 64 lines x n_z depths, written to
box_target_seg_s<S>_nz<n_z>.npz (the proposal study's box scene).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import render as orc  # noqa: E402
from synth import Box, complex_noise, freq_grid, line_points, planar_aperture, scene_fields  # noqa: E402


def main(s=64.0, weight="sample", n_z=256, out=None):
    if out is None:
        out = os.path.join(HERE, "box_target.npz" if weight == "sample" and s == 64.0 and n_z == 256
                           else f"box_target_seg_s{int(s)}_nz{n_z}.npz")
    f0, df = freq_grid(128)
    tx = planar_aperture(32, 32, 2e-3)
    xyz, _ = line_points((0.0, 0.0, 0.30), 0.20, 64, 64, n_z)
    sdf, grad, refl = scene_fields(Box((0.0, 0.0, 0.30), (0.04, 0.03, 0.02), 0.8), xyz)
    ap = orc.Aperture(tx=tx.astype(np.float64), f0=f0, df=df, n_freq=128)
    F = orc.Fields(sdf=sdf.astype(np.float64), grad=grad.astype(np.float64), refl=refl.astype(np.float64),
                   s=s, amp=1.0)
    t0 = time.time()
    clean = orc.render(ap, xyz.astype(np.float64), F, spec="clamp", weight=weight)
    noisy = clean + complex_noise(clean, 10.0, seed=0)
    np.savez(out, clean=clean, noisy=noisy)
    print(f"wrote {out} in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    if len(sys.argv) > 1:
        main(float(sys.argv[1]), sys.argv[2], int(sys.argv[3]))
    else:
        main()
