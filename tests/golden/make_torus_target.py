"""Write the measured signal of the proposal-sampler workload with the FP64 oracle.

Scene: torus R = 4 cm, r = 1 cm (axis z, a = 0.8) centred at (0, 0, 0.30) m behind
a 1 cm slab z in [0.195, 0.205] m (a = 0.1), seen by a 32 x 32 monostatic
aperture at 2 mm pitch, 128 frequencies 77-81 GHz, rendered at the full-space
grid of that workload (64 x 64 lines x 256 depths in a 20 cm cube centred at
(0, 0, 0.28) m), s = 64 / m (or the s given as the first argument), A' = 1,
clamped specular factor; then circular complex Gaussian noise at 10 dB SNR
(seed 0).  Output: torus_target.npz (torus_target_s<S>.npz for another s) with
`clean` and `noisy` complex128 [1024, 128].  Only the oracle and the seeded
generators are used.

With a second argument "segment" and a third, the depth count n_z: the render
uses the segment weight (the exact integral of T^2 rho over each segment,
placed at its midpoint) on 64 x 64 lines x n_z depths, written to
torus_target_seg_s<S>_nz<n_z>.npz; with n_z well above the full-space grid's
256 it stands for the continuous integral the sparse renders estimate.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import render as orc  # noqa: E402
from synth import (Slab, Torus, Union, complex_noise, freq_grid, line_points,  # noqa: E402
                   planar_aperture, scene_fields)


def main(s=64.0, out=None, weight="sample", n_z=256):
    if out is None:
        if weight == "segment":
            out = os.path.join(HERE, f"torus_target_seg_s{int(s)}_nz{n_z}.npz")
        else:
            out = os.path.join(HERE, "torus_target.npz" if s == 64.0 else f"torus_target_s{int(s)}.npz")
    f0, df = freq_grid(128)
    tx = planar_aperture(32, 32, 2e-3)
    xyz, _ = line_points((0.0, 0.0, 0.28), 0.20, 64, 64, n_z)
    scene = Union([Slab(0.20, 0.005, 0.1), Torus((0.0, 0.0, 0.30), 0.04, 0.01, 0.8)])
    sdf, grad, refl = scene_fields(scene, xyz)
    ap = orc.Aperture(tx=tx.astype(np.float64), f0=f0, df=df, n_freq=128)
    F = orc.Fields(sdf=sdf.astype(np.float64), grad=grad.astype(np.float64), refl=refl.astype(np.float64),
                   s=s, amp=1.0)
    t0 = time.time()
    clean = orc.render(ap, xyz.astype(np.float64), F, spec="clamp", weight=weight)
    noisy = clean + complex_noise(clean, 10.0, seed=0)
    np.savez(out, clean=clean, noisy=noisy)
    print(f"wrote {out} in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main(float(sys.argv[1]) if len(sys.argv) > 1 else 64.0,
         weight=sys.argv[2] if len(sys.argv) > 2 else "sample",
         n_z=int(sys.argv[3]) if len(sys.argv) > 3 else 256)
