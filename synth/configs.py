"""The five synthetic workloads, as concrete numbers.

``small_sphere``      8x8 aperture, 32 freqs, 16^3 points in a 10 cm cube, sphere
                      R = 3 cm at 0.30 m (+-5 mm seeded jitter), s = 64, a = 0.8.
``mlp_box``           32x32 aperture, 128 freqs, 2^20 points (64x64 lines x 256
                      depths) in a 20 cm cube, 8x256 softplus MLP on a 6-octave
                      encoding, 2x64 head; target: box 8x6x4 cm + 10 dB noise.
``mlp_box_bf16``      the same with a BF16 MLP (precision study).
``proposal_torus``    the same aperture; torus R=4 cm r=1 cm at 0.30 m behind a
                      1 cm slab (a = 0.1) at 0.20 m; 64x64 lines x (16 importance
                      + 4 uniform) points vs 2^20 uniform.
``batched8``          8 scenes, apertures 32x32 .. 64x64, 256 freqs, 2^22 points
                      per scene (128x128 lines x 256), seeded unions of 1-3
                      primitives in a 25 cm cube at 0.25-0.40 m, SNR 5-20 dB.
"""
from __future__ import annotations

import numpy as np

PITCH = 2e-3
F_LO, F_HI = 77e9, 81e9

CONFIGS = {
    "small_sphere": dict(
        ap=(8, 8), n_freq=32, cube_centre=(0.0, 0.0, 0.30), cube_side=0.10,
        lines=(16, 16), n_z=16, sphere_radius=0.03, jitter_mm=5.0,
        s=64.0, refl=0.8, amp=1.0, mlp=None),
    "mlp_box": dict(
        ap=(32, 32), n_freq=128, cube_centre=(0.0, 0.0, 0.30), cube_side=0.20,
        lines=(64, 64), n_z=256, box_half=(0.04, 0.03, 0.02), box_refl=0.8,
        snr_db=10.0, s=64.0, amp=1.0,
        mlp=dict(n_layers=8, width=256, pe_octaves=6, head_width=64, head_layers=2,
                 beta=100.0, precision="fp32")),
    "mlp_box_bf16": dict(
        ap=(32, 32), n_freq=128, cube_centre=(0.0, 0.0, 0.30), cube_side=0.20,
        lines=(64, 64), n_z=256, box_half=(0.04, 0.03, 0.02), box_refl=0.8,
        snr_db=10.0, s=64.0, amp=1.0,
        mlp=dict(n_layers=8, width=256, pe_octaves=6, head_width=64, head_layers=2,
                 beta=100.0, precision="bf16")),
    "proposal_torus": dict(
        ap=(32, 32), n_freq=128, cube_centre=(0.0, 0.0, 0.28), cube_side=0.20,
        lines=(64, 64), n_z=256, n_imp=16, n_uni=4, n_bins=64,
        slab=(0.20, 0.005, 0.1), torus=((0.0, 0.0, 0.30), 0.04, 0.01, 0.8),
        s=64.0, amp=1.0, snr_db=10.0,
        mlp=dict(n_layers=8, width=256, pe_octaves=6, head_width=64, head_layers=2,
                 beta=100.0, precision="fp32"),
        proposal=dict(pe_octaves=4, width=64, layers=2)),
    "batched8": dict(
        ap_sides=[int(round(32 + 32 * k / 7)) for k in range(8)], n_freq=256,
        cube_side=0.25, range_lo=0.25, range_hi=0.40, lines=(128, 128), n_z=256,
        n_imp=192, n_uni=64, snr_lo=5.0, snr_hi=20.0, s=64.0, amp=1.0,
        mlp=dict(n_layers=8, width=256, pe_octaves=6, head_width=64, head_layers=2,
                 beta=100.0, precision="bf16")),
}


def config(name: str) -> dict:
    return dict(CONFIGS[name])


def small_sphere_centre(seed: int) -> np.ndarray:
    """Sphere centre of the small parity workload: (0,0,0.30) + U(-5,5) mm per axis."""
    rng = np.random.default_rng(seed)
    return np.array([0.0, 0.0, 0.30]) + rng.uniform(-5e-3, 5e-3, 3)


def batched8_scene(k: int) -> dict:
    """Scene ``k`` (0..7) of the eight-scene workload: aperture side (antennas
    per axis at 2 mm), cube centre on the axis at a seeded range in
    [0.25, 0.40] m, the SNR of its measured signal, and the seed of its union
    of primitives (``synth.scenes.random_union_scene``)."""
    c = CONFIGS["batched8"]
    rng = np.random.default_rng(8000 + k)
    rc = float(rng.uniform(c["range_lo"], c["range_hi"]))
    snr = float(rng.uniform(c["snr_lo"], c["snr_hi"]))
    return dict(side=c["ap_sides"][k], centre=(0.0, 0.0, rc), half=0.5 * c["cube_side"], snr_db=snr, seed=k)
