"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module only *generates inputs*: antenna grids, frequency grids, point
sets laid out along parallel lines, analytic signed-distance scenes, network
weights and measurement noise.  It holds none of the rendering method's
arithmetic (no transmittance, no phases, no matched filter), so the FP64 CPU
oracle and the HIP library can both consume its outputs without sharing any
of the computation they are compared on.

Every generator is deterministic in its ``seed`` argument (numpy PCG64).
Arrays are returned as C-contiguous float32 unless stated otherwise; the
analytic SDF evaluators work in float64 and the caller rounds.
"""
from .scenes import (  # noqa: F401
    planar_aperture,
    ring_apertures,
    freq_grid,
    line_points,
    Sphere,
    Box,
    Torus,
    Slab,
    Union,
    scene_fields,
    complex_noise,
    random_union_scene,
)
from .mlp_init import mlp_layout, mlp_init, MLPSpec, ProposalSpec, proposal_layout, proposal_init  # noqa: F401
from .configs import CONFIGS, config  # noqa: F401
