"""Flat parameter layout and seeded initial weights of the SDF network.

Layout of the flat float32 parameter vector (row-major matrices, [out, in]):

    trunk  l = 0 .. n_layers-1 :  W_l [width, in_l]   b_l [width]
                                  (in_0 = 3 + 6 * pe_octaves, in_l = width)
    sdf output                 :  w_out [width]       b_out [1]
    head   h = 0 .. head_layers-1 : Wh_h [head_width, in_h]  bh_h [head_width]
                                  (in_0 = width, in_h = head_width)
    head output                :  wh_out [head_width] bh_out [1]

The weights are a seeded geometric initialisation (normal trunk weights with
variance 2/width, first-layer encoding columns zeroed, output weights centred
on sqrt(pi/width) and output bias -0.5), under which the network starts close
to the signed distance of a sphere of radius 0.5 in normalised coordinates.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, Tuple

import numpy as np


@dataclass(frozen=True)
class MLPSpec:
    n_layers: int = 8
    width: int = 256
    pe_octaves: int = 6
    head_width: int = 64
    head_layers: int = 2
    beta: float = 100.0
    centre: Tuple[float, float, float] = (0.0, 0.0, 0.30)
    half_size: float = 0.10

    @property
    def in_dim(self) -> int:
        return 3 + 6 * self.pe_octaves


def mlp_layout(spec: MLPSpec) -> Dict[str, Tuple[int, Tuple[int, ...]]]:
    """name -> (offset, shape) into the flat parameter vector, in storage order."""
    out = {}
    off = 0

    def add(name, shape):
        nonlocal off
        out[name] = (off, tuple(shape))
        off += int(np.prod(shape))

    for l in range(spec.n_layers):
        fan_in = spec.in_dim if l == 0 else spec.width
        add(f"W{l}", (spec.width, fan_in))
        add(f"b{l}", (spec.width,))
    add("w_out", (spec.width,))
    add("b_out", (1,))
    for h in range(spec.head_layers):
        fan_in = spec.width if h == 0 else spec.head_width
        add(f"Wh{h}", (spec.head_width, fan_in))
        add(f"bh{h}", (spec.head_width,))
    add("wh_out", (spec.head_width,))
    add("bh_out", (1,))
    out["__total__"] = (off, ())
    return out


def mlp_init(spec: MLPSpec, seed: int, sphere_radius: float = 0.5) -> np.ndarray:
    """Seeded geometric initialisation, float32 flat vector."""
    lay = mlp_layout(spec)
    rng = np.random.default_rng(seed)
    p = np.zeros(lay["__total__"][0], dtype=np.float64)

    def put(name, arr):
        off, shape = lay[name]
        p[off:off + int(np.prod(shape))] = np.asarray(arr, np.float64).ravel()

    sd = np.sqrt(2.0) / np.sqrt(spec.width)
    for l in range(spec.n_layers):
        fan_in = spec.in_dim if l == 0 else spec.width
        W = rng.normal(0.0, sd, (spec.width, fan_in))
        if l == 0:
            W[:, 3:] = 0.0
        put(f"W{l}", W)
    put("w_out", rng.normal(np.sqrt(np.pi) / np.sqrt(spec.width), 1e-4, spec.width))
    put("b_out", [-sphere_radius])
    for h in range(spec.head_layers):
        fan_in = spec.width if h == 0 else spec.head_width
        put(f"Wh{h}", rng.normal(0.0, np.sqrt(2.0 / fan_in), (spec.head_width, fan_in)))
    put("wh_out", rng.normal(0.0, np.sqrt(1.0 / spec.head_width), spec.head_width))
    return p.astype(np.float32)


@dataclass(frozen=True)
class ProposalSpec:
    pe_octaves: int = 4
    width: int = 64
    layers: int = 2
    centre: Tuple[float, float, float] = (0.0, 0.0, 0.28)
    half_size: float = 0.10

    @property
    def in_dim(self) -> int:
        return 3 + 6 * self.pe_octaves


def proposal_layout(spec: ProposalSpec) -> Dict[str, Tuple[int, Tuple[int, ...]]]:
    """Flat layout of the proposal network: W_l [width, in_l], b_l [width] for
    l < layers, then w_out [width], b_out [1]."""
    out = {}
    off = 0
    for l in range(spec.layers):
        fan_in = spec.in_dim if l == 0 else spec.width
        out[f"W{l}"] = (off, (spec.width, fan_in)); off += spec.width * fan_in
        out[f"b{l}"] = (off, (spec.width,)); off += spec.width
    out["w_out"] = (off, (spec.width,)); off += spec.width
    out["b_out"] = (off, (1,)); off += 1
    out["__total__"] = (off, ())
    return out


def proposal_init(spec: ProposalSpec, seed: int) -> np.ndarray:
    """He-normal weights, zero biases, float32 flat vector."""
    lay = proposal_layout(spec)
    rng = np.random.default_rng(seed)
    p = np.zeros(lay["__total__"][0])
    for l in range(spec.layers):
        o, shp = lay[f"W{l}"]
        p[o:o + shp[0] * shp[1]] = rng.normal(0.0, np.sqrt(2.0 / shp[1]), shp).ravel()
    o, shp = lay["w_out"]
    p[o:o + shp[0]] = rng.normal(0.0, np.sqrt(1.0 / shp[0]), shp[0])
    return p.astype(np.float32)
