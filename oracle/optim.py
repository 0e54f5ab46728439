"""Oracle of the optimiser (App. C, Training Setup): AdamW with cosine annealing.

TEST INFRASTRUCTURE ONLY.

AdamW (Loshchilov & Hutter, "Decoupled Weight Decay Regularization", ICLR 2019)
at step t >= 1 with per-parameter learning rate lr_p:
    m = b1 m + (1-b1) g ;  v = b2 v + (1-b2) g^2
    p = p - lr_p * ( m / (1-b1^t) / (sqrt(v / (1-b2^t)) + eps) + wd * p )
Cosine annealing: lr(t) = lr_min + (lr_max - lr_min) (1 + cos(pi t / T)) / 2.
The paper uses lr 1e-3 for everything except the SDF network (1e-4).
"""
from __future__ import annotations

import numpy as np


def cosine_lr(t: int, total: int, lr_max: float, lr_min: float = 0.0) -> float:
    t = min(max(t, 0), total)
    return lr_min + (lr_max - lr_min) * 0.5 * (1.0 + np.cos(np.pi * t / total))


def adamw_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8, wd=0.0):
    """One update; ``lr`` may be a scalar or a per-parameter array. Returns (p, m, v)."""
    p = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    p = p - np.asarray(lr) * (mhat / (np.sqrt(vhat) + eps) + wd * p)
    return p, m, v
