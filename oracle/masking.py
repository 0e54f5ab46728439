"""Oracle of the dynamic loss masking (Sec. Optimization).  TEST INFRASTRUCTURE ONLY.

The paper leaves a point out of the loss when its filter output was high in an
earlier iteration and is low in the current one, without fixing "high" and
"low".  Reading used here, with S the peak of the measured heatmap P* and H the
per-point maximum of the rendered filter output over earlier iterations:

    drop  <=>  H >= tau_hi * S   and   P < tau_lo * H ,     then H <- max(H, P).

The two decisions are taken in float32 (each product rounded to float32
before the comparison), the precision the GPU kernel decides them in.
"""
from __future__ import annotations

import numpy as np


def mask_update(power, power_ref, history, tau_hi=0.25, tau_lo=0.25):
    """(mask float32 [n] with 1 = keep, 0 = drop; new history float32 [n])."""
    p = np.asarray(power, np.float32).ravel()
    h = np.asarray(history, np.float32).ravel()
    peak = np.float32(np.max(np.asarray(power_ref, np.float32)))
    hi = np.float32(np.float32(tau_hi) * peak)
    drop = (h >= hi) & (p < np.float32(tau_lo) * h)
    return np.where(drop, np.float32(0.0), np.float32(1.0)), np.maximum(h, p)
