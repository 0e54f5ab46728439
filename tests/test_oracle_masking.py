"""Pins of the dynamic loss masking oracle (Sec. Optimization): invariants of
the rule and the masked loss's gradient, not a re-typing of the formula."""
import numpy as np

from oracle import render as orc
from oracle.masking import mask_update


def test_first_iteration_masks_nothing_and_records_power():
    rng = np.random.default_rng(0)
    p = rng.uniform(0, 10, 1000).astype(np.float32)
    m, h = mask_update(p, p, np.zeros(1000, np.float32))
    assert m.min() == 1.0
    np.testing.assert_array_equal(h, p)


def test_steady_or_rising_power_is_never_masked():
    rng = np.random.default_rng(1)
    ref = rng.uniform(0, 10, 500)
    h = np.zeros(500, np.float32)
    p = rng.uniform(0, 10, 500).astype(np.float32)
    for t in range(6):
        m, h = mask_update(p, ref, h, 0.25, 0.25)
        assert m.min() == 1.0
        p = (p * 1.1).astype(np.float32)          # never below its own history


def test_drop_after_a_strong_response_is_masked_weak_history_is_not():
    ref = np.array([10.0, 1.0, 1.0])
    h = np.zeros(3, np.float32)
    _, h = mask_update(np.array([8.0, 1.0, 2.0], np.float32), ref, h)   # strong, weak, strong
    m, h2 = mask_update(np.array([0.5, 0.1, 1.5], np.float32), ref, h)
    # point 0: history 8 >= 2.5 and 0.5 < 2 -> dropped; point 1: history 1 < 2.5 -> kept;
    # point 2: history 2 < 2.5 -> kept although it fell
    np.testing.assert_array_equal(m, [0.0, 1.0, 1.0])
    np.testing.assert_array_equal(h2, [8.0, 1.0, 2.0])


def test_history_is_monotone_and_bounds_every_past_power():
    rng = np.random.default_rng(2)
    ref = rng.uniform(0, 5, 300)
    h = np.zeros(300, np.float32)
    seen = np.zeros(300, np.float32)
    for t in range(8):
        p = rng.uniform(0, 5, 300).astype(np.float32)
        _, h_new = mask_update(p, ref, h)
        assert np.all(h_new >= h)
        seen = np.maximum(seen, p)
        np.testing.assert_array_equal(h_new, seen)
        h = h_new


def test_masked_points_carry_no_loss_gradient():
    rng = np.random.default_rng(3)
    p = rng.uniform(0, 5, 64)
    ps = rng.uniform(0, 5, 64)
    mask = (rng.uniform(size=64) > 0.3).astype(np.float64)
    L, g = orc.loss_l2(p, ps, mask)
    assert np.all(g[mask == 0] == 0.0)
    # the loss does not move when a masked point's prediction moves
    q = p.copy()
    q[mask == 0] += 1.0
    assert orc.loss_l2(q, ps, mask)[0] == L
