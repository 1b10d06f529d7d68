"""Host-side checks of the measurement helpers in bench.py (no GPU)."""
import math
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def _front(n=801, c=400, radius=100.0, width=1.77, harmonic=None, amp=0.1):
    y, x = np.mgrid[0:n, 0:n].astype(float)
    r = np.hypot(x - c, y - c)
    th = np.arctan2(y - c, x - c)
    rad = radius * (1 + amp * np.cos(harmonic * th)) if harmonic else radius
    return np.tanh((rad - r) / width)


def test_l2_metric_definition_on_sampled_profiles():
    # on a field that is linear in x and y the interpolation is exact, so the
    # metric equals Eq. Error_L2 evaluated on the exact profiles
    n, c = 101, 50
    y, x = np.mgrid[0:n, 0:n].astype(float)
    phi = 0.3 + 0.01 * (x - c) - 0.02 * (y - c)
    j = np.arange(0, 49)
    pa = 0.3 + 0.01 * j
    pb = 0.3 + 0.01 * (0.5 * j) - 0.02 * (-math.sqrt(3) / 2 * j)
    ref = math.sqrt(np.sum((pa - pb) ** 2) / np.sum(pa ** 2))
    assert bench.profile_l2_error(phi, (c, c)) == pytest.approx(ref, rel=1e-12)


@pytest.mark.parametrize("harmonic", [None, 6])
def test_l2_metric_small_for_sixfold_symmetric_fronts(harmonic):
    # profiles 60 degrees apart coincide: only interpolation error remains
    assert bench.profile_l2_error(_front(harmonic=harmonic), (400, 400)) < 1e-3


def test_l2_metric_detects_threefold_front():
    assert bench.profile_l2_error(_front(harmonic=3), (400, 400)) > 0.1


def test_tip_radius_on_fourfold_front():
    # a four-fold front r = 15 (1 + 0.1 cos 4 (theta - 0.3)) around an off-node centre
    n = 200
    y, x = np.mgrid[0:n, 0:n].astype(float)
    cx, cy = 100.3, 99.6
    r = np.hypot(x - cx, y - cy)
    th = np.arctan2(y - cy, x - cx)
    phi = np.tanh((15 * (1 + 0.1 * np.cos(4 * (th - 0.3))) - r) / 2.5)
    for t in (0.3, 0.3 + math.pi / 2, 0.3 + math.pi / 4):
        assert abs(bench.tip_radius(phi, cx, cy, t) - 15 * (1 + 0.1 * math.cos(4 * (t - 0.3)))) < 0.01
