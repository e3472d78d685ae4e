"""Oracle pins for the marker addition / deletion foil (Section 2.2).

* spacings inside [h/2, 1.5 h] are left alone; a curve sampled 2 h apart gets
  every gap halved; one sampled h/4 apart keeps every second or third marker
  with every kept gap in [h/2, h);
* the three-point curvature is exact on markers of a circle, and a midpoint
  added in every other interval makes it fluctuate by the full curvature (the
  midpoint and its neighbours are collinear), the fluctuation of the paper's
  figure (the B-spline relocation never adds or deletes: it re-samples the
  fitted curve at equal arc spacing).
"""
import numpy as np

from oracle import markers
from paper_1807_10504_amd import workloads as W


def test_thresholds():
    h = 1 / 64
    R = 0.25
    for spacing, expect in ((0.8, None), (2.0, "double"), (0.25, "thin")):
        n = int(round(2 * np.pi * R / (spacing * h)))
        X = W.circle_markers(n, R)
        Y = markers.add_delete(X, h)
        gaps = np.linalg.norm(np.roll(Y, -1, 0) - Y, axis=1)
        if expect is None:
            assert np.array_equal(Y, X)
        elif expect == "double":
            assert len(Y) == 2 * n and np.all(gaps < 1.5 * h)
        else:
            assert n // 3 <= len(Y) <= n // 2 and gaps.min() >= 0.5 * h and gaps.max() < 1.5 * h


def test_midpoints_make_curvature_fluctuate():
    h, R = 1 / 64, 0.25
    n = 100
    X = W.circle_markers(n, R)
    k = markers.menger_curvature(X)
    assert np.abs(k - 1 / R).max() <= 1e-9 / R
    # stretch every other interval beyond 1.5 h: drop every fourth marker of a
    # denser circle, then add midpoints
    th = 2 * np.pi * np.arange(120) / 120             # 0.84 h apart; gaps of 1.68 h after the drop
    keep = np.arange(120) % 4 != 3
    Xs = np.stack([0.5 + R * np.cos(th[keep]), 0.5 + R * np.sin(th[keep])], axis=1)
    Y = markers.add_delete(Xs, h)
    assert len(Y) == 120
    kY = markers.menger_curvature(Y)
    assert kY.min() <= 1e-9 / R and kY.max() >= 1.5 / R   # midpoints: zero; their neighbours overshoot
