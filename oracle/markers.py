"""Marker addition and deletion of the conventional front tracking (oracle;
test infrastructure only).

Section 2.2 describes the scheme of Singh et al. as the foil for the B-spline
reconstruction: a marker closer than h/2 to its neighbour is deleted, and
where two neighbours are more than 1.5 h apart a marker is added at their
midpoint; both steps make the curvature fluctuate (eq interpol_cir).

Readings (the paper gives only the two thresholds): the closed curve is
walked once from marker 0, deleting each marker closer than lo h to the last
kept one (and the last kept marker if it ends closer than lo h to marker 0,
as long as three remain); then each gap of the kept curve longer than hi h
receives one marker at its midpoint.
"""
import numpy as np


def add_delete(X, h, lo=0.5, hi=1.5):
    X = np.asarray(X, dtype=np.float64)
    kept = [X[0]]
    for k in range(1, len(X)):
        if np.hypot(*(X[k] - kept[-1])) >= lo * h:
            kept.append(X[k])
    if len(kept) > 3 and np.hypot(*(kept[0] - kept[-1])) < lo * h:
        kept.pop()
    out = []
    for k in range(len(kept)):
        a, b = kept[k], kept[(k + 1) % len(kept)]
        out.append(a)
        if np.hypot(*(b - a)) > hi * h:
            out.append(0.5 * (a + b))
    return np.array(out)


def menger_curvature(X):
    """Curvature of the circle through each marker and its two neighbours
    (a local three-point estimate, exact for markers on a circle)."""
    a, b, c = np.roll(X, 1, axis=0), X, np.roll(X, -1, axis=0)
    cross = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])
    la = np.linalg.norm(b - a, axis=1)
    lb = np.linalg.norm(c - b, axis=1)
    lc = np.linalg.norm(c - a, axis=1)
    return 2.0 * cross / (la * lb * lc)
