"""Marker binning (oracle): the plain definition of the deterministic bins.

Markers are grouped by the tile of 4^dim cells that contains them (position
wrapped into the periodic box); within a tile they keep ascending marker
index. tile_start[t] is the first position of tile t in that order.
"""
import numpy as np


def bin_markers(X, n, h, tile=4):
    X = np.asarray(X, dtype=np.float64)
    N, dim = X.shape
    key = np.zeros(N, dtype=np.int64)
    mult = 1
    for e in range(dim):
        c = np.mod(np.floor(X[:, e] / h).astype(np.int64), n[e]) // tile
        key += c * mult
        mult *= n[e] // tile
    order = np.argsort(key, kind="stable")
    start = np.searchsorted(key[order], np.arange(mult + 1), side="left")
    return key.astype(np.int32), order.astype(np.int32), start.astype(np.int32)
