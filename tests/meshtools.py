"""Independent reference computations for the pins: edge graphs, BFS levels
and Dijkstra distances through scipy.sparse.csgraph, closed-form distances.
None of this comes from the oracle or from the HIP library."""
from __future__ import annotations

import json
import os

import numpy as np
import scipy.sparse as sp
from scipy.sparse import csgraph

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name: str) -> dict:
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


def edges(F: np.ndarray) -> np.ndarray:
    e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]], axis=0).astype(np.int64)
    e = np.sort(e, axis=1)
    return np.unique(e, axis=0)


def edge_graph(V, F, weighted: bool):
    n = V.shape[0]
    e = edges(F)
    if weighted:
        X = V.astype(np.float64)
        w = np.linalg.norm(X[e[:, 0]] - X[e[:, 1]], axis=1)
    else:
        w = np.ones(e.shape[0])
    G = sp.coo_matrix((np.concatenate([w, w]),
                       (np.concatenate([e[:, 0], e[:, 1]]), np.concatenate([e[:, 1], e[:, 0]]))),
                      shape=(n, n)).tocsr()
    return G


def bfs_levels(V, F, S) -> np.ndarray:
    """Hop distance to the nearest source (-1 unreachable), by scipy."""
    G = edge_graph(V, F, weighted=False)
    d = csgraph.dijkstra(G, unweighted=True, indices=np.asarray(S), min_only=True)
    out = np.where(np.isfinite(d), d, -1).astype(np.int64)
    return out


def canonical_order(level: np.ndarray) -> np.ndarray:
    """Vertex ids sorted by (level, id) with unreachable (-1) last."""
    key = np.where(level < 0, level.max() + 1, level)
    return np.lexsort((np.arange(level.shape[0]), key))


def dijkstra(V, F, S) -> np.ndarray:
    G = edge_graph(V, F, weighted=True)
    return csgraph.dijkstra(G, indices=np.asarray(S), min_only=True)


def rel_err(got, ref, mask=None):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    m = np.isfinite(ref) & (ref > 0)
    if mask is not None:
        m &= mask
    e = np.abs(got[m] - ref[m]) / ref[m]
    return float(e.max()) if e.size else 0.0, float(e.mean()) if e.size else 0.0
