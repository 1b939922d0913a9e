"""Geodesic Voronoi cells and Lloyd steps towards a centroidal Voronoi
tessellation on PTP labels, FP64 (the paper names centroidal Voronoi
tessellations as an application of its method, Sec. 7; its Voronoi labels
come from multi-source PTP, Sec. 5.3).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Readings (the paper gives no formulas): a vertex carries the barycentric
area A_v = (1/3) sum of the areas of its incident triangles; the centroid of
cell s is sum A_v x_v / sum A_v over the vertices labelled s; a Lloyd step
moves the generator of cell s to the vertex of that cell nearest (Euclidean)
to its centroid, smallest id on a tie; a cell without vertices keeps its
generator.  The energy of a tessellation is sum A_v d(v)^2.
"""
from __future__ import annotations

import numpy as np

from . import run


def vertex_areas(V, F) -> np.ndarray:
    X = np.asarray(V, np.float32).astype(np.float64)
    F = np.asarray(F, np.int64).reshape(-1, 3)
    A = np.zeros(X.shape[0])
    for t in range(F.shape[0]):
        a, b, c = F[t]
        area = 0.5 * np.linalg.norm(np.cross(X[b] - X[a], X[c] - X[a]))
        for v in (a, b, c):
            A[v] += area / 3.0
    return A


def cell_moments(V, F, label, m):
    """Per cell: area sum_{lab v = s} A_v and area-weighted position sum."""
    X = np.asarray(V, np.float32).astype(np.float64)
    A = vertex_areas(V, F)
    area = np.zeros(m)
    mom = np.zeros((m, 3))
    for v in range(X.shape[0]):
        s = int(label[v])
        if s < 0:
            continue
        area[s] += A[v]
        mom[s] += A[v] * X[v]
    return area, mom


def lloyd_step(V, F, label, S):
    """New generators (int32 [m]) and the centroids (float64 [m, 3])."""
    X = np.asarray(V, np.float32).astype(np.float64)
    S = np.asarray(S, np.int32)
    m = S.shape[0]
    area, mom = cell_moments(V, F, label, m)
    cen = np.zeros((m, 3))
    out = S.copy()
    for s in range(m):
        if not area[s] > 0:
            cen[s] = X[S[s]]
            continue
        cen[s] = mom[s] / area[s]
        best, bv = np.inf, -1
        for v in np.nonzero(np.asarray(label) == s)[0]:
            e = X[v] - cen[s]
            q = e @ e
            if q < best:
                best, bv = q, int(v)
        out[s] = bv
    return out, cen


def energy(V, F, dist) -> float:
    d = np.asarray(dist, np.float64)
    A = vertex_areas(V, F)
    fin = np.isfinite(d)
    return float(np.sum(A[fin] * d[fin] ** 2))


def lloyd(V, F, S0, iters, tol, lib=None):
    """`iters` Lloyd steps from S0; returns the generator sets (iters + 1) and
    the energy of each tessellation."""
    S = np.asarray(S0, np.int32).copy()
    sets, energies = [S.copy()], []
    for _ in range(iters):
        r = run(V, F, S, tol, lib=lib)
        energies.append(energy(V, F, r.dist))
        S, _ = lloyd_step(V, F, r.label, S)
        sets.append(S.copy())
    r = run(V, F, S, tol, lib=lib)
    energies.append(energy(V, F, r.dist))
    return sets, energies
