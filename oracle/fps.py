"""Farthest point sampling on PTP distances (paper Sec. 5.3 and App. A), FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The sampling starts from a source set S and repeats: compute the distance map
of the current set with the PTP iteration, take the reachable vertex farthest
from it, add it to the set.  Two ways to compute each map:

* cold (the paper's use): every map from +inf;
* warm: every map starts from the previous one.  The previous map is a
  supersolution for the enlarged set (each of its values was set to the
  planar update of an earlier, pointwise larger map, and adding a source only
  lowers updates), so it is taken as the starting bound without
  certification.

The farthest vertex is decided on the map rounded to float32 (the precision
the GPU decides in), largest value first, smallest vertex id on a tie.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import run, run_warm


@dataclass
class FpsResult:
    samples: np.ndarray       # int32 [m]: S0 followed by the chosen vertices
    radius: np.ndarray        # float64 [m - len(S0)]: distance of each chosen vertex
    iterations: np.ndarray    # int64 [steps + 1]: K of every map (the last: final set)
    updates: np.ndarray       # int64 [steps + 1]: U of every map
    dist: np.ndarray          # float64 [n]: map of the final set
    maps: list                # the maps the choices were made on (keep_maps=True)


def farthest(dist: np.ndarray) -> int:
    """Vertex with the largest finite distance (float32 comparison, smallest
    id on a tie); -1 when no vertex has a positive finite distance."""
    d = np.asarray(dist, np.float64).astype(np.float32)
    fin = np.isfinite(d)
    if not fin.any():
        return -1
    best = d[fin].max()
    if not best > 0:
        return -1
    return int(np.nonzero(fin & (d == best))[0][0])


def fps(V, F, S0, m, tol, warm=False, samples=None, keep_maps=False, lib=None) -> FpsResult:
    """Grow S0 to m vertices by farthest point sampling.  `samples` (optional,
    length m) replays given choices instead of the argmax: every map is then
    the one those choices produce, so another implementation's picks can be
    checked one by one."""
    S = [int(s) for s in np.asarray(S0).ravel()]
    if m < len(S):
        raise ValueError("m below the initial set")
    radius, its, ups, maps = [], [], [], []
    prev = None
    while True:
        Sa = np.array(S, np.int32)
        if warm and prev is not None:
            r = run_warm(V, F, Sa, tol, prev, certify=False, lib=lib)
        else:
            r = run(V, F, Sa, tol, lib=lib)
        its.append(r.iterations)
        ups.append(r.updates)
        if keep_maps:
            maps.append(r.dist.copy())
        prev = r.dist
        if len(S) == m:
            break
        v = int(samples[len(S)]) if samples is not None else farthest(r.dist)
        if v < 0:
            raise ValueError("no reachable vertex left to sample")
        radius.append(float(r.dist[v]))
        S.append(v)
    return FpsResult(np.array(S, np.int32), np.array(radius), np.array(its, np.int64),
                     np.array(ups, np.int64), prev, maps)
