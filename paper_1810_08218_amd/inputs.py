"""Seeded synthetic meshes and source sets for the PTP workloads.

This module only builds inputs: vertex coordinates, triangle indices and
source vertex ids.  It contains none of the method's arithmetic (no BFS, no
distance, no local update), so both the CPU oracle and the HIP path can be
fed from it without sharing any part of the computation.

Every mesh is built in float64 and rounded once to float32; both sides read
the same float32 coordinates.  Faces are int32 ``[f, 3]``, sources int32.

Workloads (the paper's scanned meshes are not available; these stand in for
them, see the experimental section of the paper):

* ``flat_grid(s)``: s x s grid on the unit square, each cell split along the
  (i, j) -> (i+1, j+1) diagonal; all triangles right-isosceles.  The 64 x 64
  case with the source at vertex (0, 0) is the flat-plane accuracy check
  (regular grid experiment of the accuracy section).
* ``noisy_icosphere(level=7, seed=2)``: unit icosphere, tangential Gaussian
  noise of 0.1 x mean edge length, reprojected onto the sphere; one random
  source (single-source runs of the performance section).
* ``bumpy_icosphere(level=9, seed=3)``: radially displaced icosphere with 32
  random sources (multi-source / Voronoi runs, Fig. ptp_speedup_sources).
* ``batch_mesh(t)`` / ``batch_meshes()``: 512 uneven meshes, jittered grids and
  tori, 1-4 sources each (batched form).
* ``training_mesh(t)``: the warm-start network's training and evaluation
  meshes (jittered grids, noisy and bumpy icospheres, 1-32 sources).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Mesh:
    V: np.ndarray          # float32 [n, 3]
    F: np.ndarray          # int32 [f, 3]
    S: np.ndarray          # int32 [m]
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.V.shape[0])

    @property
    def f(self) -> int:
        return int(self.F.shape[0])

    @property
    def m(self) -> int:
        return int(self.S.shape[0])


def _f32(V64: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(V64, dtype=np.float64).astype(np.float32)


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a), dtype=np.int32)


# ---------------------------------------------------------------- grids ---

def grid_faces(s: int) -> np.ndarray:
    """Faces of an s x s vertex grid, vertex id j*s + i; cell (i, j) gives
    [v(i,j), v(i+1,j), v(i+1,j+1)] and [v(i,j), v(i+1,j+1), v(i,j+1)]."""
    i, j = np.meshgrid(np.arange(s - 1), np.arange(s - 1), indexing="xy")
    i = i.ravel()
    j = j.ravel()
    v00 = j * s + i
    v10 = v00 + 1
    v11 = v00 + s + 1
    v01 = v00 + s
    t1 = np.stack([v00, v10, v11], axis=1)
    t2 = np.stack([v00, v11, v01], axis=1)
    F = np.empty((2 * t1.shape[0], 3), dtype=np.int64)
    F[0::2] = t1
    F[1::2] = t2
    return _i32(F)


def grid_vertices64(s: int, extent: float = 1.0) -> np.ndarray:
    i, j = np.meshgrid(np.arange(s), np.arange(s), indexing="xy")
    h = extent / (s - 1)
    V = np.zeros((s * s, 3), dtype=np.float64)
    V[:, 0] = i.ravel() * h
    V[:, 1] = j.ravel() * h
    return V


def flat_grid(s: int = 64, source: int | tuple = 0, extent: float = 1.0) -> Mesh:
    """Regular s x s grid; ``source`` is a vertex id or an (i, j) pair."""
    if isinstance(source, tuple):
        source = source[1] * s + source[0]
    V = grid_vertices64(s, extent)
    return Mesh(_f32(V), grid_faces(s), _i32([source]), name=f"grid{s}",
                meta={"s": s, "h": extent / (s - 1)})


def jittered_grid(s: int, rng: np.random.Generator, amp: float = 0.2) -> tuple:
    """Unit-square grid, interior vertices moved by U(-amp*h, amp*h) in x and
    y; the boundary stays straight.  Returns (V64, F)."""
    V = grid_vertices64(s)
    h = 1.0 / (s - 1)
    jit = rng.uniform(-amp * h, amp * h, size=(s * s, 2))
    i = np.arange(s * s) % s
    j = np.arange(s * s) // s
    interior = (i > 0) & (i < s - 1) & (j > 0) & (j < s - 1)
    V[interior, 0:2] += jit[interior]
    return V, grid_faces(s)


def torus(nu: int, nv: int, r: float, R: float = 1.0) -> tuple:
    """Torus with nu (major) x nv (minor) vertices, quads split like the
    grid.  Returns (V64, F)."""
    iu, iv = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
    tu = 2.0 * np.pi * iu.ravel() / nu
    tv = 2.0 * np.pi * iv.ravel() / nv
    V = np.stack([(R + r * np.cos(tv)) * np.cos(tu),
                  (R + r * np.cos(tv)) * np.sin(tu),
                  r * np.sin(tv)], axis=1)
    a = iu.ravel()
    b = iv.ravel()
    v00 = a * nv + b
    v10 = ((a + 1) % nu) * nv + b
    v01 = a * nv + (b + 1) % nv
    v11 = ((a + 1) % nu) * nv + (b + 1) % nv
    t1 = np.stack([v00, v10, v11], axis=1)
    t2 = np.stack([v00, v11, v01], axis=1)
    F = np.empty((2 * t1.shape[0], 3), dtype=np.int64)
    F[0::2] = t1
    F[1::2] = t2
    return V, _i32(F)


# ----------------------------------------------------------- icospheres ---

def icosahedron() -> tuple:
    """Unit icosahedron: cyclic permutations of (0, +-1, +-phi), faces from
    the convex hull, oriented outward."""
    from scipy.spatial import ConvexHull
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    pts = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            pts.append((0.0, s1, s2 * phi))
            pts.append((s1, s2 * phi, 0.0))
            pts.append((s2 * phi, 0.0, s1))
    V = np.asarray(pts, dtype=np.float64)
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    F = ConvexHull(V).simplices.astype(np.int64)
    nrm = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    flip = np.einsum("ij,ij->i", nrm, V[F].mean(axis=1)) < 0
    F[flip] = F[flip][:, [0, 2, 1]]
    return V, F


def subdivide(V: np.ndarray, F: np.ndarray) -> tuple:
    """One midpoint subdivision step with reprojection onto the unit sphere."""
    n = V.shape[0]
    e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]], axis=0)
    lo = np.minimum(e[:, 0], e[:, 1])
    hi = np.maximum(e[:, 0], e[:, 1])
    key = lo.astype(np.int64) * n + hi
    uniq, inv = np.unique(key, return_inverse=True)
    ulo = uniq // n
    uhi = uniq % n
    mid = V[ulo] + V[uhi]
    mid /= np.linalg.norm(mid, axis=1, keepdims=True)
    nf = F.shape[0]
    m01 = n + inv[0:nf]
    m12 = n + inv[nf:2 * nf]
    m20 = n + inv[2 * nf:3 * nf]
    a, b, c = F[:, 0], F[:, 1], F[:, 2]
    F2 = np.concatenate([
        np.stack([a, m01, m20], axis=1),
        np.stack([b, m12, m01], axis=1),
        np.stack([c, m20, m12], axis=1),
        np.stack([m01, m12, m20], axis=1)], axis=0)
    return np.concatenate([V, mid], axis=0), F2


_ICO_CACHE: dict = {}


def icosphere64(level: int) -> tuple:
    """Unit icosphere after ``level`` subdivisions (float64 vertices, int64
    faces).  Returns fresh copies of a cached mesh."""
    if level not in _ICO_CACHE:
        V, F = icosahedron()
        for _ in range(level):
            V, F = subdivide(V, F)
        _ICO_CACHE[level] = (V, F)
    V, F = _ICO_CACHE[level]
    return V.copy(), F.copy()


def mean_edge_length(V: np.ndarray, F: np.ndarray) -> float:
    e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]], axis=0)
    e = e[e[:, 0] < e[:, 1]]  # each undirected edge once on a closed mesh
    return float(np.linalg.norm(V[e[:, 0]] - V[e[:, 1]], axis=1).mean())


def sphere(level: int, seed: int | None = None, n_sources: int = 1,
           noise: float = 0.0) -> Mesh:
    """Unit icosphere (optionally with tangential noise), random sources."""
    V, F = icosphere64(level)
    rng = np.random.default_rng(seed)
    if noise > 0.0:
        V = _tangential_noise(V, F, rng, noise)
    S = rng.choice(V.shape[0], n_sources, replace=False)
    return Mesh(_f32(V), _i32(F), _i32(np.sort(S)), name=f"sphere{level}")


def _tangential_noise(V, F, rng, sigma_rel):
    ell = mean_edge_length(V, F)
    g = rng.normal(size=V.shape)
    g -= np.einsum("ij,ij->i", g, V)[:, None] * V
    V = V + sigma_rel * ell * g
    return V / np.linalg.norm(V, axis=1, keepdims=True)


def noisy_icosphere(level: int = 7, seed: int = 2) -> Mesh:
    """Icosphere of radius 1, ``level`` subdivisions, each vertex displaced
    tangentially by N(0, (0.1 * mean edge)^2) and put back on the sphere; one
    source drawn uniformly.  Level 7: 163,842 vertices, 327,680 triangles."""
    V, F = icosphere64(level)
    rng = np.random.default_rng(seed)
    V = _tangential_noise(V, F, rng, 0.1)
    src = int(rng.integers(V.shape[0]))
    return Mesh(_f32(V), _i32(F), _i32([src]), name=f"noisy_icosphere{level}",
                meta={"level": level, "seed": seed})


def bumpy_icosphere(level: int = 9, seed: int = 3, n_sources: int = 32) -> Mesh:
    """Icosphere with radius r = 1 + 0.15 * sum_k a_k sin(f_k (n . u_k)),
    a_k ~ U(0,1)/k, f_k ~ U(2,12), u_k random unit vectors (k = 1..8), and
    ``n_sources`` distinct random sources.  Level 9: 2,621,442 vertices,
    5,242,880 triangles."""
    N, F = icosphere64(level)
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.0, 1.0, 8) / np.arange(1, 9)
    fr = rng.uniform(2.0, 12.0, 8)
    u = rng.normal(size=(8, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    r = 1.0 + 0.15 * (a[None, :] * np.sin(fr[None, :] * (N @ u.T))).sum(axis=1)
    V = N * r[:, None]
    S = rng.choice(V.shape[0], n_sources, replace=False)
    return Mesh(_f32(V), _i32(F), _i32(S), name=f"bumpy_icosphere{level}",
                meta={"level": level, "seed": seed})


# ---------------------------------------------------------------- batch ---

def batch_mesh(t: int, seed: int = 4) -> Mesh:
    """Mesh t of the 512-mesh batch: t < 256 jittered grid with side
    round(exp(U(ln 32, ln 1024))); t >= 256 torus with 2^k x 2^(k-1)
    vertices, k ~ U{5..10}, r ~ U(0.2, 0.5), R = 1.  1-4 distinct sources."""
    rng = np.random.default_rng([seed, t])
    if t < 256:
        s = int(round(math.exp(rng.uniform(math.log(32.0), math.log(1024.0)))))
        V, F = jittered_grid(s, rng)
        name = f"jgrid{s}"
    else:
        k = int(rng.integers(5, 11))
        r = float(rng.uniform(0.2, 0.5))
        V, F = torus(2 ** k, 2 ** (k - 1), r)
        name = f"torus{k}"
    m = int(rng.integers(1, 5))
    S = rng.choice(V.shape[0], m, replace=False)
    return Mesh(_f32(V), F, _i32(S), name=name, meta={"t": t})


def batch_meshes(count: int = 512, seed: int = 4, first: int = 0) -> list:
    return [batch_mesh(t, seed) for t in range(first, first + count)]


# ------------------------------------------------------- warm-start data ---

def training_mesh(t: int, seed: int = 5) -> Mesh:
    """Mesh t of the warm-start training set (another ``seed`` gives held-out
    meshes).  t % 3 == 0: jittered grid, side round(exp(U(ln 32, ln 256)));
    1: icosphere of level U{3..6} with tangential noise of 0.1 mean edge;
    2: bumpy icosphere (radial sum of 8 sines as in ``bumpy_icosphere``) of
    level U{4..6}.  1-32 distinct random sources."""
    rng = np.random.default_rng([seed, t])
    kind = t % 3
    if kind == 0:
        s = int(round(math.exp(rng.uniform(math.log(32.0), math.log(256.0)))))
        V, F = jittered_grid(s, rng)
        name = f"jgrid{s}"
        V64 = V.astype(np.float64)
    elif kind == 1:
        level = int(rng.integers(3, 7))
        V64, F = icosphere64(level)
        V64 = _tangential_noise(V64, F, rng, 0.1)
        name = f"noisy_icosphere{level}"
    else:
        level = int(rng.integers(4, 7))
        N, F = icosphere64(level)
        a = rng.uniform(0.0, 1.0, 8) / np.arange(1, 9)
        fr = rng.uniform(2.0, 12.0, 8)
        u = rng.normal(size=(8, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        r = 1.0 + 0.15 * (a[None, :] * np.sin(fr[None, :] * (N @ u.T))).sum(axis=1)
        V64 = N * r[:, None]
        name = f"bumpy_icosphere{level}"
    n = V64.shape[0]
    m = int(rng.integers(1, 33))
    S = np.sort(rng.choice(n, m, replace=False))
    return Mesh(_f32(V64), _i32(F), _i32(S), name=name, meta={"t": t, "seed": seed})
