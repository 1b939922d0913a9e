"""Pins of the oracle's applications of the distance maps: farthest point
sampling (paper Sec. 5.3) and Lloyd steps on geodesic Voronoi cells (Sec. 7
names centroidal Voronoi tessellations).  CPU only."""
import numpy as np
import pytest

import oracle as O
from meshtools import dijkstra
from oracle import cvt as OC
from oracle import fps as OF
from paper_1810_08218_amd import inputs as I


def test_fps_grid_first_picks():
    """Flat grid from corner (0, 0).  The far corner is the unique farthest
    vertex: the scheme is exact on the diagonal (63 sqrt2 h) and every other
    vertex lies below its Dijkstra distance, at most 62 sqrt2 h + h.  Then
    the two other corners tie in float32 (each is reached along a straight
    edge path from a source); the smaller id wins."""
    m = I.flat_grid(64)
    r = OF.fps(m.V, m.F, m.S, 4, 1e-6)
    assert r.samples.tolist() == [0, 4095, 63, 4032]
    assert r.radius[0] == pytest.approx(np.sqrt(2.0), rel=1e-12)
    dj = dijkstra(m.V, m.F, np.array([0, 4095]))
    assert r.radius[1] <= dj[63] * (1 + 1e-12)


def test_fps_picks_are_farthest_and_radius_falls():
    m = I.noisy_icosphere(level=4, seed=3)
    r = OF.fps(m.V, m.F, m.S, 30, 1e-7, keep_maps=True)
    for i, mp in enumerate(r.maps[:-1]):
        v = r.samples[m.m + i]
        f32 = mp.astype(np.float32)
        assert f32[v] == f32[np.isfinite(f32)].max()
        assert v == np.nonzero(f32 == f32[v])[0][0]
        assert r.radius[i] == mp[v]
    assert (np.diff(r.radius) <= 1e-12).all()
    assert len(set(r.samples.tolist())) == 30
    # the final map is the PTP map of the final set
    o = O.run(m.V, m.F, r.samples, 1e-7)
    assert np.array_equal(o.dist, r.dist)


def test_fps_warm_equals_cold_and_descends():
    """Warm restarts pick the same samples; every warm map lies at or below
    the map it started from, and the maps agree with the cold ones to the
    iteration's tolerance.  The previous map is a supersolution up to
    rounding: certification withdraws only values whose planar update
    exceeds them by float64 rounding."""
    m = I.noisy_icosphere(level=4, seed=3)
    c = OF.fps(m.V, m.F, m.S, 20, 1e-7, keep_maps=True)
    w = OF.fps(m.V, m.F, m.S, 20, 1e-7, warm=True, keep_maps=True)
    assert np.array_equal(c.samples, w.samples)
    for a, b in zip(w.maps[:-1], w.maps[1:]):
        assert (b <= a).all()
    for a, b in zip(c.maps, w.maps):
        fin = a > 0
        assert np.max(np.abs(a[fin] - b[fin]) / a[fin]) < 1e-5
    assert (w.updates[1:] <= c.updates[1:]).all() and w.updates[1:].sum() < c.updates[1:].sum()


def test_fps_replay_of_given_picks():
    m = I.noisy_icosphere(level=3, seed=1)
    r = OF.fps(m.V, m.F, m.S, 10, 1e-6)
    p = OF.fps(m.V, m.F, m.S, 10, 1e-6, samples=r.samples)
    assert np.array_equal(p.samples, r.samples) and np.array_equal(p.dist, r.dist)


def test_vertex_areas_closed_form():
    """Unit-square grid: the areas sum to 1; an interior vertex touches six
    right triangles of area h^2 / 2, so it carries h^2; the corner (0, 0)
    lies on its cell's diagonal and touches both triangles (h^2 / 3), the
    corner (1, 0) only one (h^2 / 6)."""
    s = 64
    m = I.flat_grid(s)
    A = OC.vertex_areas(m.V, m.F)
    h = 1.0 / (s - 1)
    X = m.V.astype(np.float64)
    assert A.sum() == pytest.approx(1.0, rel=1e-12)
    v = 10 * s + 10
    hx = X[v + 1, 0] - X[v, 0]
    assert A[v] == pytest.approx(hx * (X[v + s, 1] - X[v, 1]), rel=1e-6)
    assert A[0] == pytest.approx(h * h / 3, rel=1e-6)
    assert A[s - 1] == pytest.approx(h * h / 6, rel=1e-6)


def test_single_cell_centroid_is_the_surface_centroid():
    """One cell: its centroid is the centre of mass of the piecewise-flat
    surface, sum over triangles of area x (mean of the corners) / total area
    (the centroid of a triangle is the mean of its corners); (1/2, 1/2, 0)
    on the unit square."""
    for m in (I.flat_grid(40), I.bumpy_icosphere(level=3, seed=2, n_sources=1)):
        lab = np.zeros(m.n, np.int32)
        _, cen = OC.lloyd_step(m.V, m.F, lab, np.array([0], np.int32))
        X = m.V.astype(np.float64)
        T = X[m.F]
        ar = 0.5 * np.linalg.norm(np.cross(T[:, 1] - T[:, 0], T[:, 2] - T[:, 0]), axis=1)
        ref = (ar[:, None] * T.mean(axis=1)).sum(axis=0) / ar.sum()
        assert np.allclose(cen[0], ref, rtol=0, atol=1e-13)
    g = I.flat_grid(40)
    _, cen = OC.lloyd_step(g.V, g.F, np.zeros(g.n, np.int32), np.array([0], np.int32))
    assert np.allclose(cen[0], [0.5, 0.5, 0.0], atol=1e-7)


def test_lloyd_on_the_plane_reaches_the_quadrants():
    """Four generators on the unit square: the centroidal tessellation is the
    four quadrants with generators at (1/4, 1/4), ... (geodesic = Euclidean
    on a plane up to the scheme's O(h) error); the energy sum A d^2 falls."""
    m = I.flat_grid(64)
    sets, en = OC.lloyd(m.V, m.F, np.array([5, 70, 200, 300], np.int32), 12, 1e-6)
    X = m.V.astype(np.float64)[sets[-1], :2]
    quads = np.array([[0.25, 0.25], [0.75, 0.25], [0.25, 0.75], [0.75, 0.75]])
    dmin = np.min(np.linalg.norm(X[:, None, :] - quads[None], axis=2), axis=0)
    assert (dmin < 0.03).all()
    assert all(b <= a * (1 + 1e-12) for a, b in zip(en, en[1:]))


def test_lloyd_step_picks_the_nearest_cell_vertex():
    m = I.bumpy_icosphere(level=3, seed=5, n_sources=6)
    r = O.run(m.V, m.F, m.S, 1e-6)
    S2, cen = OC.lloyd_step(m.V, m.F, r.label, m.S)
    X = m.V.astype(np.float64)
    for s in range(m.m):
        cell = np.nonzero(r.label == s)[0]
        d = np.linalg.norm(X[cell] - cen[s], axis=1)
        assert S2[s] == cell[np.argmin(d)]
        assert r.label[S2[s]] == s
