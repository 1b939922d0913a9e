"""Pins of the oracle's planar update (paper Sec. 3.2, update_step) against
closed forms and properties fixed by the mathematics, not by the oracle."""
import math

import numpy as np
import pytest

import oracle as O
from meshtools import golden


def _frame(rng):
    """Random orthonormal in-plane frame (u, w) of a random plane in 3D."""
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    return q[:, 0], q[:, 1]


def _tri(rng, obtuse_ok=True):
    u, w = _frame(rng)
    origin = rng.normal(size=3)
    while True:
        p = rng.uniform(-1, 1, size=(3, 2))
        a = p[1] - p[0]
        b = p[2] - p[0]
        area = abs(a[0] * b[1] - a[1] * b[0]) / 2
        if area > 0.05:
            break
    pts = [origin + pp[0] * u + pp[1] * w for pp in p]
    return pts, u, w


@pytest.mark.parametrize("case", golden("local_update_closed_forms.json")["cases"],
                         ids=lambda c: c["name"])
def test_closed_forms(case):
    d2 = float(case["d2"]) if case["d2"] != "inf" else math.inf
    p, _ = O.local_update(case["x0"], case["x1"], case["x2"], case["d1"], d2)
    assert p == pytest.approx(case["expected"], rel=1e-13, abs=1e-13)


def test_both_infinite():
    p, who = O.local_update([0, 0, 0], [1, 0, 0], [0, 1, 0], math.inf, math.inf)
    assert math.isinf(p) and who == -1


def test_plane_wave_exact_when_upwind():
    """Inputs sampled from a unit-gradient in-plane linear field whose
    characteristic reaches x0 through the opposite edge reproduce the field
    at x0 (the update is exact for plane fronts)."""
    rng = np.random.default_rng(11)
    worst = 0.0
    for _ in range(3000):
        (x0, x1, x2), u, w = _tri(rng)
        t = rng.uniform(0.05, 0.95)
        y = (1 - t) * x1 + t * x2               # foot of the characteristic on edge x1x2
        n = x0 - y
        if np.linalg.norm(n) < 1e-3:
            continue
        n /= np.linalg.norm(n)
        c0 = rng.uniform(-5, 5) + 10.0
        d1, d2 = n @ x1 + c0, n @ x2 + c0
        p, _ = O.local_update(x0, x1, x2, d1, d2)
        worst = max(worst, abs(p - (n @ x0 + c0)))
    assert worst < 1e-10


def test_symmetric_in_the_two_inputs():
    rng = np.random.default_rng(12)
    for _ in range(2000):
        (x0, x1, x2), _, _ = _tri(rng)
        d1, d2 = rng.uniform(0, 3, size=2)
        a, _ = O.local_update(x0, x1, x2, d1, d2)
        b, _ = O.local_update(x0, x2, x1, d2, d1)
        assert a == pytest.approx(b, rel=1e-12, abs=1e-12)


def test_never_above_edge_updates_and_shift_scale():
    rng = np.random.default_rng(13)
    for _ in range(2000):
        (x0, x1, x2), _, _ = _tri(rng)
        d1, d2 = rng.uniform(0, 3, size=2)
        p, _ = O.local_update(x0, x1, x2, d1, d2)
        pedge = min(d1 + np.linalg.norm(x1 - x0), d2 + np.linalg.norm(x2 - x0))
        assert p <= pedge + 1e-12
        c = rng.uniform(-1, 5)
        q, _ = O.local_update(x0, x1, x2, d1 + c, d2 + c)
        assert q == pytest.approx(p + c, rel=1e-11, abs=1e-11)
        lam = rng.uniform(0.1, 10)
        r, _ = O.local_update(lam * x0, lam * x1, lam * x2, lam * d1, lam * d2)
        assert r == pytest.approx(lam * p, rel=1e-11, abs=1e-11)


def test_monotone_with_unit_total_slope():
    """dU/dd_i lies in [0, 1]; where the planar value is used the two slopes
    add up to 1 (the value moves with a common shift of both inputs)."""
    rng = np.random.default_rng(14)
    h = 1e-6
    planar = 0
    for _ in range(2000):
        (x0, x1, x2), _, _ = _tri(rng)
        d1, d2 = rng.uniform(0, 3, size=2)
        p, _ = O.local_update(x0, x1, x2, d1, d2)
        g1 = (O.local_update(x0, x1, x2, d1 + h, d2)[0] - O.local_update(x0, x1, x2, d1 - h, d2)[0]) / (2 * h)
        g2 = (O.local_update(x0, x1, x2, d1, d2 + h)[0] - O.local_update(x0, x1, x2, d1, d2 - h)[0]) / (2 * h)
        assert -1e-6 <= g1 <= 1 + 1e-6 and -1e-6 <= g2 <= 1 + 1e-6
        pedge = min(d1 + np.linalg.norm(x1 - x0), d2 + np.linalg.norm(x2 - x0))
        if p < pedge - 1e-6:
            planar += 1
            assert g1 + g2 == pytest.approx(1.0, abs=1e-5)
            assert g1 > 0 and g2 > 0
    assert planar > 200


def test_acute_triangle_accepts_planar_between_edges():
    """Equal inputs on an acute triangle: the front is parallel to x1x2 and
    the value is d + height (the foot of the height lies inside the edge)."""
    rng = np.random.default_rng(15)
    for _ in range(500):
        (x0, x1, x2), _, _ = _tri(rng)
        e = x2 - x1
        t = np.dot(x0 - x1, e) / np.dot(e, e)
        if not (0.05 < t < 0.95):
            continue
        height = np.linalg.norm(x0 - (x1 + t * e))
        d = rng.uniform(0, 4)
        p, _ = O.local_update(x0, x1, x2, d, d)
        assert p == pytest.approx(d + height, rel=1e-12, abs=1e-12)
