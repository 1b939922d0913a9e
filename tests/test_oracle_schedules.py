"""Pins of the oracle's band schedules (paper Sec. 4.2, Eq. upper_band and Eq.
lower_band; the fixed half band of Sec. 6; the library's window cap) and of
its replay mode, which re-runs the iteration under a given schedule."""
import numpy as np
import pytest

import oracle as O
from meshtools import golden
from paper_1810_08218_amd import inputs as I


def _ladder():
    g = golden("ladder_window_and_fixed_band.json")
    return g, np.array(g["V"], np.float32), np.array(g["F"], np.int32), np.array(g["S"], np.int32)


def _recursion_row1():
    """(r, 1) of the ladder: D(1) = sqrt2, D(r) = D(r-1) + sqrt(1 - (D(r-1) - (r-1))^2)
    (the plane front through (r-1, 0) and (r-1, 1), derived in the fixture)."""
    D = [1.0, np.sqrt(2.0)]
    for r in range(2, 6):
        D.append(D[-1] + np.sqrt(1.0 - (D[-1] - (r - 1)) ** 2))
    return np.array(D)


@pytest.mark.parametrize("run", ["unbounded", "window1", "window2", "fixed_half_band"])
def test_ladder_golden(run):
    g, V, F, S = _ladder()
    c = g["runs"][run]
    r = O.run(V, F, S, g["tol"], window=c["window"], band_rule=c["band_rule"])
    _, _, offsets, rho = O.toplesets(V, F, S)
    assert rho == g["expected_rho"] and np.diff(offsets).tolist() == g["expected_sizes"]
    assert r.status == O.OK
    assert (r.iterations, r.updates) == (c["K"], c["U"])
    assert r.retire_k.tolist() == c["retire"]
    assert r.trace_lo[1:].tolist() == c["lo"]
    assert np.array_equal(r.dist[:6], g["expected_dist_row0"])
    assert np.allclose(r.dist[6:], _recursion_row1(), rtol=1e-15, atol=0)


def test_fixed_band_reaches_fixed_point_on_regular_grids():
    """Sec. 6: on a regular valence-6 mesh whose toplesets grow monotonically,
    V_r is final after 2r - 1 Jacobi iterations, so the half band
    [floor((k+1)/2), k] run for 2 rho - 3 iterations gives the fixed point."""
    for m in (I.flat_grid(64), I.flat_grid(37, source=(20, 11))):
        fp, _, _ = O.fixed_point(m.V, m.F, m.S)
        r = O.run(m.V, m.F, m.S, 1e-6, band_rule=1)
        assert r.status == O.OK and r.iterations == 2 * r.rho - 3
        assert np.array_equal(r.dist, fp)


def test_fixed_band_schedule_formula():
    """Any mesh: band [max(1, floor((k+1)/2)), min(k, rho-1)], K = 2 rho - 3,
    V_r last updated at min(2r, K), U the sum of the band sizes."""
    m = I.noisy_icosphere(level=4, seed=21)
    r = O.run(m.V, m.F, m.S, 1e-4, band_rule=1)
    _, _, offsets, rho = O.toplesets(m.V, m.F, m.S)
    K = 2 * rho - 3
    assert r.iterations == K
    lo = [max(1, (k + 1) // 2) for k in range(1, K + 1)]
    assert r.trace_lo[1:].tolist() == lo
    U = sum(offsets[min(k, rho - 1) + 1] - offsets[lo[k - 1]] for k in range(1, K + 1))
    assert r.updates == U
    assert r.retire_k.tolist() == [0] + [min(2 * q, K) for q in range(1, rho)]
    fp, _, _ = O.fixed_point(m.V, m.F, m.S)
    assert (r.dist >= fp * (1 - 1e-12)).all()


def test_window_caps_the_band():
    """With a cap W the band [lo, j] never holds more than W toplesets, a cap at
    least rho changes nothing, and a smaller one keeps results at or above the
    fixed point."""
    m = I.noisy_icosphere(level=5, seed=7)
    ref = O.run(m.V, m.F, m.S, 1e-4)
    fp, _, _ = O.fixed_point(m.V, m.F, m.S)
    big = O.run(m.V, m.F, m.S, 1e-4, window=ref.rho)
    assert np.array_equal(big.dist, ref.dist) and np.array_equal(big.retire_k, ref.retire_k)
    for W in (1, 2, 3, 6):
        r = O.run(m.V, m.F, m.S, 1e-4, window=W)
        ks = np.arange(1, r.iterations + 1)
        j = np.minimum(ks, r.rho - 1)
        assert (j - r.trace_lo[1:] + 1 <= W).all()
        assert (r.dist >= fp * (1 - 1e-12)).all()


def _replay_same(m, tol, **kw):
    r = O.run(m.V, m.F, m.S, tol, **kw)
    p = O.replay(m.V, m.F, m.S, tol, r.retire_k, r.iterations)
    assert p.status == r.status
    assert (p.iterations, p.updates, p.rho) == (r.iterations, r.updates, r.rho)
    assert np.array_equal(p.dist, r.dist) and np.array_equal(p.label, r.label)
    assert np.array_equal(p.retire_k, r.retire_k)
    return r


def test_replay_reproduces_each_rule():
    """Replaying a run's own schedule gives that run bit for bit: the paper's
    rule, a window, the iteration cap (ENOCONV) and the fixed half band."""
    m = I.bumpy_icosphere(level=4, seed=3, n_sources=6)
    _replay_same(m, 1e-4)
    _replay_same(m, 1e-4, window=3)
    r = _replay_same(m, 1e-4, max_iters=7)
    assert r.status == O.ENOCONV
    _replay_same(m, 1e-4, band_rule=1)
    g, V, F, S = _ladder()
    from types import SimpleNamespace
    _replay_same(SimpleNamespace(V=V, F=F, S=S), g["tol"], window=1)


def test_replay_under_another_schedule_changes_only_the_band():
    """Replay of the fixed half band's schedule equals the fixed-band run, and
    a schedule that retires a topleset before its first update is refused."""
    m = I.noisy_icosphere(level=4, seed=21)
    fb = O.run(m.V, m.F, m.S, 1e-4, band_rule=1)
    p = O.replay(m.V, m.F, m.S, 1e-4, fb.retire_k, fb.iterations)
    assert np.array_equal(p.dist, fb.dist) and p.updates == fb.updates
    bad = fb.retire_k.copy()
    bad[1] = 0
    with pytest.raises(ValueError):
        O.replay(m.V, m.F, m.S, 1e-4, bad, fb.iterations)


def test_openmp_build_gives_identical_results():
    """The OpenMP build parallelises only the Jacobi update of a band, whose
    vertices read the previous map only: results are bit-identical."""
    m = I.bumpy_icosphere(level=5, seed=3, n_sources=8)
    a = O.run(m.V, m.F, m.S, 1e-4)
    b = O.run(m.V, m.F, m.S, 1e-4, lib=O.load_omp())
    assert np.array_equal(a.dist, b.dist) and np.array_equal(a.label, b.label)
    assert np.array_equal(a.retire_k, b.retire_k) and a.updates == b.updates
