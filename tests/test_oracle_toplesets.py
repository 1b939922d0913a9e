"""Pins of the oracle's toplesets (paper Sec. 4.1 definition of V_r) and of
the canonical order (Sec. 4.3 reorder; ascending id inside a topleset)
against scipy's BFS and closed forms."""
import numpy as np
import pytest

import oracle as O
from meshtools import bfs_levels, canonical_order, golden
from paper_1810_08218_amd import inputs as I


def _cases():
    out = [I.flat_grid(64), I.flat_grid(17, source=(8, 8)), I.sphere(3, seed=5, n_sources=1),
           I.sphere(4, seed=6, n_sources=7), I.bumpy_icosphere(level=4, seed=9, n_sources=5)]
    for t in (0, 3, 300, 301):
        out.append(I.batch_mesh(t))
    return out


@pytest.mark.parametrize("mesh", _cases(), ids=lambda m: m.name)
def test_levels_and_order_match_scipy_bfs(mesh):
    level, order, offsets, rho = O.toplesets(mesh.V, mesh.F, mesh.S)
    ref = bfs_levels(mesh.V, mesh.F, mesh.S)
    assert np.array_equal(level, ref)
    assert rho == ref.max() + 1
    assert np.array_equal(order, canonical_order(ref))
    sizes = np.bincount(ref[ref >= 0], minlength=rho)
    assert np.array_equal(np.diff(offsets), sizes)
    # partition: every reachable vertex in exactly one topleset (Sec. 4.1 properties)
    assert offsets[-1] == (ref >= 0).sum()
    assert len(set(order.tolist())) == mesh.n


def test_grid_closed_form():
    s = 64
    m = I.flat_grid(s)
    level, order, offsets, rho = O.toplesets(m.V, m.F, m.S)
    i = np.arange(s * s) % s
    j = np.arange(s * s) // s
    assert np.array_equal(level, np.maximum(i, j))          # diagonal (i,j)->(i+1,j+1)
    assert rho == 64
    assert np.array_equal(np.diff(offsets), 2 * np.arange(64) + 1)


def test_unreachable_component_goes_last():
    g = I.flat_grid(8)
    V2 = np.concatenate([g.V, g.V + np.float32(5.0)])
    F2 = np.concatenate([g.F, g.F + 64]).astype(np.int32)
    level, order, offsets, rho = O.toplesets(V2, F2, np.array([3], np.int32))
    assert (level[64:] == -1).all() and (level[:64] >= 0).all()
    assert np.array_equal(order[64:], np.arange(64, 128))
    assert offsets[-1] == 64


def test_golden_square():
    g = golden("square_antidiagonal.json")
    level, _, _, rho = O.toplesets(np.array(g["V"], np.float32), np.array(g["F"], np.int32),
                                   np.array(g["S"], np.int32))
    assert level.tolist() == g["expected_level"] and rho == g["expected_rho"]


def test_invalid_inputs_raise():
    g = I.flat_grid(4)
    bad = g.F.copy()
    bad[0, 0] = 99
    with pytest.raises(ValueError):
        O.toplesets(g.V, bad, g.S)
    with pytest.raises(ValueError):
        O.toplesets(g.V, g.F, np.array([0, 0], np.int32))
    with pytest.raises(ValueError):
        O.toplesets(g.V, g.F, np.array([16], np.int32))
