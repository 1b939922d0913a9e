"""Plant a plausible mistake in a copy of the oracle (on the CPU) and check
that the pins catch it: every mutant below must fail at least one pin of the
battery, while the unmodified source passes them all."""
import math
import os

import numpy as np
import pytest

import oracle as O
from meshtools import bfs_levels, canonical_order, golden
from paper_1810_08218_amd import inputs as I

MUTANTS = {
    "smaller root": ("double p = (s1t + sqrt(disc)) / s11;", "double p = (s1t - sqrt(disc)) / s11;"),
    "no monotonicity test": ("if (al1 < 0.0 && al2 < 0.0) {", "if (1) {"),
    "monotonicity sign flipped": ("if (al1 < 0.0 && al2 < 0.0) {", "if (al1 > 0.0 && al2 > 0.0) {"),
    "Q entry transposed": ("double al1 = q11 * r1 + q12 * r2;", "double al1 = q11 * r1 + q22 * r2;"),
    "dropped constant in discriminant": ("double disc = s1t * s1t - s11 * (stt - 1.0);",
                                         "double disc = s1t * s1t - s11 * stt;"),
    "band upper end one ahead": ("int j = k < rho ? k : rho - 1;                   /* Eq. upper_band */",
                                 "int j = k + 1 < rho ? k + 1 : rho - 1;"),
    "BFS level step of two": ("level[u] = level[v] + 1;", "level[u] = level[v] + 2;"),
    "order inside topleset reversed": ("for (int v = 0; v < n; ++v) {\n        int b = level[v] < 0 ? rho : level[v];\n        order[count[b]++] = v;",
                                       "for (int v = n - 1; v >= 0; --v) {\n        int b = level[v] < 0 ? rho : level[v];\n        order[count[b]++] = v;"),
    "label tie to larger index": ("else *lab_out = l1 < l2 ? l1 : l2;\n        return p;",
                                  "else *lab_out = l1 > l2 ? l1 : l2;\n        return p;"),
    "retire without the relative test": ("if (!(rel < opt->tol)) ok = 0;", "(void)0;"),
}


def _battery(lib) -> list:
    """Returns the names of the pins that fail for this oracle build."""
    failed = []

    def check(name, fn):
        try:
            if not fn():
                failed.append(name)
        except Exception:  # a crash in a mutant counts as caught
            failed.append(name)

    def closed_forms():
        for c in golden("local_update_closed_forms.json")["cases"]:
            d2 = float(c["d2"]) if c["d2"] != "inf" else math.inf
            p, _ = O.local_update(c["x0"], c["x1"], c["x2"], c["d1"], d2, lib=lib)
            if not math.isclose(p, c["expected"], rel_tol=1e-12, abs_tol=1e-12):
                return False
        return True

    def plane_wave():
        rng = np.random.default_rng(1)
        for _ in range(300):
            x0, x1, x2 = rng.normal(size=(3, 3))
            t = rng.uniform(0.1, 0.9)
            n = x0 - ((1 - t) * x1 + t * x2)
            n /= np.linalg.norm(n)
            p, _ = O.local_update(x0, x1, x2, n @ x1 + 7, n @ x2 + 7, lib=lib)
            if abs(p - (n @ x0 + 7)) > 1e-9:
                return False
        return True

    def squares():
        for name in ("square_antidiagonal.json", "square_two_sources.json",
                     "triangle_two_sources.json"):
            g = golden(name)
            r = O.run(np.array(g["V"], np.float32), np.array(g["F"], np.int32),
                      np.array(g["S"], np.int32), g["tol"], lib=lib)
            if not np.allclose(r.dist, g["expected_dist"], rtol=1e-13):
                return False
            if (r.iterations, r.updates) != (g["expected_K"], g["expected_U"]):
                return False
            if "expected_label" in g and r.label.tolist() != g["expected_label"]:
                return False
        return True

    m = I.flat_grid(24)
    ms = I.sphere(3, seed=2, n_sources=3)

    def grid_rays():
        r = O.run(m.V, m.F, m.S, 1e-6, lib=lib)
        X = m.V.astype(np.float64)
        eu = np.linalg.norm(X - X[0], axis=1)
        i, j = np.arange(m.n) % 24, np.arange(m.n) // 24
        ray = (i == 0) | (j == 0) | (i == j)
        return (np.allclose(r.dist[ray], eu[ray], rtol=1e-12) and (r.dist >= eu - 1e-12).all()
                and r.rho <= r.iterations <= 2 * r.rho - 1)

    def bfs():
        level, order, _, _ = O.toplesets(ms.V, ms.F, ms.S, lib=lib)
        ref = bfs_levels(ms.V, ms.F, ms.S)
        return np.array_equal(level, ref) and np.array_equal(order, canonical_order(ref))

    def fixed_point_bounds():
        r = O.run(ms.V, ms.F, ms.S, 1e-6, lib=lib)
        fp, _, _ = O.fixed_point(ms.V, ms.F, ms.S, lib=lib)
        from meshtools import dijkstra
        dj = dijkstra(ms.V, ms.F, ms.S)
        close = np.abs(r.dist - fp).max() <= 1e-5 * fp.max()
        return (fp <= dj * (1 + 1e-12)).all() and (r.dist >= fp * (1 - 1e-12)).all() and close

    check("closed forms", closed_forms)
    check("plane wave", plane_wave)
    check("golden squares", squares)
    check("grid rays", grid_rays)
    check("bfs", bfs)
    check("fixed point bounds", fixed_point_bounds)
    return failed


def test_unmodified_oracle_passes_battery():
    assert _battery(O._L()) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = O.source_text()
    assert src.count(old) == 1, f"mutation anchor not found once: {name}"
    path = O.build_variant(src.replace(old, new), os.path.join(str(tmp_path), "mutant.so"))
    lib = O.load_library(path)
    assert _battery(lib), f"no pin caught the mutant '{name}'"
