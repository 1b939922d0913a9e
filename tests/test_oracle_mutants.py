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
    "window lower end one below": ("j - opt->window + 1 > lo) {\n            lo = j - opt->window + 1;",
                                   "j - opt->window > lo) {\n            lo = j - opt->window;"),
    "window push-out recorded one late": ("for (int r = i; r < lo; ++r) retire_k[r] = k - 1;",
                                          "for (int r = i; r < lo; ++r) retire_k[r] = k;"),
    "fixed band lower end floor(k/2)": ("lo = (k + 1) / 2;                            /* fixed half band */",
                                        "lo = k / 2;"),
    "fixed band runs 2 rho - 1 iterations": ("const int kfix = 2 * rho - 3 > 1 ? 2 * rho - 3 : 1;",
                                             "const int kfix = 2 * rho - 1 > 1 ? 2 * rho - 1 : 1;"),
    "parent tie to the larger id": ("if (u < bu || (u == bu && g < bg)) {", "if (u < bu || (u == bu && g > bg)) {"),
    "parent from the first triangle": ("if (u < bu || (u == bu && g < bg)) {", "if (bg < 0) {"),
    "replay drops a topleset in its retiring iteration": (
        "while (lo < rho && replay[lo] >= 0 && replay[lo] < k) lo++;",
        "while (lo < rho && replay[lo] >= 0 && replay[lo] <= k) lo++;"),
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

    def ladder():
        g = golden("ladder_window_and_fixed_band.json")
        V, F, S = (np.array(g[k], t) for k, t in (("V", np.float32), ("F", np.int32), ("S", np.int32)))
        for c in g["runs"].values():
            r = O.run(V, F, S, g["tol"], window=c["window"], band_rule=c["band_rule"], lib=lib)
            if (r.iterations, r.updates) != (c["K"], c["U"]) or r.retire_k.tolist() != c["retire"]:
                return False
            if r.trace_lo[1:].tolist() != c["lo"]:
                return False
        return True

    mb = I.bumpy_icosphere(level=4, seed=3, n_sources=6)

    def replay():
        for kw in ({}, {"window": 3}, {"band_rule": 1}):
            r = O.run(mb.V, mb.F, mb.S, 1e-4, lib=lib, **kw)
            p = O.replay(mb.V, mb.F, mb.S, 1e-4, r.retire_k, r.iterations, lib=lib)
            if not (np.array_equal(p.dist, r.dist) and p.updates == r.updates):
                return False
        return True

    mt = I.batch_mesh(263)

    def parents():
        from test_oracle_ptp import _brute_parents
        r = O.run(mt.V, mt.F, mt.S, 1e-4, lib=lib)
        lab, par = O.labels_from_map(mt.V, mt.F, mt.S, r.dist, lib=lib)
        bp, bl = _brute_parents(mt.V, mt.F, mt.S, r.dist)
        return np.array_equal(par, bp) and np.array_equal(lab, bl) and np.array_equal(r.label, lab)

    check("closed forms", closed_forms)
    check("parents", parents)
    check("ladder schedules", ladder)
    check("replay", replay)
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
