"""The band trace derived from a retirement record equals the band the oracle
actually used (its own per-iteration trace), for the paper's rule, a window
and the fixed half band; the update count follows."""
import numpy as np
import pytest

import oracle as O
from paper_1810_08218_amd import diagnostics as D
from paper_1810_08218_amd import inputs as I


@pytest.mark.parametrize("kw", [{}, {"window": 3}, {"band_rule": 1}])
def test_band_trace_matches_oracle(kw):
    m = I.bumpy_icosphere(level=4, seed=3, n_sources=5)
    r = O.run(m.V, m.F, m.S, 1e-4, **kw)
    _, _, offsets, rho = O.toplesets(m.V, m.F, m.S)
    t = D.band_trace(r.retire_k, offsets, r.iterations)
    assert t["lo"].tolist() == r.trace_lo[1:].tolist()
    assert D.updates(r.retire_k, offsets, r.iterations) == r.updates
    assert (t["toplesets"] >= 1).all()
