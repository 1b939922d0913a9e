"""Write the stored oracle values the GPU tests compare against for meshes the
oracle is too slow to run inside a test (the level-9 bumpy icosphere with 32
sources: about 90 s single-threaded).  Calls only ``oracle`` and the input
generators.

    python tests/golden/make_oracle_samples.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1810_08218_amd import inputs as I  # noqa: E402

N_SAMPLES = 20000


def main():
    m = I.bumpy_icosphere(level=9, seed=3, n_sources=32)
    tol = 1e-4
    r = O.run(m.V, m.F, m.S, tol)
    rng = np.random.default_rng(12345)
    idx = np.sort(rng.choice(m.n, N_SAMPLES, replace=False)).astype(np.int64)
    out = os.path.join(HERE, "bumpy_icosphere9_oracle_samples.npz")
    np.savez_compressed(
        out,
        idx=idx,
        dist=r.dist[idx],
        label=r.label[idx],
        iterations=np.int64(r.iterations),
        rho=np.int64(r.rho),
        updates=np.int64(r.updates),
        status=np.int64(r.status),
        retire_k=r.retire_k,
        trace_maxrel=r.trace_maxrel,
        tol=np.float64(tol),
        dist_max=np.float64(np.max(r.dist[np.isfinite(r.dist)])),
        dist_sum=np.float64(np.sum(r.dist)),
    )
    print(out, r.iterations, r.rho, r.updates)


if __name__ == "__main__":
    main()
