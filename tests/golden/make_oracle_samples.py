"""Write the stored oracle values the GPU tests compare against for meshes the
oracle is too slow to run inside a test.  Calls only ``oracle``, the input
generators and scipy (for the Dijkstra distances that define a warm-start
bound both sides can compute); uses the OpenMP build of the oracle, whose
results are bit-identical to the sequential one.

    python tests/golden/make_oracle_samples.py [name ...]

Files (tests/golden/):
  bumpy_icosphere9_oracle_samples.npz   level-9 bumpy icosphere, 32 sources,
      tol 1e-4: distances at 20,000 sampled vertices, K, rho, U and the
      retirement schedule
  bumpy_icosphere9_warm_dijkstra.npz    the same mesh without labels, started
      from float32(1.05 x Dijkstra distance): sampled distances, K, U, schedule
  batch_largest_oracle_samples.npz      the largest jittered grid (t = 95) and
      the largest torus (t = 262) of the 512-mesh batch, tol 1e-4
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import oracle as O  # noqa: E402
from meshtools import dijkstra  # noqa: E402
from paper_1810_08218_amd import inputs as I  # noqa: E402

N_SAMPLES = 20000
BATCH_LARGEST = (95, 262)


def _sample(n, seed=12345, k=N_SAMPLES):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, min(k, n), replace=False)).astype(np.int64)


def bumpy9():
    lib = O.load_omp()
    m = I.bumpy_icosphere(level=9, seed=3, n_sources=32)
    tol = 1e-4
    r = O.run(m.V, m.F, m.S, tol, lib=lib)
    idx = _sample(m.n)
    out = os.path.join(HERE, "bumpy_icosphere9_oracle_samples.npz")
    np.savez_compressed(
        out, idx=idx, dist=r.dist[idx], iterations=np.int64(r.iterations), rho=np.int64(r.rho),
        updates=np.int64(r.updates), status=np.int64(r.status), retire_k=r.retire_k,
        trace_maxrel=r.trace_maxrel, tol=np.float64(tol),
        dist_max=np.float64(np.max(r.dist[np.isfinite(r.dist)])), dist_sum=np.float64(np.sum(r.dist)))
    print(out, r.iterations, r.rho, r.updates, flush=True)


def warm_bound(m):
    """float32(1.05 x Dijkstra distance): an upper bound of the fixed point
    (the Dijkstra distance D satisfies D >= U(D) since the planar update never
    exceeds an edge update, and so does 1.05 D)."""
    return (1.05 * dijkstra(m.V, m.F, m.S)).astype(np.float32)


def bumpy9_warm():
    lib = O.load_omp()
    m = I.bumpy_icosphere(level=9, seed=3, n_sources=32)
    tol = 1e-4
    up = warm_bound(m)
    r = O.run_warm(m.V, m.F, m.S, tol, up.astype(np.float64), lib=lib)
    idx = _sample(m.n, seed=777)
    out = os.path.join(HERE, "bumpy_icosphere9_warm_dijkstra.npz")
    np.savez_compressed(out, idx=idx, dist=r.dist[idx], iterations=np.int64(r.iterations),
                        rho=np.int64(r.rho), updates=np.int64(r.updates), status=np.int64(r.status),
                        retire_k=r.retire_k, rejected=np.int64(r.rejected), tol=np.float64(tol))
    print(out, r.iterations, r.rho, r.updates, r.rejected, flush=True)


def batch_largest():
    lib = O.load_omp()
    tol = 1e-4
    rec = {"tol": np.float64(tol), "ts": np.array(BATCH_LARGEST, np.int64)}
    for t in BATCH_LARGEST:
        m = I.batch_mesh(t)
        r = O.run(m.V, m.F, m.S, tol, lib=lib)
        idx = _sample(m.n, seed=1000 + t)
        rec[f"t{t}_n"] = np.int64(m.n)
        rec[f"t{t}_idx"] = idx
        rec[f"t{t}_dist"] = r.dist[idx]
        rec[f"t{t}_iterations"] = np.int64(r.iterations)
        rec[f"t{t}_rho"] = np.int64(r.rho)
        rec[f"t{t}_updates"] = np.int64(r.updates)
        rec[f"t{t}_status"] = np.int64(r.status)
        rec[f"t{t}_retire_k"] = r.retire_k
        rec[f"t{t}_trace_maxrel"] = r.trace_maxrel
        print(t, m.n, r.iterations, r.rho, r.updates, flush=True)
    out = os.path.join(HERE, "batch_largest_oracle_samples.npz")
    np.savez_compressed(out, **rec)
    print(out, flush=True)


JOBS = {"bumpy9": bumpy9, "bumpy9_warm": bumpy9_warm, "batch_largest": batch_largest}

if __name__ == "__main__":
    for name in (sys.argv[1:] or list(JOBS)):
        JOBS[name]()
