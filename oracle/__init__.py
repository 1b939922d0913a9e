"""CPU FP64 oracle for PTP: ctypes wrapper around ``ptp_oracle.c``.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares nothing with
the HIP library; the shared library it loads is built from ``ptp_oracle.c``
alone by ``oracle.build_oracle()`` (plain gcc).

All functions take numpy arrays: V float32 [n, 3] (promoted exactly to
float64 here), F int32 [f, 3], S int32 [m].
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ptp_oracle.c")
_LIB = os.path.join(_HERE, "libptp_oracle.so")
_LIB_OMP = os.path.join(_HERE, "libptp_oracle_omp.so")

OK, EINVAL, ENOMEM, ENOCONV = 0, -1, -2, -4


def _compile(out: str, extra: list, force: bool) -> str:
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
                               *extra, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, out)
    return out


def build_oracle(force: bool = False) -> str:
    """Compile ptp_oracle.c into libptp_oracle.so next to it (gcc -O3,
    sequential) and libptp_oracle_omp.so (the same source with its one
    OpenMP loop, the Jacobi update of a band, on all host cores)."""
    _compile(_LIB_OMP, ["-fopenmp"], force)
    return _compile(_LIB, ["-Wno-unknown-pragmas"], force)


class _Opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iters", C.c_int), ("band_rule", C.c_int),
                ("window", C.c_int)]


class _Stats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("rho", C.c_int), ("reachable", C.c_int),
                ("updates", C.c_longlong)]


_lib = None
_lib_omp = None


def load_omp() -> C.CDLL:
    """The OpenMP build (same results, band updates on every host core)."""
    global _lib_omp
    if _lib_omp is None:
        build_oracle()
        _lib_omp = load_library(_LIB_OMP)
    return _lib_omp


def load_library(path: str) -> C.CDLL:
    """Load an oracle build (the default one, or a variant compiled by a test)
    and declare its signatures."""
    lib = C.CDLL(path)
    _declare(lib)
    return lib


def build_variant(c_source: str, out_path: str) -> str:
    """Compile a modified copy of the oracle source (used by the tests that
    plant a mistake in the oracle to show the pins catch it)."""
    src = out_path + ".c"
    with open(src, "w") as fh:
        fh.write(c_source)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", out_path, src, "-lm"])
    return out_path


def source_text() -> str:
    with open(_SRC) as fh:
        return fh.read()


def _L(lib=None):
    global _lib
    if lib is not None:
        return lib
    if _lib is None:
        build_oracle()
        _lib = load_library(_LIB)
    return _lib


def _declare(lib):
    P = np.ctypeslib.ndpointer
    dptr = P(np.float64, flags="C")
    iptr = P(np.int32, flags="C")
    lib.ptpo_toplesets.argtypes = [C.c_int, C.c_int, iptr, C.c_int, iptr, iptr, iptr, iptr,
                                   C.POINTER(C.c_int)]
    lib.ptpo_local_update.argtypes = [dptr, dptr, dptr, C.c_double, C.c_double,
                                      C.POINTER(C.c_int)]
    lib.ptpo_local_update.restype = C.c_double
    lib.ptpo_run.argtypes = [C.c_int, C.c_int, dptr, iptr, C.c_int, iptr, C.POINTER(_Opts),
                             dptr, iptr, C.POINTER(_Stats), iptr, iptr, dptr, C.c_int]
    lib.ptpo_run_replay.argtypes = [C.c_int, C.c_int, dptr, iptr, C.c_int, iptr, C.POINTER(_Opts),
                                    iptr, C.c_int, dptr, iptr, C.POINTER(_Stats), iptr]
    lib.ptpo_run_warm.argtypes = [C.c_int, C.c_int, dptr, iptr, C.c_int, iptr, C.POINTER(_Opts),
                                  dptr, C.c_int, dptr, iptr, C.POINTER(_Stats), iptr,
                                  C.POINTER(C.c_int), dptr]
    lib.ptpo_fixed_point.argtypes = [C.c_int, C.c_int, dptr, iptr, C.c_int, iptr, C.c_int,
                                     dptr, iptr, C.POINTER(C.c_int)]
    lib.ptpo_fast_marching.argtypes = [C.c_int, C.c_int, dptr, iptr, C.c_int, iptr, dptr]
    lib.ptpo_labels_from_map.argtypes = [C.c_int, C.c_int, dptr, iptr, C.c_int, iptr, dptr, iptr, iptr]


def _prep(V, F, S):
    X = np.ascontiguousarray(np.asarray(V, dtype=np.float32), dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.int32)
    S = np.ascontiguousarray(S, dtype=np.int32)
    return X, F, S


def local_update(x0, x1, x2, d1, d2, lib=None):
    """Planar update of x0 from (x1, d1), (x2, d2).  Returns (value, who):
    who = 1 or 2 when the result is the edge update through x1 / x2 (or a
    planar solution whose smaller input is that vertex), -1 when both inputs
    are infinite."""
    lab = C.c_int(0)
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (x0, x1, x2)]
    p = _L(lib).ptpo_local_update(a[0], a[1], a[2], float(d1), float(d2), C.byref(lab))
    return p, lab.value


def toplesets(V, F, S, lib=None):
    """Returns (level[n], order[n], offsets[rho + 1], rho)."""
    _, F, S = _prep(V, F, S)
    n = int(np.asarray(V).shape[0])
    level = np.empty(n, np.int32)
    order = np.empty(n, np.int32)
    offsets = np.empty(n + 2, np.int32)
    rho = C.c_int(0)
    rc = _L(lib).ptpo_toplesets(n, F.shape[0], F, S.shape[0], S, level, order, offsets,
                             C.byref(rho))
    if rc != OK:
        raise ValueError(f"ptpo_toplesets failed: {rc}")
    return level, order, offsets[: rho.value + 1].copy(), rho.value


@dataclass
class Result:
    dist: np.ndarray
    label: np.ndarray
    status: int
    iterations: int
    rho: int
    reachable: int
    updates: int
    retire_k: np.ndarray
    trace_lo: np.ndarray
    trace_maxrel: np.ndarray


def run(V, F, S, tol, max_iters=0, band_rule=0, window=0, trace_len=None, lib=None) -> Result:
    """PTP with the paper's band rule (band_rule=0: Eq. upper_band and Eq.
    lower_band, optionally capped at `window` toplesets) or the fixed half band
    [floor((k+1)/2), k] of the complexity analysis (band_rule=1).  Returns
    distances and labels in the caller's order."""
    X, F, S = _prep(V, F, S)
    n = X.shape[0]
    dist = np.empty(n, np.float64)
    label = np.empty(n, np.int32)
    retire = np.empty(n, np.int32)
    if trace_len is None:
        trace_len = (max_iters if max_iters > 0 else 4 * n + 16) + 1
        trace_len = min(trace_len, 1 << 22)
    tlo = np.full(trace_len, -1, np.int32)
    tmr = np.full(trace_len, np.nan, np.float64)
    st = _Stats()
    opts = _Opts(float(tol), int(max_iters), int(band_rule), int(window))
    rc = _L(lib).ptpo_run(n, F.shape[0], X, F, S.shape[0], S, C.byref(opts), dist, label,
                       C.byref(st), retire, tlo, tmr, trace_len)
    if rc not in (OK, ENOCONV):
        raise ValueError(f"ptpo_run failed: {rc}")
    K = st.iterations
    return Result(dist, label, rc, K, st.rho, st.reachable, int(st.updates),
                  retire[: st.rho].copy(), tlo[: K + 1].copy(), tmr[: K + 1].copy())


def replay(V, F, S, tol, retire, K, lib=None) -> Result:
    """The PTP iteration under a given schedule: retire[rho] = the last
    iteration that updated each topleset (-1: never retired), K = the number
    of iterations.  Used to compare arithmetic under another run's band."""
    X, F, S = _prep(V, F, S)
    n = X.shape[0]
    dist = np.empty(n, np.float64)
    label = np.empty(n, np.int32)
    ret_out = np.empty(n, np.int32)
    rin = np.full(n, -1, np.int32)
    r = np.asarray(retire, np.int32)
    rin[: r.shape[0]] = r
    st = _Stats()
    opts = _Opts(float(tol), 0, 0, 0)
    rc = _L(lib).ptpo_run_replay(n, F.shape[0], X, F, S.shape[0], S, C.byref(opts), rin, int(K),
                                 dist, label, C.byref(st), ret_out)
    if rc not in (OK, ENOCONV):
        raise ValueError(f"ptpo_run_replay failed: {rc}")
    e = np.empty(0)
    return Result(dist, label, rc, st.iterations, st.rho, st.reachable, int(st.updates),
                  ret_out[: st.rho].copy(), e, e)


@dataclass
class WarmResult:
    dist: np.ndarray
    label: np.ndarray
    status: int
    iterations: int
    rho: int
    reachable: int
    updates: int
    retire_k: np.ndarray
    rejected: int
    certified: np.ndarray


def run_warm(V, F, S, tol, upper, max_iters=0, window=0, certify=True, lib=None) -> WarmResult:
    """PTP started from the upper bound `upper[n]` (caller order): certified
    first (`rejected` counts the bounds withdrawn), or with certify=False taken
    as a known supersolution (a distance map of a subset of S)."""
    X, F, S = _prep(V, F, S)
    n = X.shape[0]
    w = np.ascontiguousarray(upper, dtype=np.float64)
    if w.shape != (n,):
        raise ValueError("upper must have n entries")
    dist = np.empty(n, np.float64)
    label = np.empty(n, np.int32)
    cert = np.empty(n, np.float64)
    retire = np.empty(n, np.int32)
    st = _Stats()
    rej = C.c_int(0)
    opts = _Opts(float(tol), int(max_iters), 0, int(window))
    rc = _L(lib).ptpo_run_warm(n, F.shape[0], X, F, S.shape[0], S, C.byref(opts), w,
                               int(bool(certify)), dist, label, C.byref(st), retire,
                               C.byref(rej), cert)
    if rc not in (OK, ENOCONV):
        raise ValueError(f"ptpo_run_warm failed: {rc}")
    return WarmResult(dist, label, rc, st.iterations, st.rho, st.reachable, int(st.updates),
                      retire[: st.rho].copy(), rej.value, cert)


def fixed_point(V, F, S, max_sweeps=100000, lib=None):
    """Jacobi from +inf until no value changes.  Returns (dist, label, sweeps)."""
    X, F, S = _prep(V, F, S)
    n = X.shape[0]
    dist = np.empty(n, np.float64)
    label = np.empty(n, np.int32)
    sw = C.c_int(0)
    rc = _L(lib).ptpo_fixed_point(n, F.shape[0], X, F, S.shape[0], S, int(max_sweeps), dist,
                               label, C.byref(sw))
    if rc != OK:
        raise ValueError(f"ptpo_fixed_point failed: {rc}")
    return dist, label, sw.value


def labels_from_map(V, F, S, dist, lib=None):
    """Voronoi labels of a distance map (caller order): every vertex takes the
    index in S of the source at the root of its chain of parents, the parent
    being the vertex its value comes from under its best triangle (only
    parents before it in (distance, id) order).  Returns (label, parent);
    parent is the vertex itself for a source, -1 where there is none."""
    X, F, S = _prep(V, F, S)
    n = X.shape[0]
    d = np.ascontiguousarray(dist, dtype=np.float64)
    label = np.empty(n, np.int32)
    parent = np.empty(n, np.int32)
    rc = _L(lib).ptpo_labels_from_map(n, F.shape[0], X, F, S.shape[0], S, d, label, parent)
    if rc != OK:
        raise ValueError(f"ptpo_labels_from_map failed: {rc}")
    return label, parent


def fast_marching(V, F, S, lib=None):
    X, F, S = _prep(V, F, S)
    n = X.shape[0]
    dist = np.empty(n, np.float64)
    rc = _L(lib).ptpo_fast_marching(n, F.shape[0], X, F, S.shape[0], S, dist)
    if rc != OK:
        raise ValueError(f"ptpo_fast_marching failed: {rc}")
    return dist
