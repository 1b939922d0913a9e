"""Python binding of the PTP C ABI (``include/ptp.h``), via ctypes.

Argument marshalling only: every step of the computation runs in the HIP
library ``libptp.so``.  PyTorch supplies device memory and the stream.  If the
library is missing or fails to load, every call raises; there is no fallback.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libptp.so")

PTP_OK = 0
PTP_EINVAL = -1
PTP_ENOMEM = -2
PTP_EDEVICE = -3
PTP_ENOCONV = -4
PTP_EUNSUPPORTED = -5
_NAMES = {0: "PTP_OK", -1: "PTP_EINVAL", -2: "PTP_ENOMEM", -3: "PTP_EDEVICE",
          -4: "PTP_ENOCONV", -5: "PTP_EUNSUPPORTED"}

# every symbol include/ptp.h declares
EXPORTS = ("ptp_plan_create", "ptp_workspace_bytes", "ptp_prepare", "ptp_run", "ptp_solve",
           "ptp_get_stats", "ptp_get_order", "ptp_get_schedule", "ptp_n_toplesets",
           "ptp_last_error", "ptp_plan_destroy", "ptp_version",
           "ptp_batch_create", "ptp_batch_workspace_bytes", "ptp_batch_prepare", "ptp_batch_run",
           "ptp_batch_get_stats", "ptp_batch_set_schedule", "ptp_batch_get_schedule",
           "ptp_batch_autotune", "ptp_batch_last_error", "ptp_batch_destroy",
           "ptp_warm_features", "ptp_warm_predict", "ptp_run_warm", "ptp_batch_warm_features",
           "ptp_batch_warm_predict", "ptp_batch_run_warm", "ptp_mlp_params", "ptp_mlp_apply",
           "ptp_mlp_scratch_bytes", "ptp_mlp_grad", "ptp_adam_step", "ptp_set_window",
           "ptp_batch_set_window", "ptp_run_f64", "ptp_batch_run_f64", "ptp_fps", "ptp_lloyd_step",
           "ptp_solve_noalloc", "ptp_noalloc_scratch_bytes", "ptp_get_parents", "ptp_batch_get_parents")

BAND_PAPER = 0          # PTP_BAND_PAPER: Eq. upper_band / Eq. lower_band
BAND_FIXED_HALF = 1     # PTP_BAND_FIXED_HALF: [floor((k+1)/2), k], 2 rho - 3 iterations
BAND_JACOBI = 2         # PTP_BAND_JACOBI: every topleset until nothing changes

MLP_PARAMS = 4481       # PTP_MLP_PARAMS


class PTPError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_NAMES.get(status, status)}: {msg}")
        self.status = status


class Options(C.Structure):
    _fields_ = [("tol", C.c_float), ("max_iters", C.c_int32), ("window", C.c_int32),
                ("want_labels", C.c_int32), ("workgroups", C.c_int32),
                ("lds_bfs_max", C.c_int32), ("band_rule", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("n_toplesets", C.c_int32),
                ("reachable", C.c_int32), ("workgroups", C.c_int32),
                ("vertex_updates", C.c_int64), ("certify_rounds", C.c_int32),
                ("certify_rejected", C.c_int32), ("ms_prepare", C.c_float), ("ms_run", C.c_float),
                ("ms_mesh_begin", C.c_float), ("ms_mesh_end", C.c_float),
                ("evaluated_updates", C.c_int64)]

    def as_dict(self) -> dict:
        return {f: (float(getattr(self, f)) if t is C.c_float else int(getattr(self, f)))
                for f, t in self._fields_}


class MeshDesc(C.Structure):
    """One mesh of a batch: where its rows start in the concatenated V, F, S
    and in the outputs (ptp_mesh)."""
    _fields_ = [("v_off", C.c_int64), ("f_off", C.c_int64), ("s_off", C.c_int64),
                ("out_off", C.c_int64), ("n_vertices", C.c_int32), ("n_faces", C.c_int32),
                ("n_sources", C.c_int32), ("reserved", C.c_int32)]


class Schedule(C.Structure):
    """Work distribution of a batch (ptp_schedule); 0 fields = defaults."""
    _fields_ = [("workgroups", C.c_int32), ("small_limit", C.c_int32),
                ("large_limit", C.c_int32), ("medium_group", C.c_int32),
                ("large_group", C.c_int32), ("xcd_pack", C.c_int32)]

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


_lib = None

# Plans and batches still open when the interpreter exits are destroyed by an
# exit hook, while the HIP runtime is certainly still up (a destructor run
# during interpreter teardown could call into a runtime already unloaded).
_live = weakref.WeakSet()


@atexit.register
def _close_all():
    for obj in list(_live):
        obj.close()


def load() -> C.CDLL:
    """Load libptp.so; raises when it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_1810_08218_amd.build`")
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    lib.ptp_plan_create.argtypes = [C.POINTER(vp), C.c_int32, C.c_int32, C.c_int32,
                                    C.POINTER(Options)]
    lib.ptp_plan_create.restype = C.c_int
    lib.ptp_workspace_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
    lib.ptp_workspace_bytes.restype = C.c_int
    lib.ptp_prepare.argtypes = [vp, vp, vp, vp, vp, C.c_size_t, vp]
    lib.ptp_prepare.restype = C.c_int
    lib.ptp_run.argtypes = [vp, vp, vp, vp]
    lib.ptp_run.restype = C.c_int
    lib.ptp_solve.argtypes = [vp, vp, vp, vp, vp, C.c_size_t, vp, vp, C.POINTER(Stats), vp]
    lib.ptp_solve.restype = C.c_int
    lib.ptp_solve_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, C.POINTER(Stats), vp]
    lib.ptp_solve_noalloc.restype = C.c_int
    lib.ptp_noalloc_scratch_bytes.argtypes = []
    lib.ptp_noalloc_scratch_bytes.restype = C.c_size_t
    lib.ptp_get_stats.argtypes = [vp, C.POINTER(Stats)]
    lib.ptp_get_stats.restype = C.c_int
    lib.ptp_get_parents.argtypes = [vp, vp, vp]
    lib.ptp_get_parents.restype = C.c_int
    lib.ptp_batch_get_parents.argtypes = [vp, vp, vp]
    lib.ptp_batch_get_parents.restype = C.c_int
    lib.ptp_get_order.argtypes = [vp, vp, vp, vp]
    lib.ptp_get_order.restype = C.c_int
    lib.ptp_get_schedule.argtypes = [vp, vp]
    lib.ptp_get_schedule.restype = C.c_int
    lib.ptp_n_toplesets.argtypes = [vp]
    lib.ptp_n_toplesets.restype = C.c_int32
    lib.ptp_last_error.argtypes = [vp]
    lib.ptp_last_error.restype = C.c_char_p
    lib.ptp_plan_destroy.argtypes = [vp]
    lib.ptp_plan_destroy.restype = None
    lib.ptp_version.argtypes = []
    lib.ptp_version.restype = C.c_char_p
    lib.ptp_batch_create.argtypes = [C.POINTER(vp), C.POINTER(MeshDesc), C.c_int32,
                                     C.POINTER(Options)]
    lib.ptp_batch_create.restype = C.c_int
    lib.ptp_batch_workspace_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
    lib.ptp_batch_workspace_bytes.restype = C.c_int
    lib.ptp_batch_prepare.argtypes = [vp, vp, vp, vp, vp, C.c_size_t, vp]
    lib.ptp_batch_prepare.restype = C.c_int
    lib.ptp_batch_run.argtypes = [vp, vp, vp, vp]
    lib.ptp_batch_run.restype = C.c_int
    lib.ptp_batch_get_stats.argtypes = [vp, vp, vp]
    lib.ptp_batch_get_stats.restype = C.c_int
    lib.ptp_batch_set_schedule.argtypes = [vp, C.POINTER(Schedule)]
    lib.ptp_batch_set_schedule.restype = C.c_int
    lib.ptp_batch_get_schedule.argtypes = [vp, C.POINTER(Schedule)]
    lib.ptp_batch_get_schedule.restype = C.c_int
    lib.ptp_batch_autotune.argtypes = [vp, C.POINTER(Schedule), C.c_int32, vp, vp, vp,
                                       C.POINTER(C.c_int32), vp]
    lib.ptp_batch_autotune.restype = C.c_int
    lib.ptp_batch_last_error.argtypes = [vp]
    lib.ptp_batch_last_error.restype = C.c_char_p
    lib.ptp_batch_destroy.argtypes = [vp]
    lib.ptp_batch_destroy.restype = None
    for name in ("ptp_warm_features", "ptp_batch_warm_features"):
        getattr(lib, name).argtypes = [vp, vp, vp, vp]
        getattr(lib, name).restype = C.c_int
    for name in ("ptp_warm_predict", "ptp_batch_warm_predict"):
        getattr(lib, name).argtypes = [vp, vp, C.c_float, vp, vp]
        getattr(lib, name).restype = C.c_int
    for name in ("ptp_run_warm", "ptp_batch_run_warm"):
        getattr(lib, name).argtypes = [vp, vp, vp, vp]
        getattr(lib, name).restype = C.c_int
    for name in ("ptp_set_window", "ptp_batch_set_window"):
        getattr(lib, name).argtypes = [vp, C.c_int32]
        getattr(lib, name).restype = C.c_int
    lib.ptp_run_f64.argtypes = [vp, vp, vp]
    lib.ptp_run_f64.restype = C.c_int
    lib.ptp_batch_run_f64.argtypes = [vp, vp, vp]
    lib.ptp_batch_run_f64.restype = C.c_int
    lib.ptp_fps.argtypes = [vp, vp, vp, vp, C.c_int32, vp, C.c_size_t, C.c_int32, vp, vp, vp, vp]
    lib.ptp_fps.restype = C.c_int
    lib.ptp_lloyd_step.argtypes = [vp, vp, vp, vp, vp]
    lib.ptp_lloyd_step.restype = C.c_int
    lib.ptp_mlp_params.argtypes = []
    lib.ptp_mlp_params.restype = C.c_int32
    lib.ptp_mlp_apply.argtypes = [vp, vp, vp, C.c_int64, vp, vp]
    lib.ptp_mlp_apply.restype = C.c_int
    lib.ptp_mlp_scratch_bytes.argtypes = []
    lib.ptp_mlp_scratch_bytes.restype = C.c_size_t
    lib.ptp_mlp_grad.argtypes = [vp, vp, vp, vp, C.c_int64, vp, C.c_size_t, vp, vp, vp]
    lib.ptp_mlp_grad.restype = C.c_int
    lib.ptp_adam_step.argtypes = [vp, vp, vp, vp, C.c_int32, C.c_float, C.c_float, C.c_float,
                                  C.c_float, vp]
    lib.ptp_adam_step.restype = C.c_int
    if lib.ptp_mlp_params() != MLP_PARAMS:
        raise RuntimeError("libptp.so was built with another network size")
    _lib = lib
    return lib


def _ptr(t) -> C.c_void_p:
    return C.c_void_p(0 if t is None else t.data_ptr())


def _stream(stream) -> C.c_void_p:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _check_dev(t, dtype, shape_tail, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape_tail is not None and tuple(t.shape[1:]) != shape_tail:
        raise ValueError(f"{name} must have shape [*, {shape_tail}]")


class Plan:
    """One mesh size + options.  Owns the host plan and (by default) a torch
    workspace tensor; all device memory is torch's."""

    def __init__(self, n: int, f: int, m: int, tol: float, max_iters: int = 0, window: int = 0,
                 want_labels: bool = False, workgroups: int = 0, lds_bfs_max: int = 0,
                 band_rule: int = BAND_PAPER):
        lib = load()
        self._lib = lib
        self.n, self.f, self.m = int(n), int(f), int(m)
        self.want_labels = bool(want_labels)
        opt = Options(float(tol), int(max_iters), int(window), int(bool(want_labels)),
                      int(workgroups), int(lds_bfs_max), int(band_rule))
        h = C.c_void_p()
        rc = lib.ptp_plan_create(C.byref(h), self.n, self.f, self.m, C.byref(opt))
        if rc != PTP_OK:
            raise PTPError(rc, "ptp_plan_create")
        self._h = h
        self._work = None
        _live.add(self)

    def close(self):
        """Destroy the host plan and drop the workspace (idempotent)."""
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.ptp_plan_destroy(h)
        self._h = None
        self._work = None
        self._keep = None

    def __del__(self):
        self.close()

    def _err(self, rc, what):
        msg = self._lib.ptp_last_error(self._h)
        return PTPError(rc, f"{what}: {msg.decode() if msg else ''}")

    def workspace_bytes(self) -> int:
        b = C.c_size_t(0)
        rc = self._lib.ptp_workspace_bytes(self._h, C.byref(b))
        if rc != PTP_OK:
            raise self._err(rc, "ptp_workspace_bytes")
        return int(b.value)

    def workspace(self, device=None):
        import torch
        need = self.workspace_bytes()
        if self._work is None or self._work.numel() < need + 256:
            self._work = torch.empty(need + 256, dtype=torch.uint8, device=device or "cuda")
        off = (-self._work.data_ptr()) % 256
        return self._work[off:off + need]

    def prepare(self, V, F, S, work=None, stream=None):
        import torch
        _check_dev(V, torch.float32, (3,), "V")
        _check_dev(F, torch.int32, (3,), "F")
        _check_dev(S, torch.int32, None, "S")
        if V.shape[0] != self.n or F.shape[0] != self.f or S.numel() != self.m:
            raise ValueError("mesh sizes differ from the plan")
        if work is None:
            work = self.workspace(V.device)
        rc = self._lib.ptp_prepare(self._h, _ptr(V), _ptr(F), _ptr(S), _ptr(work),
                                   work.numel(), _stream(stream))
        if rc != PTP_OK:
            raise self._err(rc, "ptp_prepare")
        self._keep = (V, F, S, work)

    def run(self, dist, label=None, stream=None):
        import torch
        _check_dev(dist, torch.float32, None, "dist")
        if dist.numel() != self.n:
            raise ValueError("dist must have n elements")
        if label is not None:
            _check_dev(label, torch.int32, None, "label")
            if label.numel() != self.n:
                raise ValueError("label must have n elements")
        rc = self._lib.ptp_run(self._h, _ptr(dist), _ptr(label), _stream(stream))
        if rc != PTP_OK:
            raise self._err(rc, "ptp_run")

    def solve_noalloc(self, V, F, S, dist, label=None, stream=None) -> dict:
        """ptp_solve on the library's fixed scratch (no workspace, no device
        allocation): prepare + run + synchronise; returns the stats (status
        included, PTP_ENOCONV allowed)."""
        import torch
        _check_dev(V, torch.float32, (3,), "V")
        _check_dev(F, torch.int32, (3,), "F")
        _check_dev(S, torch.int32, None, "S")
        _check_dev(dist, torch.float32, None, "dist")
        if V.shape[0] != self.n or F.shape[0] != self.f or S.numel() != self.m:
            raise ValueError("mesh sizes differ from the plan")
        if dist.numel() != self.n:
            raise ValueError("dist must have n elements")
        if label is not None:
            _check_dev(label, torch.int32, None, "label")
            if label.numel() != self.n:
                raise ValueError("label must have n elements")
        st = Stats()
        rc = self._lib.ptp_solve_noalloc(self._h, _ptr(V), _ptr(F), _ptr(S), _ptr(dist), _ptr(label),
                                         C.byref(st), _stream(stream))
        self._keep = (V, F, S, None)
        if rc != PTP_OK and rc != PTP_ENOCONV:
            raise self._err(rc, "ptp_solve_noalloc")
        d = st.as_dict()
        d["status"] = rc
        return d

    def run_f64(self, dist, stream=None):
        """The same iteration in float64: dist is a float64 [n] device tensor."""
        import torch
        _check_dev(dist, torch.float64, None, "dist")
        if dist.numel() != self.n:
            raise ValueError("dist must have n elements")
        rc = self._lib.ptp_run_f64(self._h, _ptr(dist), _stream(stream))
        if rc != PTP_OK:
            raise self._err(rc, "ptp_run_f64")

    def fps(self, V, F, S, n_initial: int, dist, radius=None, steps=None, warm: bool = False,
            work=None, stream=None):
        """Farthest point sampling: S (int32 [m] device, m = the plan's source
        count) holds the first n_initial sources and receives the samples;
        dist the final map; radius [m - n_initial] and steps int64
        [2 (m - n_initial + 1)] optional device tensors.  Synchronises."""
        import torch
        _check_dev(V, torch.float32, (3,), "V")
        _check_dev(F, torch.int32, (3,), "F")
        _check_dev(S, torch.int32, None, "S")
        _check_dev(dist, torch.float32, None, "dist")
        if V.shape[0] != self.n or F.shape[0] != self.f or S.numel() != self.m:
            raise ValueError("mesh sizes differ from the plan")
        if dist.numel() != self.n:
            raise ValueError("dist must have n elements")
        if radius is not None:
            _check_dev(radius, torch.float32, None, "radius")
            if radius.numel() < self.m - n_initial:
                raise ValueError("radius needs m - n_initial entries")
        if steps is not None:
            _check_dev(steps, torch.int64, None, "steps")
            if steps.numel() < 2 * (self.m - n_initial + 1):
                raise ValueError("steps needs 2 (m - n_initial + 1) entries")
        if work is None:
            work = self.workspace(V.device)
        rc = self._lib.ptp_fps(self._h, _ptr(V), _ptr(F), _ptr(S), int(n_initial), _ptr(work),
                               work.numel(), int(bool(warm)), _ptr(dist), _ptr(radius), _ptr(steps),
                               _stream(stream))
        self._keep = (V, F, S, work)
        if rc != PTP_OK and rc != PTP_ENOCONV:
            raise self._err(rc, "ptp_fps")
        return rc

    def lloyd_step(self, label, S_out, centroid=None, stream=None):
        """One Lloyd step on the labels of the last run over the prepared mesh
        and sources: S_out [m] (device int32) receives the new generators,
        centroid (float64 [m, 4]) the centroids and cell areas."""
        import torch
        _check_dev(label, torch.int32, None, "label")
        _check_dev(S_out, torch.int32, None, "S_out")
        if label.numel() != self.n or S_out.numel() != self.m:
            raise ValueError("sizes differ from the plan")
        if centroid is not None:
            _check_dev(centroid, torch.float64, (4,), "centroid")
            if centroid.shape[0] != self.m:
                raise ValueError("centroid must be [m, 4]")
        rc = self._lib.ptp_lloyd_step(self._h, _ptr(label), _ptr(S_out), _ptr(centroid), _stream(stream))
        if rc != PTP_OK:
            raise self._err(rc, "ptp_lloyd_step")

    # -- learned warm start --------------------------------------------------
    def warm_features(self, stream=None):
        """Network inputs X [n, 3] and scale [n] (caller order) as device tensors."""
        import torch
        X = torch.empty((self.n, 3), dtype=torch.float32, device="cuda")
        scale = torch.empty(self.n, dtype=torch.float32, device="cuda")
        rc = self._lib.ptp_warm_features(self._h, _ptr(X), _ptr(scale), _stream(stream))
        if rc != PTP_OK:
            raise self._err(rc, "ptp_warm_features")
        return X, scale

    def warm_predict(self, params, upper, inflate: float = 1.05, stream=None):
        """upper[n] = inflate * predicted distance (0 at sources, +inf unreachable)."""
        import torch
        _check_dev(params, torch.float32, None, "params")
        _check_dev(upper, torch.float32, None, "upper")
        if params.numel() != MLP_PARAMS or upper.numel() != self.n:
            raise ValueError("params must have MLP_PARAMS values and upper n")
        rc = self._lib.ptp_warm_predict(self._h, _ptr(params), float(inflate), _ptr(upper),
                                        _stream(stream))
        if rc != PTP_OK:
            raise self._err(rc, "ptp_warm_predict")

    def run_warm(self, upper, dist, stream=None):
        """Certify `upper` and run PTP from it (may be the same tensor as dist)."""
        import torch
        _check_dev(upper, torch.float32, None, "upper")
        _check_dev(dist, torch.float32, None, "dist")
        if upper.numel() != self.n or dist.numel() != self.n:
            raise ValueError("upper and dist must have n elements")
        rc = self._lib.ptp_run_warm(self._h, _ptr(upper), _ptr(dist), _stream(stream))
        if rc != PTP_OK:
            raise self._err(rc, "ptp_run_warm")

    def set_window(self, window: int):
        """Band cap for the following runs (changes results; 0 = unbounded)."""
        rc = self._lib.ptp_set_window(self._h, int(window))
        if rc != PTP_OK:
            raise self._err(rc, "ptp_set_window")

    def stats(self, allow_noconv: bool = True) -> dict:
        st = Stats()
        rc = self._lib.ptp_get_stats(self._h, C.byref(st))
        d = st.as_dict()
        d["status"] = rc
        if rc != PTP_OK and not (allow_noconv and rc == PTP_ENOCONV):
            raise self._err(rc, "ptp_get_stats")
        return d

    def n_toplesets(self) -> int:
        return int(self._lib.ptp_n_toplesets(self._h))

    def parents(self, stream=None):
        """Parents behind the labels of the last (labelled) run: int32 [n]
        device tensor of caller vertex ids (a source its own id, -1 where
        unreachable)."""
        import torch
        out = torch.empty(self.n, dtype=torch.int32, device="cuda")
        rc = self._lib.ptp_get_parents(self._h, _ptr(out), _stream(stream))
        if rc != PTP_OK:
            raise self._err(rc, "ptp_get_parents")
        return out

    def order(self, stream=None):
        """(perm[n], offsets[rho + 1]) as int32 device tensors."""
        import torch
        rho = self.n_toplesets()
        perm = torch.empty(self.n, dtype=torch.int32, device="cuda")
        offs = torch.empty(rho + 1, dtype=torch.int32, device="cuda")
        rc = self._lib.ptp_get_order(self._h, _ptr(perm), _ptr(offs), _stream(stream))
        if rc != PTP_OK:
            raise self._err(rc, "ptp_get_order")
        return perm, offs

    def schedule(self) -> np.ndarray:
        """Last iteration that updated each topleset (host int32 [rho])."""
        rho = self.n_toplesets()
        out = np.empty(rho, np.int32)
        rc = self._lib.ptp_get_schedule(self._h, C.c_void_p(out.ctypes.data))
        if rc != PTP_OK:
            raise self._err(rc, "ptp_get_schedule")
        return out


@dataclass
class Solution:
    dist: object       # torch float32 [n] (device)
    label: object      # torch int32 [n] (device) or None
    stats: dict
    plan: Plan


def solve(V, F, S, tol: float, labels: bool = False, max_iters: int = 0, window: int = 0,
          workgroups: int = 0, band_rule: int = BAND_PAPER, stream=None) -> Solution:
    """Geodesic distances from the source set S on mesh (V, F): prepare + run
    + stats.  V float32 [n, 3], F int32 [f, 3], S int32 [m], all on the GPU."""
    import torch
    plan = Plan(V.shape[0], F.shape[0], S.numel(), tol, max_iters=max_iters, window=window,
                want_labels=labels, workgroups=workgroups, band_rule=band_rule)
    plan.prepare(V, F, S, stream=stream)
    dist = torch.empty(V.shape[0], dtype=torch.float32, device=V.device)
    lab = torch.empty(V.shape[0], dtype=torch.int32, device=V.device) if labels else None
    plan.run(dist, lab, stream=stream)
    st = plan.stats()
    return Solution(dist, lab, st, plan)


# ---------------------------------------------------------------- batches ---

def concat(meshes, share=None):
    """Concatenate meshes (objects with V, F, S numpy arrays) into one V, F, S
    and a list of MeshDesc.  `share` (optional list) gives, per mesh, the index
    of an earlier mesh whose V and F rows it reuses (many source sets on one
    mesh); outputs never overlap."""
    Vs, Fs, Ss, descs = [], [], [], []
    v_off = f_off = s_off = out_off = 0
    rows = {}
    for i, m in enumerate(meshes):
        src = share[i] if share is not None and share[i] is not None else None
        if src is not None:
            vo, fo = rows[src]
        else:
            vo, fo = v_off, f_off
            Vs.append(np.asarray(m.V, np.float32))
            Fs.append(np.asarray(m.F, np.int32).reshape(-1, 3))
            v_off += m.V.shape[0]
            f_off += Fs[-1].shape[0]
        rows[i] = (vo, fo)
        Ss.append(np.asarray(m.S, np.int32))
        descs.append(MeshDesc(vo, fo, s_off, out_off, m.V.shape[0], np.asarray(m.F).shape[0],
                              len(m.S), 0))
        s_off += len(m.S)
        out_off += m.V.shape[0]
    V = np.ascontiguousarray(np.concatenate(Vs, axis=0))
    F = np.ascontiguousarray(np.concatenate(Fs, axis=0)) if Fs else np.zeros((0, 3), np.int32)
    S = np.ascontiguousarray(np.concatenate(Ss))
    return V, F, S, descs, out_off


class Batch:
    """Many meshes solved in one persistent launch (ptp_batch_*).  Every mesh
    gets exactly the result a Plan would give it alone."""

    def __init__(self, descs, tol: float, max_iters: int = 0, window: int = 0,
                 want_labels: bool = False, lds_bfs_max: int = 0, band_rule: int = BAND_PAPER):
        lib = load()
        self._lib = lib
        self.count = len(descs)
        self._descs = (MeshDesc * self.count)(*descs)
        self.out_len = max(int(d.out_off) + int(d.n_vertices) for d in descs)
        self.want_labels = bool(want_labels)
        opt = Options(float(tol), int(max_iters), int(window), int(bool(want_labels)), 0,
                      int(lds_bfs_max), int(band_rule))
        h = C.c_void_p()
        rc = lib.ptp_batch_create(C.byref(h), self._descs, self.count, C.byref(opt))
        if rc != PTP_OK:
            raise PTPError(rc, "ptp_batch_create")
        self._h = h
        self._work = None
        _live.add(self)

    def close(self):
        """Destroy the host batch and drop the workspace (idempotent)."""
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.ptp_batch_destroy(h)
        self._h = None
        self._work = None
        self._keep = None

    def __del__(self):
        self.close()

    def _err(self, rc, what):
        msg = self._lib.ptp_batch_last_error(self._h)
        return PTPError(rc, f"{what}: {msg.decode() if msg else ''}")

    def workspace_bytes(self) -> int:
        b = C.c_size_t(0)
        rc = self._lib.ptp_batch_workspace_bytes(self._h, C.byref(b))
        if rc != PTP_OK:
            raise self._err(rc, "ptp_batch_workspace_bytes")
        return int(b.value)

    def workspace(self, device=None):
        import torch
        need = self.workspace_bytes()
        if self._work is None or self._work.numel() < need + 256:
            self._work = torch.empty(need + 256, dtype=torch.uint8, device=device or "cuda")
        off = (-self._work.data_ptr()) % 256
        return self._work[off:off + need]

    def prepare(self, V, F, S, work=None, stream=None):
        import torch
        _check_dev(V, torch.float32, (3,), "V")
        _check_dev(F, torch.int32, (3,), "F")
        _check_dev(S, torch.int32, None, "S")
        if work is None:
            work = self.workspace(V.device)
        rc = self._lib.ptp_batch_prepare(self._h, _ptr(V), _ptr(F), _ptr(S), _ptr(work),
                                         work.numel(), _stream(stream))
        if rc != PTP_OK:
            raise self._err(rc, "ptp_batch_prepare")
        self._keep = (V, F, S, work)

    def run(self, dist, label=None, stream=None):
        import torch
        _check_dev(dist, torch.float32, None, "dist")
        if dist.numel() < self.out_len:
            raise ValueError("dist too short for the batch outputs")
        if label is not None:
            _check_dev(label, torch.int32, None, "label")
        rc = self._lib.ptp_batch_run(self._h, _ptr(dist), _ptr(label), _stream(stream))
        if rc != PTP_OK:
            raise self._err(rc, "ptp_batch_run")

    def run_f64(self, dist, stream=None):
        import torch
        _check_dev(dist, torch.float64, None, "dist")
        if dist.numel() < self.out_len:
            raise ValueError("dist too short for the batch outputs")
        rc = self._lib.ptp_batch_run_f64(self._h, _ptr(dist), _stream(stream))
        if rc != PTP_OK:
            raise self._err(rc, "ptp_batch_run_f64")

    def warm_features(self, stream=None):
        """Network inputs X [out_len, 3] and scale [out_len] as device tensors."""
        import torch
        X = torch.empty((self.out_len, 3), dtype=torch.float32, device="cuda")
        scale = torch.empty(self.out_len, dtype=torch.float32, device="cuda")
        rc = self._lib.ptp_batch_warm_features(self._h, _ptr(X), _ptr(scale), _stream(stream))
        if rc != PTP_OK:
            raise self._err(rc, "ptp_batch_warm_features")
        return X, scale

    def warm_predict(self, params, upper, inflate: float = 1.05, stream=None):
        import torch
        _check_dev(params, torch.float32, None, "params")
        _check_dev(upper, torch.float32, None, "upper")
        if params.numel() != MLP_PARAMS or upper.numel() < self.out_len:
            raise ValueError("params must have MLP_PARAMS values and upper out_len")
        rc = self._lib.ptp_batch_warm_predict(self._h, _ptr(params), float(inflate), _ptr(upper),
                                              _stream(stream))
        if rc != PTP_OK:
            raise self._err(rc, "ptp_batch_warm_predict")

    def run_warm(self, upper, dist, stream=None):
        import torch
        _check_dev(upper, torch.float32, None, "upper")
        _check_dev(dist, torch.float32, None, "dist")
        if upper.numel() < self.out_len or dist.numel() < self.out_len:
            raise ValueError("upper and dist too short for the batch outputs")
        rc = self._lib.ptp_batch_run_warm(self._h, _ptr(upper), _ptr(dist), _stream(stream))
        if rc != PTP_OK:
            raise self._err(rc, "ptp_batch_run_warm")

    def stats(self):
        """(aggregate status, [per-mesh stats dict], [per-mesh status])"""
        st = (Stats * self.count)()
        status = (C.c_int32 * self.count)()
        rc = self._lib.ptp_batch_get_stats(self._h, st, status)
        # one dict per mesh, built from a structured view of the array (a
        # field-by-field read of 512 structures costs milliseconds)
        names = [f for f, _ in Stats._fields_]
        rows = np.ctypeslib.as_array(st).tolist()
        return rc, [dict(zip(names, r)) for r in rows], list(status)

    def parents(self, stream=None):
        """Parents behind the labels of the last (labelled) run: int32
        [out_len] device tensor of local vertex ids, indexed like the
        outputs."""
        import torch
        out = torch.empty(self.out_len, dtype=torch.int32, device="cuda")
        rc = self._lib.ptp_batch_get_parents(self._h, _ptr(out), _stream(stream))
        if rc != PTP_OK:
            raise self._err(rc, "ptp_batch_get_parents")
        return out

    def set_window(self, window: int):
        """Band cap for the following runs of every mesh (changes results)."""
        rc = self._lib.ptp_batch_set_window(self._h, int(window))
        if rc != PTP_OK:
            raise self._err(rc, "ptp_batch_set_window")

    def set_schedule(self, **kw):
        sch = Schedule(**{k: int(v) for k, v in kw.items()})
        rc = self._lib.ptp_batch_set_schedule(self._h, C.byref(sch))
        if rc != PTP_OK:
            raise self._err(rc, "ptp_batch_set_schedule")

    def get_schedule(self) -> dict:
        sch = Schedule()
        rc = self._lib.ptp_batch_get_schedule(self._h, C.byref(sch))
        if rc != PTP_OK:
            raise self._err(rc, "ptp_batch_get_schedule")
        return sch.as_dict()

    def autotune(self, candidates, dist, label=None, stream=None):
        """Time each candidate schedule (dicts of Schedule fields) on the
        prepared batch, keep the fastest.  Returns (best index, ms list)."""
        n = len(candidates)
        arr = (Schedule * n)(*[Schedule(**{k: int(v) for k, v in c.items()}) for c in candidates])
        ms = (C.c_float * n)()
        best = C.c_int32(-1)
        rc = self._lib.ptp_batch_autotune(self._h, arr, n, _ptr(dist), _ptr(label), ms,
                                          C.byref(best), _stream(stream))
        if rc != PTP_OK:
            raise self._err(rc, "ptp_batch_autotune")
        return int(best.value), [float(x) for x in ms]


# ------------------------------------------------------- warm-start network ---

def mlp_apply(params, X, scale, out=None, stream=None):
    """out[i] = 64 scale[i] softplus(o(X[i])) on the GPU (ptp_mlp_apply)."""
    import torch
    lib = load()
    _check_dev(params, torch.float32, None, "params")
    _check_dev(X, torch.float32, (3,), "X")
    _check_dev(scale, torch.float32, None, "scale")
    n = X.shape[0]
    if params.numel() != MLP_PARAMS or scale.numel() != n:
        raise ValueError("params / scale sizes")
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=X.device)
    rc = lib.ptp_mlp_apply(_ptr(params), _ptr(X), _ptr(scale), n, _ptr(out), _stream(stream))
    if rc != PTP_OK:
        raise PTPError(rc, "ptp_mlp_apply")
    return out


class MlpTrainer:
    """Device buffers for training the warm-start network with the library's
    forward/backward and Adam kernels (gradient scratch, moments)."""

    def __init__(self, params, lr=1e-3, betas=(0.9, 0.999), eps=1e-8):
        import torch
        lib = load()
        self._lib = lib
        _check_dev(params, torch.float32, None, "params")
        if params.numel() != MLP_PARAMS:
            raise ValueError("params must have MLP_PARAMS values")
        self.params = params
        self.lr, self.betas, self.eps = float(lr), betas, float(eps)
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.grad = torch.zeros_like(params)
        self.loss = torch.zeros(1, dtype=torch.float32, device=params.device)
        nb = int(lib.ptp_mlp_scratch_bytes())
        self.scratch = torch.empty((nb + 3) // 4, dtype=torch.float32, device=params.device)
        self.t = 0

    def grad_loss(self, X, scale, target, stream=None):
        """Gradient (into self.grad) and loss (self.loss) over the rows."""
        import torch
        _check_dev(X, torch.float32, (3,), "X")
        _check_dev(scale, torch.float32, None, "scale")
        _check_dev(target, torch.float32, None, "target")
        n = X.shape[0]
        if scale.numel() != n or target.numel() != n or n < 1:
            raise ValueError("row counts")
        rc = self._lib.ptp_mlp_grad(_ptr(self.params), _ptr(X), _ptr(scale), _ptr(target), n,
                                    _ptr(self.scratch), self.scratch.numel() * 4, _ptr(self.grad),
                                    _ptr(self.loss), _stream(stream))
        if rc != PTP_OK:
            raise PTPError(rc, "ptp_mlp_grad")
        return self.grad, self.loss

    def adam(self, stream=None):
        self.t += 1
        rc = self._lib.ptp_adam_step(_ptr(self.params), _ptr(self.grad), _ptr(self.m), _ptr(self.v),
                                     self.t, self.lr, float(self.betas[0]), float(self.betas[1]),
                                     self.eps, _stream(stream))
        if rc != PTP_OK:
            raise PTPError(rc, "ptp_adam_step")

    def step(self, X, scale, target, stream=None):
        self.grad_loss(X, scale, target, stream)
        self.adam(stream)
        return self.loss
