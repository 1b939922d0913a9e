"""Benchmark of the PTP hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--only batch]

Headline workload: the batch of 512 meshes of uneven size (256 jittered grids
of side 32..1024, 256 tori of 2^k x 2^(k-1) vertices, k = 5..10, 1-4 random
sources each; 71.2M vertices, 142M triangles; seed 4, tol 1e-4), already
resident in HBM.  One step is the whole path over that batch: validation,
incidence, BFS toplesets and reorder of every mesh (ptp_batch_prepare), then
the band relaxation of every mesh in one persistent launch with unpermute
(ptp_batch_run), with the work distribution the library's autotuner picked
for this workload.  `value` is vertex updates per second over whole steps.

Alongside, in sub-keys: the same meshes one plan at a time, the learned warm
start, the error of plain and warm results against the fixed point (Jacobi on
the GPU), the autotuner and band-cap legs; the flat 64 x 64 grid (tol 1e-6)
and the 1001 x 1001 grid of the paper's accuracy figure; the noisy level-7
icosphere (single mesh: step, roofline, warm start, float64, the fixed half
band, band diagnostics, farthest point sampling against Fast Marching on the
CPU); the level-9 bumpy icosphere with 32 sources and labels (plus the
learned warm start and Lloyd steps); 64 source sets on it; and the CPU
oracle (one core and all cores) on a sample of the batch.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import os
import platform
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E
BYTES_PER_UPDATE = 48           # own xyz 12 + d read 4 + d write 4 + fan row 4 + 6 neighbour ids 24
BYTES_PER_SKIP = 4              # a band vertex no neighbour changed: its mark only
CSRC = os.path.join(ROOT, "paper_1810_08218_amd", "csrc")
RELAX_SOURCES = [os.path.join(CSRC, f) for f in ("ptp_relax.hip", "ptp_device.h", "ptp_kernels.h")]
PMC_FILE = os.path.join(ROOT, "profiles", "relax_batch512_pmc.json")
METRIC = "ms to converge + vertex-updates/s at <=1e-4 rel err; warm-start/batched vs plain"
TOL = 1e-4


def relax_source_hash() -> str:
    h = hashlib.sha256()
    for p in RELAX_SOURCES:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per batched relaxation launch from the committed rocprofv3
    counter summary, only while the relaxation sources are the profiled ones."""
    if not os.path.exists(PMC_FILE):
        return None
    with open(PMC_FILE) as fh:
        rec = json.load(fh)
    if rec.get("relax_sources_sha256_16") != relax_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def note(msg):
    """Progress line on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _timed(fn, stream, reps, warm=3):
    """Median device time (ms) of fn() over reps runs after `warm` warm-ups."""
    import torch
    for _ in range(warm):
        fn()
    ts = []
    for _ in range(reps):
        a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        z.record(stream)
        z.synchronize()
        ts.append(a.elapsed_time(z))
    return statistics.median(ts)


def _rel(a, b):
    """max and mean |a - b| / b over entries with finite positive b."""
    import torch
    a = a.double()
    b = b.double()
    fin = torch.isfinite(b) & (b > 0)
    e = (a[fin] - b[fin]).abs() / b[fin]
    return float(e.max()), float(e.mean())


def host_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"logical_cpus": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)),
            "model": model or platform.processor()}


# ------------------------------------------------------------------ CPU ---

def cpu_baseline(meshes, budget_s=15.0):
    """The FP64 oracle on a bounded sample of the batch (meshes in order until
    the budget is spent), one core; then the same sample with the OpenMP build
    of the same source on every host core."""
    import oracle as O
    t_all, U, names = 0.0, 0, []
    done = []
    for m in meshes:
        t0 = time.perf_counter()
        r = O.run(m.V, m.F, m.S, TOL)
        t_all += time.perf_counter() - t0
        U += r.updates
        done.append(m)
        if t_all > budget_s:
            break
    lib = O.load_omp()
    t_omp = 0.0
    for m in done:
        t0 = time.perf_counter()
        O.run(m.V, m.F, m.S, TOL, lib=lib)
        t_omp += time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    nv = sum(m.n for m in done)
    base = {"value": U / t_all, "unit": "vertex-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"the first {len(done)} meshes of the 512-mesh batch ({nv} vertices, U={U}), "
                      f"one full FP64 solve each by the sequential oracle ({t_all:.1f} s)"}
    allc = {"value": U / t_omp, "unit": "vertex-updates/s", "cores": threads, "kind": "oracle (OpenMP build)",
            "sample": "the same meshes, band updates on every host core", "seconds": round(t_omp, 2)}
    return base, allc


def cpu_fast_marching(mesh, reps=3):
    """Sequential Fast Marching (the paper's baseline, FP64, same planar
    update) on one mesh, median of reps."""
    import oracle as O
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        O.fast_marching(mesh.V, mesh.F, mesh.S)
        ts.append(time.perf_counter() - t0)
    return statistics.median(ts) * 1e3


# ------------------------------------------------------------- headline ---

class BatchWorkload:
    def __init__(self, P, I):
        import torch
        note("batch: generating 512 meshes")
        self.meshes = I.batch_meshes(512)
        V, F, S, self.descs, self.out_len = P.concat(self.meshes)
        self.dV, self.dF, self.dS = (torch.from_numpy(x).cuda() for x in (V, F, S))
        self.n = int(V.shape[0])
        self.f = int(F.shape[0])
        del V, F, S


def bench_batch_steps(P, W, steps, warmup, stream):
    """The timed steps: prepare + run of the whole batch."""
    import torch
    from paper_1810_08218_amd import autotune
    b = P.Batch(W.descs, TOL)
    b.set_schedule(**autotune.BATCH512_SCHEDULE)
    work = b.workspace()
    dist = torch.empty(W.out_len, dtype=torch.float32, device="cuda")

    def step(ev=None):
        b.prepare(W.dV, W.dF, W.dS, work=work, stream=stream)
        if ev is not None:
            ev[0].record(stream)
        b.run(dist, stream=stream)
        if ev is not None:
            ev[1].record(stream)
        return b.stats()

    note(f"batch: {warmup} warm-up + {steps} timed steps")
    for _ in range(warmup):
        step()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        rc, stats, status = step(evs[k])
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / steps
    runs = [a.elapsed_time(z) for a, z in evs]
    U = sum(x["vertex_updates"] for x in stats)
    return {"batch": b, "work": work, "dist": dist, "rc": rc, "stats": stats, "status": status,
            "ms_step": ms_step, "ms_run": statistics.mean(runs), "ms_run_min": min(runs), "U": U,
            "ms_prepare": statistics.mean(x["ms_prepare"] for x in stats[:1])}


def bench_warm(obj, n_out, stream, reps, fixed_point=None):
    """Learned warm start against the plain run on a prepared plan or batch:
    ms to converge of (features + network + certified run) vs (run); both 3
    warm-ups then the median of `reps`; iterations, updates; the difference of
    the two results and, given the fixed point, each one's error against it."""
    import torch
    from paper_1810_08218_amd import train_warmstart
    params = train_warmstart.load_params()
    plain = torch.empty(n_out, dtype=torch.float32, device="cuda")
    warm = torch.empty(n_out, dtype=torch.float32, device="cuda")

    def run_plain():
        obj.run(plain, stream=stream)

    def run_warm():
        obj.warm_predict(params, warm, inflate=1.05, stream=stream)
        obj.run_warm(warm, warm, stream=stream)

    ms_plain = _timed(run_plain, stream, reps)
    sp = obj.stats()
    ms_warm = _timed(run_warm, stream, reps)
    sw = obj.stats()
    if isinstance(sp, tuple):                   # batch: (rc, per-mesh stats, status)
        agg = lambda st, k: sum(x[k] for x in st[1])
        kp, kw = max(x["iterations"] for x in sp[1]), max(x["iterations"] for x in sw[1])
        up, uw = agg(sp, "vertex_updates"), agg(sw, "vertex_updates")
        rej, reach = agg(sw, "certify_rejected"), agg(sw, "reachable")
        rounds = max(x["certify_rounds"] for x in sw[1])
    else:
        kp, kw, up, uw = sp["iterations"], sw["iterations"], sp["vertex_updates"], sw["vertex_updates"]
        rej, reach, rounds = sw["certify_rejected"], sw["reachable"], sw["certify_rounds"]
    diff_max, _ = _rel(warm, plain)
    out = {"ms_to_converge_plain": round(ms_plain, 3), "ms_to_converge_warm": round(ms_warm, 3),
           "speedup": round(ms_plain / ms_warm, 3), "iterations_plain": kp, "iterations_warm": kw,
           "vertex_updates_plain": int(up), "vertex_updates_warm": int(uw),
           "certify_rejected_frac": round(rej / max(1, reach), 4), "certify_rounds_max": rounds,
           "max_rel_diff_warm_vs_plain": diff_max, "inflate": 1.05,
           "timed": f"3 warm-ups, median of {reps}; warm includes features, network and certification"}
    if fixed_point is not None:
        pm, pa = _rel(plain, fixed_point)
        wm, wa = _rel(warm, fixed_point)
        out.update({"plain_vs_fixed_point_max": pm, "plain_vs_fixed_point_mean": pa,
                    "warm_vs_fixed_point_max": wm, "warm_vs_fixed_point_mean": wa})
    return out


def batch_fixed_point(P, W, stream):
    """The fixed point d = min(d, U(d)) of every batch mesh (Jacobi on the
    GPU, float32), and its time."""
    import torch
    b = P.Batch(W.descs, TOL, band_rule=P.BAND_JACOBI)
    from paper_1810_08218_amd import autotune
    b.set_schedule(**autotune.BATCH512_SCHEDULE)
    b.prepare(W.dV, W.dF, W.dS, stream=stream)
    fp = torch.empty(W.out_len, dtype=torch.float32, device="cuda")
    ms = _timed(lambda: b.run(fp, stream=stream), stream, 1, warm=1)
    rc, st, _ = b.stats()
    out = {"ms": round(ms, 2), "status": rc, "max_sweeps": max(x["iterations"] for x in st),
           "vertex_updates": int(sum(x["vertex_updates"] for x in st))}
    b.close()
    return fp, out


def bench_batch_legs(P, W, H, stream, args):
    import torch
    from paper_1810_08218_amd import autotune
    b, dist = H["batch"], H["dist"]
    out = {}
    # critical path: the mesh that finished last
    st = H["stats"]
    last = max(range(len(st)), key=lambda t: st[t]["ms_mesh_end"])
    out["last_mesh"] = {"t": last, "name": W.meshes[last].name, "n": W.meshes[last].n,
                        "workgroups": st[last]["workgroups"], "iterations": st[last]["iterations"],
                        "vertex_updates": st[last]["vertex_updates"],
                        "ms_begin": round(st[last]["ms_mesh_begin"], 3), "ms_end": round(st[last]["ms_mesh_end"], 3)}
    ends = np.array([x["ms_mesh_end"] for x in st])
    out["mesh_end_ms_quantiles"] = [round(float(np.quantile(ends, q)), 2) for q in (0.5, 0.9, 0.99, 1.0)]
    note("batch: fixed point (Jacobi)")
    fp, out["fixed_point"] = batch_fixed_point(P, W, stream)
    e_max, e_mean = _rel(dist, fp)
    out["plain_vs_fixed_point"] = {"max": e_max, "mean": e_mean}
    if not args.no_warm:
        note("batch: learned warm start")
        b.set_window(0)
        out["warm_start"] = bench_warm(b, W.out_len, stream, 3, fixed_point=fp)
    del fp
    note("batch: one plan per mesh")
    plain_ms = 0.0
    for t, m in enumerate(W.meshes):
        d0 = W.descs[t]
        vo, fo, so = int(d0.v_off), int(d0.f_off), int(d0.s_off)
        p = P.Plan(m.n, m.f, m.m, TOL)
        p.prepare(W.dV[vo:vo + m.n], W.dF[fo:fo + m.f], W.dS[so:so + m.m], stream=stream)
        d = torch.empty(m.n, dtype=torch.float32, device="cuda")
        a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        p.run(d, stream=stream)
        z.record(stream)
        p.stats()
        plain_ms += a.elapsed_time(z)
        p.close()
    out["plain_ms_to_converge_sum"] = round(plain_ms, 3)
    out["speedup_vs_plain_per_mesh"] = round(plain_ms / H["ms_run"], 3)
    if not args.no_autotune:
        note("batch: autotuner (schedule candidates, then band cap)")
        tuned = autotune.tune(b, W.descs, dist, use_cache=False)
        b.run(dist, stream=stream)
        b.stats()
        tuned_ms = _timed(lambda: b.run(dist, stream=stream), stream, 2, warm=1)
        win = autotune.tune_window(b, dist)
        out["autotune"] = {"best_schedule": tuned["schedule"], "best_ms": round(tuned_ms, 3),
                           "timed_schedule": autotune.BATCH512_SCHEDULE, "timed_ms": round(H["ms_run"], 3),
                           "window": win["window"], "window_max_rel_diff_vs_unbounded": win["max_rel_diff"],
                           "window_tried": [[w, None if ms != ms else round(ms, 3), d] for w, ms, d in win["tried"]]}
        b.set_window(0)
        b.set_schedule(**autotune.BATCH512_SCHEDULE)
    return out


# --------------------------------------------------------- other configs ---

def bench_single(P, I, stream, args):
    """Noisy level-7 icosphere, one source (single mesh)."""
    import torch
    mesh = I.noisy_icosphere(level=7, seed=2)
    V, F, S = (torch.from_numpy(x).cuda() for x in (mesh.V, mesh.F, mesh.S))
    plan = P.Plan(mesh.n, mesh.f, mesh.m, TOL)
    work = plan.workspace()
    dist = torch.empty(mesh.n, dtype=torch.float32, device="cuda")

    def step():
        plan.prepare(V, F, S, work=work, stream=stream)
        plan.run(dist, stream=stream)
        return plan.stats()

    for _ in range(5):
        step()
    torch.cuda.synchronize()
    reps = 30
    t0 = time.perf_counter()
    runs, preps = [], []
    for _ in range(reps):
        st = step()
        runs.append(st["ms_run"])
        preps.append(st["ms_prepare"])
    ms_step = (time.perf_counter() - t0) * 1e3 / reps
    U = st["vertex_updates"]
    ms_run = statistics.mean(runs)
    out = {"workload": "noisy icosphere level 7 (163,842 vertices), 1 source, seed 2, tol 1e-4",
           "ms_per_step": round(ms_step, 4), "ms_to_converge": round(ms_run, 4),
           "ms_prepare": round(statistics.mean(preps), 4), "iterations": st["iterations"],
           "toplesets": st["n_toplesets"], "vertex_updates": U, "workgroups": st["workgroups"],
           "vertex_updates_per_s_step": round(U / (ms_step * 1e-3), 1),
           "vertex_updates_per_s_run": round(U / (ms_run * 1e-3), 1),
           "alg_GBps": round(U * BYTES_PER_UPDATE / (ms_run * 1e-3) / 1e9, 2)}
    # fixed point on the GPU (Jacobi), the error of the plain result
    pj = P.Plan(mesh.n, mesh.f, mesh.m, TOL, band_rule=P.BAND_JACOBI)
    pj.prepare(V, F, S, stream=stream)
    fp = torch.empty(mesh.n, dtype=torch.float32, device="cuda")
    pj.run(fp, stream=stream)
    sj = pj.stats()
    mx, mean = _rel(dist, fp)
    out["fixed_point"] = {"sweeps": sj["iterations"], "ms": round(sj["ms_run"], 3),
                          "plain_vs_fixed_point_max": mx, "plain_vs_fixed_point_mean": mean}
    pj.close()
    # the fixed half band of the complexity analysis against the paper's rule
    pf = P.Plan(mesh.n, mesh.f, mesh.m, TOL, band_rule=P.BAND_FIXED_HALF)
    pf.prepare(V, F, S, stream=stream)
    dfix = torch.empty(mesh.n, dtype=torch.float32, device="cuda")
    ms_f = _timed(lambda: pf.run(dfix, stream=stream), stream, 10)
    sf = pf.stats()
    out["fixed_half_band"] = {"ms_to_converge": round(ms_f, 4), "iterations": sf["iterations"],
                              "vertex_updates": sf["vertex_updates"],
                              "vs_fixed_point_max": _rel(dfix, fp)[0]}
    out["band_diagnostics"] = band_diagnostics(plan, pf, st, sf)
    pf.close()
    # float64 run of the same plan
    d64 = torch.empty(mesh.n, dtype=torch.float64, device="cuda")
    ms64 = _timed(lambda: plan.run_f64(d64, stream=stream), stream, 10)
    s64 = plan.stats()
    out["float64"] = {"ms_to_converge": round(ms64, 4), "iterations": s64["iterations"],
                      "vertex_updates": s64["vertex_updates"], "ms_ratio_f64_over_f32": round(ms64 / ms_run, 3),
                      "max_rel_diff_f32_vs_f64": _rel(dist, d64)[0]}
    plan.run(dist, stream=stream)
    plan.stats()
    if not args.no_warm:
        note("single mesh: learned warm start")
        out["warm_start"] = bench_warm(plan, mesh.n, stream, 20, fixed_point=fp)
    if not args.no_cpu_baseline:
        note("single mesh: CPU Fast Marching")
        fm_ms = cpu_fast_marching(mesh)
        out["cpu_fast_marching_ms"] = round(fm_ms, 2)
        out["speedup_step_vs_cpu_fast_marching"] = round(fm_ms / ms_step, 2)
    plan.close()
    return out, mesh


def band_diagnostics(plan, pf, st, sf):
    """Band per iteration from the retirement record (Sec. 6 figures: updated
    vertices and toplesets per iteration, dynamic band against the fixed
    half band), summarised."""
    from paper_1810_08218_amd import diagnostics as D
    _, offs = plan.order()
    offs = offs.cpu().numpy()
    dyn = D.band_trace(plan.schedule(), offs, st["iterations"])
    fix = D.band_trace(pf.schedule(), offs, sf["iterations"])
    rho = st["n_toplesets"]
    return {"rho": rho, "K_dynamic": st["iterations"], "K_fixed": sf["iterations"],
            "K_over_rho_dynamic": round(st["iterations"] / rho, 3),
            "max_band_toplesets_dynamic": int(dyn["toplesets"].max()),
            "max_band_toplesets_fixed": int(fix["toplesets"].max()),
            "mean_band_toplesets_dynamic": round(float(dyn["toplesets"].mean()), 2),
            "mean_band_toplesets_fixed": round(float(fix["toplesets"].mean()), 2),
            "U_dynamic": int(dyn["vertices"].sum()), "U_fixed": int(fix["vertices"].sum())}


def bench_grids(P, I, stream):
    """Flat grids: the 64 x 64 workload (tol 1e-6) and the 1001 x 1001 grid of
    the paper's accuracy figure (corner and centre source), with the mean
    absolute percent error against the Euclidean distance."""
    import torch
    out = {}
    for name, mesh, tol in (("flat_grid_64_tol1e-6", I.flat_grid(64), 1e-6),
                            ("flat_grid_1001_corner_tol1e-6", I.flat_grid(1001), 1e-6),
                            ("flat_grid_1001_centre_tol1e-6", I.flat_grid(1001, source=(500, 500)), 1e-6)):
        V, F, S = (torch.from_numpy(x).cuda() for x in (mesh.V, mesh.F, mesh.S))
        plan = P.Plan(mesh.n, mesh.f, mesh.m, tol)
        plan.prepare(V, F, S, stream=stream)
        d = torch.empty(mesh.n, dtype=torch.float32, device="cuda")
        ms = _timed(lambda: plan.run(d, stream=stream), stream, 5)
        st = plan.stats()
        X = mesh.V.astype(np.float64)
        eu = np.linalg.norm(X - X[mesh.S[0]], axis=1)
        g = d.cpu().numpy().astype(np.float64)
        m = eu > 0
        mape = float(np.mean(np.abs(g[m] - eu[m]) / eu[m]) * 100)
        out[name] = {"n_vertices": mesh.n, "ms_to_converge": round(ms, 4), "ms_prepare": round(st["ms_prepare"], 3),
                     "iterations": st["iterations"], "toplesets": st["n_toplesets"],
                     "vertex_updates": st["vertex_updates"], "mape_vs_euclid_percent": round(mape, 4)}
        plan.close()
    return out


def bench_bumpy9(P, I, stream, args, full=True):
    """Level-9 bumpy icosphere, 32 sources: labelled run; unless `full` is
    false, the learned warm start (distances only) and Lloyd steps on its
    Voronoi cells."""
    import torch
    mesh = I.bumpy_icosphere(level=9, seed=3, n_sources=32)
    V, F, S = (torch.from_numpy(x).cuda() for x in (mesh.V, mesh.F, mesh.S))
    plan = P.Plan(mesh.n, mesh.f, mesh.m, TOL, want_labels=True)
    work = plan.workspace()
    d = torch.empty(mesh.n, dtype=torch.float32, device="cuda")
    lab = torch.empty(mesh.n, dtype=torch.int32, device="cuda")
    for _ in range(4):
        plan.prepare(V, F, S, work=work, stream=stream)
    ms = _timed(lambda: plan.run(d, lab, stream=stream), stream, 10)
    st = plan.stats()
    U = st["vertex_updates"]
    out = {"workload": "bumpy icosphere level 9 (2,621,442 vertices), 32 sources, labels, seed 3, tol 1e-4",
           "ms_to_converge": round(ms, 4), "ms_prepare": round(st["ms_prepare"], 3),
           "iterations": st["iterations"], "toplesets": st["n_toplesets"], "vertex_updates": U,
           "vertex_updates_per_s_run": round(U / (ms * 1e-3), 1), "workgroups": st["workgroups"],
           "alg_GBps": round(U * BYTES_PER_UPDATE / (ms * 1e-3) / 1e9, 1)}   # label passes timed, not counted
    if not full:
        plan.close()
        return out
    # Lloyd steps on the Voronoi cells (a few iterations: prepare, labelled run, step)
    Sg = S.clone()
    t0 = time.perf_counter()
    iters = 5
    for _ in range(iters):
        plan.prepare(V, F, Sg, work=work, stream=stream)
        plan.run(d, lab, stream=stream)
        S2 = torch.empty_like(Sg)
        plan.lloyd_step(lab, S2, stream=stream)
        Sg = S2
    torch.cuda.synchronize()
    out["lloyd"] = {"iterations": iters, "ms_per_iteration": round((time.perf_counter() - t0) * 1e3 / iters, 3),
                    "generators_moved_last": int((Sg != S).sum())}
    plan.close()
    if not args.no_warm:
        note("bumpy L9: learned warm start (distances only)")
        pw = P.Plan(mesh.n, mesh.f, mesh.m, TOL)
        pw.prepare(V, F, S, stream=stream)
        pj = P.Plan(mesh.n, mesh.f, mesh.m, TOL, band_rule=P.BAND_JACOBI)
        pj.prepare(V, F, S, stream=stream)
        fp = torch.empty(mesh.n, dtype=torch.float32, device="cuda")
        pj.run(fp, stream=stream)
        sj = pj.stats()
        pj.close()
        out["warm_start"] = bench_warm(pw, mesh.n, stream, 5, fixed_point=fp)
        out["fixed_point_sweeps"] = sj["iterations"]
        pw.close()
    return out


def bench_fps(P, mesh, stream, ms_list=(10, 100, 1000)):
    """Farthest point sampling on the noisy level-7 icosphere from its source:
    GPU time to reach m samples, cold (every map from +inf) and warm (from the
    previous map), against sequential Fast Marching on the CPU (the same map
    per sample: time of one FM solve x (m - 1), from the measured FM time)."""
    import torch
    V, F = (torch.from_numpy(x).cuda() for x in (mesh.V, mesh.F))
    out = {}
    for m in ms_list:
        row = {}
        for warm in (False, True):
            plan = P.Plan(mesh.n, mesh.f, m, TOL)
            S = torch.zeros(m, dtype=torch.int32, device="cuda")
            S[0] = int(mesh.S[0])
            dist = torch.empty(mesh.n, dtype=torch.float32, device="cuda")
            steps = torch.empty(2 * m, dtype=torch.int64, device="cuda")
            plan.fps(V, F, S, 1, dist, steps=steps, warm=warm, stream=stream)     # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.fps(V, F, S, 1, dist, steps=steps, warm=warm, stream=stream)
            ms = (time.perf_counter() - t0) * 1e3
            stp = steps.cpu().numpy().reshape(-1, 2)
            row["warm" if warm else "cold"] = {"ms": round(ms, 2), "vertex_updates": int(stp[:, 1].sum()),
                                               "iterations": int(stp[:, 0].sum())}
            plan.close()
        row["speedup_warm_vs_cold"] = round(row["cold"]["ms"] / row["warm"]["ms"], 3)
        out[f"m{m}"] = row
    return out


def bench_source_sets(P, I, stream, sets=64, steps=3):
    """The 2.6M-vertex bumpy icosphere with 64 seeded sets of 32 sources
    (labels, tol 1e-4): one batch whose meshes share the V and F rows,
    against one plan re-prepared per source set (run time summed)."""
    import torch
    base = I.bumpy_icosphere(level=9, seed=3, n_sources=32)
    rng = np.random.default_rng(31)
    meshes = [I.Mesh(base.V, base.F, rng.choice(base.n, 32, replace=False).astype(np.int32), name=f"set{k}")
              for k in range(sets)]
    V, F, S, descs, out_len = P.concat(meshes, [None] + [0] * (sets - 1))
    dV, dF, dS = (torch.from_numpy(x).cuda() for x in (V, F, S))
    b = P.Batch(descs, TOL, want_labels=True)
    work = b.workspace()
    dist = torch.empty(out_len, dtype=torch.float32, device="cuda")
    lab = torch.empty(out_len, dtype=torch.int32, device="cuda")
    b.prepare(dV, dF, dS, work=work, stream=stream)
    b.set_schedule(workgroups=1 << 20, small_limit=1, large_limit=1, large_group=16)
    runs = []
    for _ in range(steps):
        b.prepare(dV, dF, dS, work=work, stream=stream)
        a1, a2 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a1.record(stream)
        b.run(dist, lab, stream=stream)
        a2.record(stream)
        rc, stats, _ = b.stats()
        runs.append(a1.elapsed_time(a2))
    ms_run = statistics.median(runs)
    U = sum(x["vertex_updates"] for x in stats)
    plan = P.Plan(base.n, base.f, 32, TOL, want_labels=True)
    d1 = torch.empty(base.n, dtype=torch.float32, device="cuda")
    l1 = torch.empty(base.n, dtype=torch.int32, device="cuda")
    single_ms = 0.0
    for m in meshes:
        plan.prepare(dV[:base.n], dF[:base.f], torch.from_numpy(m.S).cuda(), stream=stream)
        plan.run(d1, l1, stream=stream)
        single_ms += plan.stats()["ms_run"]
    alg = U * BYTES_PER_UPDATE          # the label passes are timed, their bytes not counted
    out = {"workload": f"bumpy icosphere level 9 x {sets} source sets of 32, labels, tol 1e-4, seed 31",
           "status": rc, "ms_to_converge": round(ms_run, 3), "vertex_updates": int(U),
           "vertex_updates_per_s": round(U / (ms_run * 1e-3), 1),
           "alg_frac_of_hbm": round(alg / (ms_run * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "single_plan_ms_to_converge_sum": round(single_ms, 3),
           "speedup_vs_single_plans": round(single_ms / ms_run, 3), "workspace_GB": round(work.numel() / 1e9, 2)}
    b.close()
    plan.close()
    return out


# ------------------------------------------------------------------ main ---

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--only", choices=["all", "batch", "l9"], default="all",
                    help="batch: the timed batch steps only (for profiling the timed launch); "
                         "l9: the labelled runs of the level-9 bumpy icosphere only")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-warm", action="store_true", help="skip the learned warm-start legs")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-source-sets", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run 3 device copies of 256 MiB (a kernel of known traffic for "
                         "scaling the rocprofv3 FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(independent meshes shard without communication; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1810_08218_amd as P
    from paper_1810_08218_amd import inputs as I

    P.load()
    stream = torch.cuda.current_stream()
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.only == "l9":
        note("bumpy icosphere level 9 (labelled runs only)")
        out = bench_bumpy9(P, I, stream, args, full=False)
        gc.collect()
        torch.cuda.synchronize()
        print(json.dumps({"workload": out["workload"], "bumpy_icosphere_l9": out}), flush=True)
        return

    W = BatchWorkload(P, I)
    H = bench_batch_steps(P, W, args.steps, args.warmup, stream)
    U, ms_step, ms_run = H["U"], H["ms_step"], H["ms_run"]
    EV = sum(x["evaluated_updates"] for x in H["stats"])
    alg_bytes = U * BYTES_PER_UPDATE
    achieved = alg_bytes / (ms_run * 1e-3) / 1e9
    traffic = measured_traffic()
    # the bytes the kernel has to move once unchanged band vertices are
    # skipped: 48 B per evaluated update, the 4-byte mark per skipped one
    model = EV * BYTES_PER_UPDATE + (U - EV) * BYTES_PER_SKIP
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
                "kernel": "k_relax<float,false,false,false> (batched persistent band relaxation)",
                "alg_bytes_per_launch": alg_bytes, "bytes_per_update": BYTES_PER_UPDATE,
                "avg_launch_ms": round(ms_run, 3),
                "evaluated_updates": EV,
                "skip_model_bytes_per_launch": model,
                "skip_model_frac": round(model / (ms_run * 1e-3) / 1e9 / HBM_PEAK_GBS, 5),
                "traffic_frac": None if traffic is None else round(traffic / (ms_run * 1e-3) / 1e9 / HBM_PEAK_GBS, 5)}
    line = {
        "metric": METRIC,
        "value": round(U / (ms_step * 1e-3), 1),
        "unit": "vertex-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batch512: 256 jittered grids (side 32..1024) + 256 tori (2^k x 2^(k-1), "
                               "k=5..10), 1-4 sources each, seed 4, tol 1e-4",
                   "n_meshes": 512, "n_vertices": W.n, "n_faces": W.f, "tol": TOL, "parallelism": "none",
                   "schedule": H["batch"].get_schedule()},
        "ms_to_converge": round(ms_run, 3),
        "ms_to_converge_min": round(H["ms_run_min"], 3),
        "ms_prepare": round(H["ms_prepare"], 3),
        "status": H["rc"],
        "vertex_updates": U,
        "evaluated_updates": EV,
        "vertex_updates_per_s_run": round(U / (ms_run * 1e-3), 1),
        "max_iterations": max(x["iterations"] for x in H["stats"]),
        "max_toplesets": max(x["n_toplesets"] for x in H["stats"]),
        "roofline": roofline,
    }
    if args.only == "batch":
        H["batch"].close()
        del H, W
        gc.collect()
        torch.cuda.synchronize()
        print(json.dumps(line), flush=True)
        return

    line["batched"] = bench_batch_legs(P, W, H, stream, args)
    H["batch"].close()
    del H
    gc.collect()
    torch.cuda.empty_cache()
    cpu = allc = None
    if not args.no_cpu_baseline:
        note("CPU baseline (oracle, one core, then all cores)")
        cpu, allc = cpu_baseline(W.meshes)
    line["cpu_baseline"] = cpu
    line["cpu_all_cores"] = allc
    line["host"] = host_info()
    del W
    gc.collect()
    torch.cuda.empty_cache()
    note("flat grids")
    line["grids"] = bench_grids(P, I, stream)
    note("noisy icosphere level 7")
    single, l7 = bench_single(P, I, stream, args)
    line["single_mesh"] = single
    note("farthest point sampling")
    line["fps"] = bench_fps(P, l7, stream)
    if "cpu_fast_marching_ms" in single:
        line["fps"]["cpu_fast_marching_ms_per_map"] = single["cpu_fast_marching_ms"]
        for key, row in line["fps"].items():
            if key.startswith("m"):
                m = int(key[1:])
                est = single["cpu_fast_marching_ms"] * (m - 1)
                row["cpu_fast_marching_estimate_ms"] = round(est, 1)
                row["speedup_warm_vs_cpu_fast_marching"] = round(est / row["warm"]["ms"], 1)
    note("bumpy icosphere level 9")
    line["bumpy_icosphere_l9"] = bench_bumpy9(P, I, stream, args)
    if not args.no_source_sets:
        note("64 source sets on the level-9 icosphere")
        line["source_sets"] = bench_source_sets(P, I, stream)
    gc.collect()
    torch.cuda.synchronize()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
