"""Benchmark of the PTP hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

One step is the whole path on one mesh already resident in HBM: validation,
incidence, BFS toplesets, reorder (ptp_prepare) and the persistent band
relaxation with unpermute (ptp_run).  Workload: unit icosphere subdivided 7
times (163,842 vertices, 327,680 triangles) with tangential noise of 0.1 x
mean edge length, one random source (seed 2), tolerance 1e-4.

Prints ONE JSON line: vertex-updates/s over whole steps (value), ms per step,
ms to converge (ptp_run alone), the roofline of the relaxation kernel, the
oracle's single-thread CPU rate on the same mesh, and the max relative error
of the GPU distances against the oracle.  Alongside ("batched"): the 512-mesh
uneven batch (jittered grids and tori, 71M vertices) in one persistent launch
with an autotuned schedule and band cap (window; the fastest whose result
stays within 1e-4 of the unbounded run's), against the same meshes run one
plan at a time with the paper's unbounded band;
and ("warm_start", for the single mesh and the batch) the learned warm start
against the plain run at the same tolerance.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E
BYTES_PER_UPDATE = 48           # own xyz 12 + d read 4 + d write 4 + row 4 + 6 neighbour ids 24
BYTES_PER_UPDATE_LABELS = 8     # label read + write
RELAX_SRC = os.path.join(ROOT, "paper_1810_08218_amd", "csrc", "ptp_relax.hip")
PMC_FILE = os.path.join(ROOT, "profiles", "relax_noisy_icosphere7_pmc.json")


def relax_source_hash() -> str:
    with open(RELAX_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per relaxation launch from the committed rocprofv3 counter
    summary, only while the kernel source is the one that was profiled."""
    if not os.path.exists(PMC_FILE):
        return None
    with open(PMC_FILE) as fh:
        rec = json.load(fh)
    if rec.get("relax_source_sha256_16") != relax_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(mesh, tol, budget_s=12.0):
    import oracle as O
    t_all = []
    res = None
    t_start = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        res = O.run(mesh.V, mesh.F, mesh.S, tol)
        t_all.append(time.perf_counter() - t0)
        if time.perf_counter() - t_start > budget_s or len(t_all) >= 5:
            break
    t = statistics.median(t_all)
    return res, {"value": res.updates / t, "unit": "vertex-updates/s", "cores": 1, "kind": "oracle",
                 "sample": f"{len(t_all)} full FP64 solve(s) of the same mesh by the sequential "
                           f"oracle (median {t * 1e3:.0f} ms each, U={res.updates})"}


def note(msg):
    """Progress line on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _timed(fn, stream, reps):
    """Median device time (ms) of fn() over reps runs after 3 warm-ups."""
    import torch
    for _ in range(3):
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


def bench_warm(obj, n_out, stream, reps):
    """Learned warm start against the plain run on a prepared plan or batch:
    ms to converge of (features + network + certified run) vs (run), both
    3 warm-ups then the median of `reps`; iterations, updates and the
    largest relative difference of the results."""
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
    p, w = plain.double(), warm.double()
    fin = torch.isfinite(p) & (p > 0)
    diff = (w[fin] - p[fin]) / p[fin]
    rel = float(diff.abs().max())
    lower = float((diff < -1e-4).double().mean())     # warm clearly below (closer to the fixed point)
    higher = float((diff > 1e-4).double().mean())
    return {"ms_to_converge_plain": round(ms_plain, 3), "ms_to_converge_warm": round(ms_warm, 3),
            "speedup": round(ms_plain / ms_warm, 3), "iterations_plain": kp,
            "iterations_warm": kw, "vertex_updates_plain": int(up), "vertex_updates_warm": int(uw),
            "certify_rejected_frac": round(rej / max(1, reach), 4), "certify_rounds_max": rounds,
            "max_rel_diff_warm_vs_plain": rel, "frac_warm_below_plain_1e-4": round(lower, 6),
            "frac_warm_above_plain_1e-4": round(higher, 6), "inflate": 1.05,
            "timed": f"3 warm-ups, median of {reps}; warm includes features, network and "
                     f"certification"}


def bench_other_configs(P, I, reps=10):
    """The flat 64 x 64 grid (tol 1e-6) and the 2.6M-vertex bumpy icosphere
    with 32 sources and Voronoi labels (tol 1e-4): ms to converge (ptp_run,
    median of reps after warm-up), ms to prepare, vertex updates per second
    of the run."""
    import torch
    out = {}
    for name, mesh, tol, labels in (("flat_grid_64_tol1e-6", I.flat_grid(64), 1e-6, False),
                                    ("bumpy_icosphere_l9_32src_labels_tol1e-4",
                                     I.bumpy_icosphere(level=9, seed=3, n_sources=32), 1e-4, True)):
        note(f"config {name}")
        V, F, S = (torch.from_numpy(x).cuda() for x in (mesh.V, mesh.F, mesh.S))
        plan = P.Plan(mesh.n, mesh.f, mesh.m, tol, want_labels=labels)
        work = plan.workspace()
        stream = torch.cuda.current_stream()
        dist = torch.empty(mesh.n, dtype=torch.float32, device="cuda")
        lab = torch.empty(mesh.n, dtype=torch.int32, device="cuda") if labels else None
        t0 = time.perf_counter()
        plan.prepare(V, F, S, work=work, stream=stream)
        prep = []
        for _ in range(3):
            t0 = time.perf_counter()
            plan.prepare(V, F, S, work=work, stream=stream)
            prep.append((time.perf_counter() - t0) * 1e3)
        ms = _timed(lambda: plan.run(dist, lab, stream=stream), stream, reps)
        st = plan.stats()
        out[name] = {"n_vertices": mesh.n, "n_sources": mesh.m, "labels": labels, "tol": tol,
                     "ms_to_converge": round(ms, 4), "ms_prepare_and_sync": round(min(prep), 4),
                     "iterations": st["iterations"], "toplesets": st["n_toplesets"],
                     "vertex_updates": st["vertex_updates"],
                     "vertex_updates_per_s": round(st["vertex_updates"] / (ms * 1e-3), 1),
                     "workgroups": st["workgroups"]}
    return out


def bench_batched(steps, P, I, warm=True):
    """512 uneven meshes in one persistent launch vs one plan per mesh."""
    import torch
    from paper_1810_08218_amd import autotune
    note("batched: generating 512 meshes")
    meshes = I.batch_meshes(512)
    V, F, S, descs, out_len = P.concat(meshes)
    dV, dF, dS = (torch.from_numpy(x).cuda() for x in (V, F, S))
    del V, F
    tol = 1e-4
    b = P.Batch(descs, tol)
    work = b.workspace()
    dist = torch.empty(out_len, dtype=torch.float32, device="cuda")
    b.prepare(dV, dF, dS, work=work)
    note("batched: autotuning the schedule")
    tuned = autotune.tune(b, descs, dist, use_cache=False)
    note("batched: autotuning the window against the unbounded run")
    win = autotune.tune_window(b, dist)
    stream = torch.cuda.current_stream()
    b.run(dist, stream=stream)              # warm-up with the tuned schedule
    rc, stats, _ = b.stats()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        b.prepare(dV, dF, dS, work=work, stream=stream)
        ev[k][0].record(stream)
        b.run(dist, stream=stream)
        ev[k][1].record(stream)
        rc, stats, _ = b.stats()
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / steps
    ms_run = statistics.mean(a.elapsed_time(z) for a, z in ev)
    U = sum(x["vertex_updates"] for x in stats)
    # the same meshes, one plan each (run only)
    note("batched: one plan per mesh")
    plain_ms = 0.0
    for m in meshes:
        Vm, Fm, Sm = (torch.from_numpy(x).cuda() for x in (m.V, m.F, m.S))
        p = P.Plan(m.n, m.f, m.m, tol)
        p.prepare(Vm, Fm, Sm)
        d = torch.empty(m.n, dtype=torch.float32, device="cuda")
        a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        p.run(d)
        z.record()
        p.stats()
        plain_ms += a.elapsed_time(z)
    alg = U * BYTES_PER_UPDATE
    return {"workload": "512 uneven meshes: jittered grids 32..1024 and tori 2^k x 2^(k-1), "
                        "k=5..10, 1-4 sources, seed 4, tol 1e-4",
            "n_vertices": int(sum(m.n for m in meshes)), "status": rc,
            "ms_to_converge": round(ms_run, 3), "ms_per_step": round(ms_step, 3),
            "vertex_updates": int(U), "vertex_updates_per_s": round(U / (ms_run * 1e-3), 1),
            "alg_GBps": round(alg / (ms_run * 1e-3) / 1e9, 1),
            "alg_frac_of_hbm": round(alg / (ms_run * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "plain_ms_to_converge_sum": round(plain_ms, 3),
            "speedup_vs_plain": round(plain_ms / ms_run, 3),
            "schedule": tuned["schedule"],
            "window": win["window"],
            "window_max_rel_diff_vs_unbounded": win["max_rel_diff"],
            "window_tried_ms": [[w, None if ms != ms else round(ms, 3), d] for w, ms, d in win["tried"]],
            "max_iterations": max(x["iterations"] for x in stats),
            "max_toplesets": max(x["n_toplesets"] for x in stats),
            "warm_start": bench_warm(b, out_len, stream, 3) if warm else None}


def bench_source_sets(P, I, sets=64, steps=3):
    """The 2.6M-vertex bumpy icosphere with 64 seeded sets of 32 sources
    (Voronoi labels, tol 1e-4): one batch whose meshes share the V and F rows,
    against one plan re-prepared per source set (run time summed)."""
    import torch
    note(f"source sets: bumpy icosphere level 9 x {sets} source sets")
    base = I.bumpy_icosphere(level=9, seed=3, n_sources=32)
    rng = np.random.default_rng(31)
    meshes = [I.Mesh(base.V, base.F, rng.choice(base.n, 32, replace=False).astype(np.int32),
                     name=f"set{k}") for k in range(sets)]
    V, F, S, descs, out_len = P.concat(meshes, [None] + [0] * (sets - 1))
    dV, dF, dS = (torch.from_numpy(x).cuda() for x in (V, F, S))
    tol = 1e-4
    b = P.Batch(descs, tol, want_labels=True)
    work = b.workspace()
    dist = torch.empty(out_len, dtype=torch.float32, device="cuda")
    lab = torch.empty(out_len, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    b.prepare(dV, dF, dS, work=work, stream=stream)
    best = None
    for lg in (16, 32, 64):
        b.set_schedule(workgroups=1 << 20, small_limit=1, large_limit=1, large_group=lg)
        ms = _timed(lambda: b.run(dist, lab, stream=stream), stream, 2)
        if best is None or ms < best[0]:
            best = (ms, lg)
    b.set_schedule(workgroups=1 << 20, small_limit=1, large_limit=1, large_group=best[1])
    prep, runs = [], []
    for _ in range(steps):
        a0, a1, a2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        a0.record(stream)
        b.prepare(dV, dF, dS, work=work, stream=stream)
        a1.record(stream)
        b.run(dist, lab, stream=stream)
        a2.record(stream)
        rc, stats, _ = b.stats()
        prep.append(a0.elapsed_time(a1))
        runs.append(a1.elapsed_time(a2))
    ms_run = statistics.median(runs)
    U = sum(x["vertex_updates"] for x in stats)
    note("source sets: one plan per source set")
    plan = P.Plan(base.n, base.f, 32, tol, want_labels=True)
    d1 = torch.empty(base.n, dtype=torch.float32, device="cuda")
    l1 = torch.empty(base.n, dtype=torch.int32, device="cuda")
    single_ms, same = 0.0, True
    for k, m in enumerate(meshes):
        plan.prepare(dV[:base.n], dF[:base.f], torch.from_numpy(m.S).cuda(), stream=stream)
        a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        plan.run(d1, l1, stream=stream)
        z.record(stream)
        plan.stats()
        single_ms += a.elapsed_time(z)
        if k < 4:
            o0 = int(descs[k].out_off)
            same &= bool(torch.equal(d1, dist[o0:o0 + base.n]) and torch.equal(l1, lab[o0:o0 + base.n]))
    alg = U * (BYTES_PER_UPDATE + 8)
    return {"workload": f"bumpy icosphere level 9 (2,621,442 vertices) x {sets} source sets of 32, "
                        "labels, tol 1e-4, seed 31",
            "status": rc, "ms_to_converge": round(ms_run, 3), "ms_prepare": round(statistics.median(prep), 3),
            "vertex_updates": int(U), "vertex_updates_per_s": round(U / (ms_run * 1e-3), 1),
            "alg_GBps": round(alg / (ms_run * 1e-3) / 1e9, 1),
            "alg_frac_of_hbm": round(alg / (ms_run * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "bytes_per_update": BYTES_PER_UPDATE + 8, "large_group": best[1],
            "single_plan_ms_to_converge_sum": round(single_ms, 3),
            "speedup_vs_single_plans": round(single_ms / ms_run, 3),
            "first_4_sets_identical_to_single_plans": same,
            "workspace_GB": round(work.numel() / 1e9, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workgroups", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=5)
    ap.add_argument("--no-warm", action="store_true", help="skip the learned warm-start legs")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the flat-grid and bumpy-icosphere timings")
    ap.add_argument("--no-source-sets", action="store_true",
                    help="skip the 64-source-set batch on the level-9 icosphere")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run 3 device copies of 256 MiB (a kernel of known traffic for "
                         "scaling the rocprofv3 FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(independent meshes shard without communication; see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1810_08218_amd as P
    from paper_1810_08218_amd import inputs as I

    P.load()
    tol = 1e-4
    mesh = I.noisy_icosphere(level=7, seed=2)
    dev = torch.device("cuda:0")
    V = torch.from_numpy(mesh.V).to(dev)
    F = torch.from_numpy(mesh.F).to(dev)
    S = torch.from_numpy(mesh.S).to(dev)
    plan = P.Plan(mesh.n, mesh.f, mesh.m, tol, workgroups=args.workgroups)
    work = plan.workspace(dev)
    dist = torch.empty(mesh.n, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        plan.prepare(V, F, S, work=work, stream=stream)
        if ev is not None:
            ev[0].record(stream)
        plan.run(dist, stream=stream)
        if ev is not None:
            ev[1].record(stream)
        return plan.stats()

    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    note(f"single mesh: {args.warmup} warm-up + {args.steps} timed steps")
    for _ in range(args.warmup):
        st = step()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        st = step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    run_ms = [a.elapsed_time(b) for a, b in evs]
    ms_step = (t1 - t0) * 1e3 / args.steps
    ms_run = statistics.mean(run_ms)
    U = st["vertex_updates"]
    value = U / (ms_step * 1e-3)

    alg_bytes = U * BYTES_PER_UPDATE
    achieved = alg_bytes / (ms_run * 1e-3) / 1e9
    traffic = measured_traffic()
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
                "kernel": "k_relax (persistent band relaxation)",
                "alg_bytes_per_launch": alg_bytes, "avg_launch_ms": round(ms_run, 4)}

    gpu_d = dist.cpu().numpy().astype(np.float64)
    cpu = None
    max_rel = None
    if not args.no_cpu_baseline:
        note("CPU baseline (oracle)")
        res, cpu = cpu_baseline(mesh, tol)
        o = res.dist
        mask = np.isfinite(o) & (o > 0)
        max_rel = float(np.max(np.abs(gpu_d[mask] - o[mask]) / o[mask]))
        same_sched = bool(np.array_equal(plan.schedule(), res.retire_k))
    note("warm start on the single mesh")
    warm = None if args.no_warm else bench_warm(plan, mesh.n, stream, 20)
    batched = None if args.no_batched else bench_batched(args.batched_steps, P, I,
                                                         warm=not args.no_warm)
    line = {
        "metric": "vertex-updates/s at <=1e-4 rel err (ms to converge alongside)",
        "value": round(value, 1),
        "unit": "vertex-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "noisy_icosphere_l7_1src_tol1e-4", "n_vertices": mesh.n,
                   "n_faces": mesh.f, "n_sources": mesh.m, "tol": tol, "parallelism": "none"},
        "ms_to_converge": round(ms_run, 4),
        "ms_prepare_and_sync": round(ms_step - ms_run, 4),
        "iterations": st["iterations"],
        "toplesets": st["n_toplesets"],
        "vertex_updates": U,
        "workgroups": st["workgroups"],
        "roofline": roofline,
        "cpu_baseline": cpu,
        "max_rel_err_vs_oracle": max_rel,
    }
    if cpu is not None:
        line["schedule_matches_oracle"] = same_sched
    line["warm_start"] = warm
    line["other_configs"] = None if args.no_configs else bench_other_configs(P, I)
    line["batched"] = batched
    line["source_sets"] = None if (args.no_source_sets or args.no_batched) else bench_source_sets(P, I)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
