"""Helpers for the GPU tests: run a mesh through the C ABI (via the binding)
and compare with the oracle."""
from __future__ import annotations

import sys

import numpy as np

import paper_1810_08218_amd as P


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(mesh, device="cuda"):
    import torch
    V = torch.from_numpy(np.ascontiguousarray(mesh.V, np.float32)).to(device)
    F = torch.from_numpy(np.ascontiguousarray(mesh.F, np.int32)).to(device)
    S = torch.from_numpy(np.ascontiguousarray(mesh.S, np.int32)).to(device)
    return V, F, S


class GpuResult:
    pass


def gpu_run(mesh, tol, labels=False, workgroups=0, max_iters=0, window=0, want_order=True,
            lds_bfs_max=0):
    import torch
    say(f"[gpu] {mesh.name} n={mesh.n} f={mesh.f} m={mesh.m} tol={tol} labels={labels} "
        f"wg={workgroups} max_iters={max_iters} window={window} lds_bfs_max={lds_bfs_max}")
    V, F, S = to_dev(mesh)
    plan = P.Plan(mesh.n, mesh.f, mesh.m, tol, max_iters=max_iters, window=window,
                  want_labels=labels, workgroups=workgroups, lds_bfs_max=lds_bfs_max)
    plan.prepare(V, F, S)
    dist = torch.empty(mesh.n, dtype=torch.float32, device="cuda")
    lab = torch.empty(mesh.n, dtype=torch.int32, device="cuda") if labels else None
    plan.run(dist, lab)
    st = plan.stats()
    r = GpuResult()
    r.stats = st
    r.status = st["status"]
    r.dist = dist.cpu().numpy()
    r.label = lab.cpu().numpy() if labels else None
    r.iterations = st["iterations"]
    r.rho = st["n_toplesets"]
    r.updates = st["vertex_updates"]
    r.retire = plan.schedule()
    if want_order:
        perm, offs = plan.order()
        r.perm = perm.cpu().numpy()
        r.offsets = offs.cpu().numpy()
    r.plan = plan
    torch.cuda.synchronize()
    return r


def rel_errors(g, o, S):
    """max and mean |g - o| / o over non-source vertices with finite o."""
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    mask = np.isfinite(o) & (o > 0)
    mask[np.asarray(S)] = False
    e = np.abs(g[mask] - o[mask]) / o[mask]
    return (float(e.max()) if e.size else 0.0), (float(e.mean()) if e.size else 0.0)
