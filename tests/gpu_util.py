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
            lds_bfs_max=0, band_rule=0, f64=False):
    import torch
    say(f"[gpu] {mesh.name} n={mesh.n} f={mesh.f} m={mesh.m} tol={tol} labels={labels} "
        f"wg={workgroups} max_iters={max_iters} window={window} lds_bfs_max={lds_bfs_max} "
        f"band_rule={band_rule} f64={f64}")
    V, F, S = to_dev(mesh)
    plan = P.Plan(mesh.n, mesh.f, mesh.m, tol, max_iters=max_iters, window=window,
                  want_labels=labels, workgroups=workgroups, lds_bfs_max=lds_bfs_max,
                  band_rule=band_rule)
    plan.prepare(V, F, S)
    dist = torch.empty(mesh.n, dtype=torch.float64 if f64 else torch.float32, device="cuda")
    lab = torch.empty(mesh.n, dtype=torch.int32, device="cuda") if labels else None
    if f64:
        plan.run_f64(dist)
    else:
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


def label_candidates(mesh, v, dist, label):
    """Per source label, the smallest planar update the vertex v receives from
    its incident triangles under the map (dist, label) (caller order): the
    distance each competing front offers v.  Computed with the oracle's local
    update (the label of a planar value is that of its smaller input, an edge
    update that of its vertex)."""
    import oracle as O
    X = np.asarray(mesh.V, np.float64)
    cand = {}
    for t in np.nonzero((mesh.F == v).any(axis=1))[0]:
        f = [int(x) for x in mesh.F[t]]
        c = f.index(v)
        a, b = f[(c + 1) % 3], f[(c + 2) % 3]
        u, who = O.local_update(X[v], X[a], X[b], dist[a], dist[b])
        if not np.isfinite(u):
            continue
        if who == 1:
            lab = label[a] if dist[a] != dist[b] or np.isinf(dist[b]) else min(label[a], label[b])
        else:
            lab = label[b] if dist[a] != dist[b] or np.isinf(dist[a]) else min(label[a], label[b])
        lab = int(lab)
        cand[lab] = min(cand.get(lab, np.inf), u)
    return cand


def check_labels(mesh, g_lab, o_lab, o_dist, rel=1e-4):
    """Labels equal the oracle's except where two fronts arrive within `rel`
    (relative) of each other: at every mismatch the GPU's label must offer
    the vertex a distance within `rel` of the best one under the oracle's
    map.  Returns the number of mismatches."""
    bad = np.nonzero(np.asarray(g_lab) != np.asarray(o_lab))[0]
    for v in bad:
        cand = label_candidates(mesh, int(v), o_dist, o_lab)
        best = min(cand.values())
        lg = int(g_lab[v])
        assert lg in cand, f"vertex {v}: label {lg} is not offered by any incident triangle"
        assert cand[lg] <= best * (1 + rel) + 1e-30, \
            f"vertex {v}: label {lg} offers {cand[lg]:.9g}, best {best:.9g}"
    return int(bad.size)
