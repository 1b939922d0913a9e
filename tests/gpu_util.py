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
    r.parent = plan.parents().cpu().numpy() if labels and not f64 else None
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


class _Faces:
    """Vertex -> incident faces (CSR), built once per mesh."""

    def __init__(self, F, n):
        F = np.asarray(F)
        cnt = np.bincount(F.ravel(), minlength=n)
        self.start = np.zeros(n + 1, np.int64)
        self.start[1:] = np.cumsum(cnt)
        self.face = np.argsort(F.ravel(), kind="stable") // 3
        self.F = F

    def wedges(self, v):
        for t in self.face[self.start[v]:self.start[v + 1]]:
            f = [int(x) for x in self.F[t]]
            c = f.index(v)
            yield f[(c + 1) % 3], f[(c + 2) % 3]


def parent_offers(mesh, faces, v, dist, rel):
    """The updates the vertex v receives from its triangles under the map
    `dist` (caller order), per vertex they come from: a triangle offers its
    value to its giver (the smaller input of a planar value, the other end of
    an edge update), and to both inputs when their distances are within
    `rel` of each other.  The giver is found by evaluating the triangle with
    its inputs in both orders (two different answers: a tie).  Computed with
    the oracle's local update."""
    import oracle as O
    X = np.asarray(mesh.V, np.float64)
    off = {}
    for a, b in faces.wedges(v):
        u, who = O.local_update(X[v], X[a], X[b], dist[a], dist[b])
        if not np.isfinite(u):
            continue
        _, who_sw = O.local_update(X[v], X[b], X[a], dist[b], dist[a])
        g1 = a if who == 1 else b
        g2 = b if who_sw == 1 else a
        gv = {g1, g2}
        if np.isfinite(dist[a]) and np.isfinite(dist[b]) and abs(dist[a] - dist[b]) <= rel * min(dist[a], dist[b]):
            gv |= {a, b}
        for g in gv:
            off[g] = min(off.get(g, np.inf), u)
    return off


def check_labels(mesh, g_lab, g_par, o_dist, rel=1e-4):
    """The GPU's Voronoi labels and parents against the oracle's labelling of
    its own map (parents and labels from the final map, oracle.labels_from_map).
    Exact: the GPU's labels follow its parents (each vertex has its parent's
    label; sources their index in S; unreachable -1).  Every vertex whose GPU
    parent differs from the oracle's must be a tie within `rel`: under the
    oracle's map, the update the GPU's parent offers it is within `rel` of
    its best update.  Labels then differ only below such ties.  Returns
    (label mismatches, parent mismatches)."""
    import oracle as O
    S = np.asarray(mesh.S)
    n = mesh.n
    g_lab = np.asarray(g_lab)
    g_par = np.asarray(g_par)
    o_lab, o_par = O.labels_from_map(mesh.V, mesh.F, S, o_dist)
    reach = np.isfinite(o_dist)
    assert (g_lab[~reach] == -1).all() and (g_par[~reach] == -1).all()
    assert np.array_equal(g_par[S], S) and np.array_equal(g_lab[S], np.arange(S.size))
    inner = reach.copy()
    inner[S] = False
    assert (g_par[inner] >= 0).all(), "a reachable vertex without a parent"
    assert np.array_equal(g_lab[inner], g_lab[g_par[inner]]), "labels do not follow the parents"
    bad = np.nonzero(inner & (g_par != o_par))[0]
    if bad.size:
        faces = _Faces(mesh.F, n)
        for v in bad:
            off = parent_offers(mesh, faces, int(v), o_dist, rel)
            best = min(off.values())
            pg = int(g_par[v])
            assert pg in off, f"vertex {v}: GPU parent {pg} gives it no update"
            assert off[pg] <= best * (1 + rel) + 1e-30, \
                f"vertex {v}: GPU parent {pg} offers {off[pg]:.9g}, best {best:.9g}"
    return int((g_lab != o_lab).sum()), int(bad.size)
