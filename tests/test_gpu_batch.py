"""Batched PTP (many meshes / many source sets in one persistent launch).

Bars: every mesh of a batch gets bit-identical distances and labels, and the
same K, rho and U, as the single-mesh path with the same options (the batch
changes the schedule, never the result); against the FP64 oracle the same
parity bar as the single-mesh tests; results do not depend on the work
distribution (schedules, autotuning); graph replays equal the eager run.
"""
import os

import numpy as np
import pytest

import oracle as O
import paper_1810_08218_amd as P
from gpu_util import gpu_run, rel_errors, say
from paper_1810_08218_amd import inputs as I

pytestmark = pytest.mark.gpu

REL_TOL = 1e-4


def _mesh(V64, F, S, name):
    return I.Mesh(np.asarray(V64, np.float64).astype(np.float32), np.asarray(F, np.int32),
                  np.asarray(S, np.int32), name=name)


def small_batch():
    """Uneven meshes: jittered grids, tori, spheres, multi-source, one mesh
    reused with a second source set (shared rows), a tiny one."""
    rng = np.random.default_rng(77)
    out, share = [], []
    for s in (9, 23, 57, 130):
        V, F = I.jittered_grid(s, rng)
        S = rng.choice(s * s, int(rng.integers(1, 5)), replace=False)
        out.append(_mesh(V, F, S, f"jgrid{s}"))
        share.append(None)
    for k, r in ((5, 0.3), (6, 0.45), (7, 0.25)):
        V, F = I.torus(2 ** k, 2 ** (k - 1), r)
        S = rng.choice(V.shape[0], int(rng.integers(1, 5)), replace=False)
        out.append(_mesh(V, F, S, f"torus{k}"))
        share.append(None)
    out.append(I.sphere(4, seed=11, n_sources=5))
    share.append(None)
    out.append(I.noisy_icosphere(level=5, seed=12))
    share.append(None)
    # the same rows as mesh 3 (grid 130) with another source set
    g = out[3]
    out.append(I.Mesh(g.V, g.F, np.array([5, 7000, 16000], np.int32), name="jgrid130_b"))
    share.append(3)
    out.append(I.Mesh(np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32),
                      np.array([[0, 1, 2]], np.int32), np.array([1], np.int32), name="triangle"))
    share.append(None)
    return out, share


def run_batch(meshes, share, tol, labels=True, schedule=None, window=0):
    import torch
    V, F, S, descs, out_len = P.concat(meshes, share)
    dV, dF, dS = (torch.from_numpy(x).cuda() for x in (V, F, S))
    b = P.Batch(descs, tol, want_labels=labels, window=window)
    if schedule:
        b.set_schedule(**schedule)
    b.prepare(dV, dF, dS)
    dist = torch.empty(out_len, dtype=torch.float32, device="cuda")
    lab = torch.empty(out_len, dtype=torch.int32, device="cuda") if labels else None
    b.run(dist, lab)
    rc, stats, status = b.stats()
    return b, dist, lab, descs, rc, stats, status


def _slices(descs):
    return [(int(d.out_off), int(d.out_off) + int(d.n_vertices)) for d in descs]


def test_batch_equals_single_mesh_runs(cuda):
    meshes, share = small_batch()
    b, dist, lab, descs, rc, stats, status = run_batch(meshes, share, 1e-4)
    say(f"[batch] {len(meshes)} meshes rc={rc} schedule {b.get_schedule()}")
    assert rc == P.PTP_OK and all(s == P.PTP_OK for s in status)
    d = dist.cpu().numpy()
    l = lab.cpu().numpy()
    for m, (a, z), st in zip(meshes, _slices(descs), stats):
        g = gpu_run(m, 1e-4, labels=True, want_order=False)
        assert np.array_equal(d[a:z], g.dist), m.name
        assert np.array_equal(l[a:z], g.label), m.name
        assert (st["iterations"], st["n_toplesets"], st["vertex_updates"]) == \
               (g.iterations, g.rho, g.updates), m.name


def test_batch_parity_against_oracle(cuda):
    meshes, share = small_batch()
    b, dist, lab, descs, rc, stats, status = run_batch(meshes, share, 1e-4)
    d = dist.cpu().numpy()
    for m, (a, z), st in zip(meshes, _slices(descs), stats):
        o = O.run(m.V, m.F, m.S, 1e-4)
        mx, mean = rel_errors(d[a:z], o.dist, m.S)
        say(f"  {m.name}: K {st['iterations']}/{o.iterations} U {st['vertex_updates']}/{o.updates} "
            f"max rel {mx:.2e}")
        assert (st["iterations"], st["vertex_updates"]) == (o.iterations, o.updates), m.name
        assert mx <= REL_TOL, m.name
        assert (d[a:z][m.S] == 0).all()


def test_results_independent_of_schedule_and_autotune(cuda):
    import torch
    meshes, share = small_batch()
    ref = run_batch(meshes, share, 1e-4)
    rd, rl = ref[1].cpu().numpy(), ref[2].cpu().numpy()
    for sch in ({"workgroups": 8, "small_limit": 1, "large_limit": 1 << 30, "medium_group": 1},
                {"workgroups": 300, "small_limit": 1000, "large_limit": 5000, "medium_group": 3,
                 "large_group": 7},
                {"workgroups": 2, "small_limit": 1, "large_limit": 100, "large_group": 2}):
        b, dist, lab, descs, rc, stats, status = run_batch(meshes, share, 1e-4, schedule=sch)
        assert rc == P.PTP_OK
        assert np.array_equal(dist.cpu().numpy(), rd) and np.array_equal(lab.cpu().numpy(), rl), sch
    b = ref[0]
    cands = [{"workgroups": 64}, {"workgroups": 512, "small_limit": 4096, "large_limit": 65536},
             {"workgroups": 1024, "medium_group": 2, "large_group": 8}]
    dist = torch.empty_like(ref[1])
    lab = torch.empty_like(ref[2])
    best, ms = b.autotune(cands, dist, lab)
    say(f"  autotune ms {ms} best {best}")
    assert 0 <= best < len(cands) and all(t > 0 for t in ms)
    b.run(dist, lab)
    assert b.stats()[0] == P.PTP_OK
    assert np.array_equal(dist.cpu().numpy(), rd) and np.array_equal(lab.cpu().numpy(), rl)


def test_batch_bfs_paths_agree(cuda):
    """Meshes split between the one-workgroup LDS BFS and the grid BFS (by a
    vertex limit) give the results of either path alone."""
    import torch
    meshes, share = small_batch()
    ref = run_batch(meshes, share, 1e-4)
    rd, rl = ref[1].cpu().numpy(), ref[2].cpu().numpy()
    V, F, S, descs, out_len = P.concat(meshes, share)
    dV, dF, dS = (torch.from_numpy(x).cuda() for x in (V, F, S))
    for lim in (-1, 1000, 5000):
        b = P.Batch(descs, 1e-4, want_labels=True, lds_bfs_max=lim)
        b.prepare(dV, dF, dS)
        dist = torch.empty(out_len, dtype=torch.float32, device="cuda")
        lab = torch.empty(out_len, dtype=torch.int32, device="cuda")
        b.run(dist, lab)
        rc, stats, status = b.stats()
        assert rc == P.PTP_OK, lim
        assert np.array_equal(dist.cpu().numpy(), rd) and np.array_equal(lab.cpu().numpy(), rl), lim


def test_set_window_equals_create_time_window_and_tuner(cuda):
    """A window set at run time gives exactly the results of a batch created
    with it; the window tuner keeps its choice within 1e-4 of the unbounded
    run."""
    import torch
    from paper_1810_08218_amd import autotune
    meshes, share = small_batch()
    V, F, S, descs, out_len = P.concat(meshes, share)
    dV, dF, dS = (torch.from_numpy(x).cuda() for x in (V, F, S))
    ref = run_batch(meshes, share, 1e-4, labels=False, window=5)
    b = P.Batch(descs, 1e-4)
    b.prepare(dV, dF, dS)
    dist = torch.empty(out_len, dtype=torch.float32, device="cuda")
    b.set_window(5)
    b.run(dist)
    assert b.stats()[0] == P.PTP_OK
    assert np.array_equal(dist.cpu().numpy(), ref[1].cpu().numpy())
    with pytest.raises(P.PTPError):
        b.set_window(-1)
    res = autotune.tune_window(b, dist, candidates=(0, 32, 8, 4, 2))
    say(f"  window tuner: {res}")
    assert res["max_rel_diff"] <= 1e-4
    b.run(dist)
    unb = run_batch(meshes, share, 1e-4, labels=False)[1].cpu().numpy()
    d = dist.cpu().numpy()
    fin = np.isfinite(unb) & (unb > 0)
    assert (np.abs(d[fin] - unb[fin]) / unb[fin]).max() <= 1e-4


def test_invalid_mesh_in_batch(cuda):
    import torch
    meshes, share = small_batch()
    V, F, S, descs, out_len = P.concat(meshes, share)
    F = F.copy()
    F[int(descs[2].f_off) + 5, 1] = 10 ** 6          # out of range for mesh 2
    dV, dF, dS = (torch.from_numpy(x).cuda() for x in (V, F, S))
    b = P.Batch(descs, 1e-4)
    with pytest.raises(P.PTPError) as e:
        b.prepare(dV, dF, dS)
    assert e.value.status == P.PTP_EINVAL
    rc, stats, status = b.stats()
    assert status[2] == P.PTP_EINVAL and sum(s != P.PTP_OK for s in status) == 1


def _many_small_meshes(count=300):
    """More meshes than the device has CUs, so the reorder into topleset
    order runs inside the one-workgroup BFS launch: the small batch, the
    irregular-fan mesh (fans longer than the fixed-size record, a non-manifold
    vertex, a duplicated face), a mesh with a part no source reaches, and
    small jittered grids and tori with 1-3 sources up to `count`."""
    from test_gpu_parity import _irregular_fans_mesh
    meshes, share = small_batch()
    meshes.append(_irregular_fans_mesh())
    share.append(None)
    g = I.flat_grid(6)
    V = np.concatenate([g.V, np.array([[5, 5, 0], [6, 5, 0], [5, 6, 0]], np.float32)])
    F = np.concatenate([g.F, np.array([[36, 37, 38]], np.int32)])
    meshes.append(I.Mesh(V, F, np.array([0], np.int32), name="grid6_island"))
    share.append(None)
    rng = np.random.default_rng(91)
    while len(meshes) < count:
        if rng.random() < 0.7:
            s = int(rng.integers(5, 41))
            V, F = I.jittered_grid(s, rng)
            name = f"jgrid{s}"
        else:
            k = int(rng.integers(3, 6))
            V, F = I.torus(2 ** k, 2 ** (k - 1), 0.3)
            name = f"torus{k}"
        S = rng.choice(V.shape[0], int(rng.integers(1, 4)), replace=False)
        meshes.append(_mesh(V, F, S, name))
        share.append(None)
    return meshes, share


def test_reorder_inside_bfs_launch(cuda):
    """A batch of 300 meshes (reorder inside the BFS launch) equals the
    single-mesh plans bit for bit, distances, labels, K, rho and U; the
    unreachable vertices stay at infinity with label -1."""
    meshes, share = _many_small_meshes()
    b, dist, lab, descs, rc, stats, status = run_batch(meshes, share, 1e-4)
    say(f"[batch] {len(meshes)} meshes rc={rc}")
    assert rc == P.PTP_OK and all(s == P.PTP_OK for s in status)
    d = dist.cpu().numpy()
    l = lab.cpu().numpy()
    for m, (a, z), st in zip(meshes, _slices(descs), stats):
        g = gpu_run(m, 1e-4, labels=True, want_order=False)
        assert np.array_equal(d[a:z], g.dist), m.name
        assert np.array_equal(l[a:z], g.label), m.name
        assert (st["iterations"], st["n_toplesets"], st["vertex_updates"]) == \
               (g.iterations, g.rho, g.updates), m.name
    island = [i for i, m in enumerate(meshes) if m.name == "grid6_island"][0]
    a, z = _slices(descs)[island]
    assert np.isinf(d[a:z][36:]).all() and (l[a:z][36:] == -1).all()


def test_reorder_inside_bfs_launch_duplicate_source(cuda):
    """A duplicate source in one mesh of such a batch fails the prepare for
    that mesh only (its BFS publishes nothing, the other workgroups still
    finish); the batch prepared again with valid sources gives the results
    of a fresh batch."""
    import torch
    meshes, share = _many_small_meshes()
    V, F, S, descs, out_len = P.concat(meshes, share)
    bad = 20
    S2 = S.copy()
    s0 = int(descs[bad].s_off)
    assert int(descs[bad].n_sources) >= 1
    if int(descs[bad].n_sources) == 1:
        pytest.skip("mesh 20 has one source")
    S2[s0 + 1] = S2[s0]
    dV, dF = (torch.from_numpy(x).cuda() for x in (V, F))
    b = P.Batch(descs, 1e-4, want_labels=True)
    with pytest.raises(P.PTPError) as e:
        b.prepare(dV, dF, torch.from_numpy(S2).cuda())
    assert e.value.status == P.PTP_EINVAL
    rc, stats, status = b.stats()
    assert status[bad] == P.PTP_EINVAL and sum(s != P.PTP_OK for s in status) == 1
    b.prepare(dV, dF, torch.from_numpy(S).cuda())
    dist = torch.empty(out_len, dtype=torch.float32, device="cuda")
    lab = torch.empty(out_len, dtype=torch.int32, device="cuda")
    b.run(dist, lab)
    assert b.stats()[0] == P.PTP_OK
    ref = run_batch(meshes, share, 1e-4)
    assert np.array_equal(dist.cpu().numpy(), ref[1].cpu().numpy())
    assert np.array_equal(lab.cpu().numpy(), ref[2].cpu().numpy())


def test_graph_replay_matches_eager(cuda):
    """The run enqueues kernel launches only; captured in a graph and replayed
    (with eager work and synchronisations between replays) it gives the eager
    result every time."""
    import torch
    meshes, share = small_batch()
    b, dist, lab, descs, rc, stats, status = run_batch(meshes, share, 1e-4)
    ref_d, ref_l = dist.cpu().numpy(), lab.cpu().numpy()
    d2 = torch.full_like(dist, -1.0)
    l2 = torch.full_like(lab, -7)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            b.run(d2, l2, stream=s)
    for rep in range(3):
        d2.fill_(-1.0)
        l2.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(d2.cpu().numpy(), ref_d), rep
        assert np.array_equal(l2.cpu().numpy(), ref_l), rep
        _ = (torch.ones(1000, device="cuda") * 2).sum().item()   # eager work between replays


BATCH_SAMPLES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                             "batch_largest_oracle_samples.npz")


def test_full_uneven_batch_512(cuda):
    """The 512-mesh workload (jittered grids of side 32..1024 and tori of
    2^k x 2^(k-1), k = 5..10, 1-4 sources each; 71M vertices) in one launch
    with the schedule the benchmark times: every mesh converges and equals its
    own single-mesh plan bit for bit (distances, K, U); the largest grid and
    the largest torus match stored oracle samples (written by
    tests/golden/make_oracle_samples.py, which calls only the oracle) with the
    oracle's schedule; the 12 smallest meshes match the oracle in full."""
    import torch
    from paper_1810_08218_amd import autotune
    meshes = I.batch_meshes(512)
    V, F, S, descs, out_len = P.concat(meshes)
    say(f"[batch512] n={V.shape[0]} f={F.shape[0]} m={S.shape[0]}")
    dV, dF, dS = (torch.from_numpy(x).cuda() for x in (V, F, S))
    del V, F
    b = P.Batch(descs, 1e-4)
    b.set_schedule(**autotune.BATCH512_SCHEDULE)
    b.prepare(dV, dF, dS)
    dist = torch.empty(out_len, dtype=torch.float32, device="cuda")
    b.run(dist)
    rc, stats, status = b.stats()
    say(f"  rc {rc} K max {max(s['iterations'] for s in stats)} rho max "
        f"{max(s['n_toplesets'] for s in stats)} U {sum(s['vertex_updates'] for s in stats)} "
        f"run {stats[0]['ms_run']:.1f} ms")
    assert rc == P.PTP_OK and all(s == P.PTP_OK for s in status)
    d = dist.cpu().numpy()
    assert np.isfinite(d).all()
    sl = _slices(descs)
    for m, (a, z) in zip(meshes, sl):
        assert (d[a:z][m.S] == 0).all()
    ref = np.load(BATCH_SAMPLES)
    for t in (int(x) for x in ref["ts"]):
        a, z = sl[t]
        idx = ref[f"t{t}_idx"]
        mx, mean = rel_errors(d[a:z][idx], ref[f"t{t}_dist"], np.nonzero(np.isin(idx, meshes[t].S))[0])
        say(f"  {meshes[t].name} (t={t}, n={meshes[t].n}): K {stats[t]['iterations']}/"
            f"{int(ref[f't{t}_iterations'])} U {stats[t]['vertex_updates']}/{int(ref[f't{t}_updates'])} "
            f"sampled max rel {mx:.2e} mean {mean:.2e}")
        assert stats[t]["n_toplesets"] == int(ref[f"t{t}_rho"])
        assert stats[t]["iterations"] == int(ref[f"t{t}_iterations"])
        assert stats[t]["vertex_updates"] == int(ref[f"t{t}_updates"])
        assert mx <= REL_TOL
    order = np.argsort([m.n for m in meshes])[:12]
    for t in order:
        m = meshes[t]
        a, z = sl[t]
        o = O.run(m.V, m.F, m.S, 1e-4)
        mx, _ = rel_errors(d[a:z], o.dist, m.S)
        assert (stats[t]["iterations"], stats[t]["vertex_updates"]) == (o.iterations, o.updates)
        assert mx <= REL_TOL, m.name
    # every mesh against its own plan: one plan per mesh, the batch's rows
    differ = []
    for t, m in enumerate(meshes):
        a, z = sl[t]
        plan = P.Plan(m.n, m.f, m.m, 1e-4)
        d1 = torch.empty(m.n, dtype=torch.float32, device="cuda")
        vo, fo, so = int(descs[t].v_off), int(descs[t].f_off), int(descs[t].s_off)
        plan.prepare(dV[vo:vo + m.n], dF[fo:fo + m.f], dS[so:so + m.m])
        plan.run(d1)
        st = plan.stats()
        same = np.array_equal(d1.cpu().numpy(), d[a:z])
        same &= (st["iterations"], st["vertex_updates"]) == (stats[t]["iterations"], stats[t]["vertex_updates"])
        if not same:
            differ.append(t)
    say(f"  meshes differing from their single plan: {differ}")
    assert differ == []
