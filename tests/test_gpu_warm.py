"""Learned warm start on the GPU: features, network forward / backward / Adam
against the FP64 oracle, the certified warm run against the oracle's warm
run and against the plain run, batches and graph capture.

Bars: network outputs within 2e-2 relative of the FP64 oracle (bf16
weights and layer-2 activations, float32 accumulation), gradients with
cosine > 0.999 and max deviation < 2e-2 of the largest component;
features at float32 accuracy (hop exact); warm-run distances within 1e-4
relative of the oracle and of the plain GPU run; certified starts never
below the fixed point.
"""
import numpy as np
import pytest

import oracle as O
import paper_1810_08218_amd as P
from gpu_util import gpu_run, rel_errors, say, to_dev
from oracle import warm as W
from paper_1810_08218_amd import inputs as I
from paper_1810_08218_amd import ptp as B

pytestmark = pytest.mark.gpu

REL_TOL = 1e-4


def _params(seed):
    """Seeded parameters with larger last-layer weights so the outputs vary."""
    p = W.init_params(seed).astype(np.float64)
    rng = np.random.default_rng(seed + 100)
    p[4416:4480] *= 4.0
    p[256:4352] += rng.normal(0, 0.05, 4096)
    return p.astype(np.float32)


def _rows(n, seed):
    rng = np.random.default_rng(seed)
    X = np.stack([rng.uniform(0, 4, n), rng.integers(0, 300, n) / 64.0, rng.normal(0, 0.1, n)], 1)
    s = rng.uniform(0.005, 0.05, n)
    d = 64 * s * X[:, 0] * rng.uniform(1.0, 1.4, n) + 0.5 * s
    return X.astype(np.float32), s.astype(np.float32), d.astype(np.float32)


def _dev(*arrays):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrays]


def _two_component_mesh():
    """A jittered grid plus a detached triangle strip: the strip is unreachable."""
    V, F = I.jittered_grid(40, np.random.default_rng(21))
    V2 = np.array([[2, 0, 0], [3, 0, 0], [2, 1, 0], [3, 1, 0]], np.float32)
    F2 = np.array([[0, 1, 2], [1, 3, 2]], np.int32) + V.shape[0]
    return I.Mesh(np.concatenate([V, V2]).astype(np.float32), np.concatenate([F, F2]).astype(np.int32),
                  np.array([5, 901], np.int32), name="grid40+strip")


def _meshes():
    rng = np.random.default_rng(31)
    V, F = I.torus(64, 32, 0.35)
    return [I.Mesh(*I.jittered_grid(57, rng), np.array([100, 2000], np.int32), name="jgrid57"),
            I.sphere(4, seed=3, n_sources=6), I.noisy_icosphere(level=4, seed=8),
            I.Mesh(V, F, np.array([17], np.int32), name="torus64"), _two_component_mesh()]


# -------------------------------------------------------------- network ---

@pytest.mark.parametrize("n", [1, 31, 1000, 4099])
def test_mlp_forward_matches_oracle(cuda, n):
    import torch
    params = _params(7)
    X, s, _ = _rows(n, n)
    ref, _ = W.forward(params, X, s)
    dP, dX, dS = _dev(params, X, s)
    out = P.ptp.mlp_apply(dP, dX, dS).cpu().numpy()
    rel = np.abs(out - ref) / np.abs(ref)
    say(f"[mlp fwd] n={n} max rel {rel.max():.2e} mean {rel.mean():.2e}")
    assert rel.max() < 2e-2 and rel.mean() < 5e-3
    assert B.load().ptp_mlp_apply(B._ptr(dP), B._ptr(dX), B._ptr(dS), 0, None,
                                  B._stream(None)) == P.PTP_OK
    torch.cuda.synchronize()


@pytest.mark.parametrize("n", [33, 777, 20000])
def test_mlp_gradient_matches_oracle(cuda, n):
    params = _params(9)
    X, s, d = _rows(n, 50 + n)
    L, g = W.loss_and_grad(params, X, s, d)
    dP, dX, dS, dD = _dev(params, X, s, d)
    tr = P.ptp.MlpTrainer(dP)
    grad, loss = tr.grad_loss(dX, dS, dD)
    gg = grad.cpu().numpy().astype(np.float64)
    cos = float(gg @ g / (np.linalg.norm(gg) * np.linalg.norm(g)))
    dev = float(np.abs(gg - g).max() / np.abs(g).max())
    lrel = abs(float(loss.item()) - L) / L
    say(f"[mlp grad] n={n} cos {cos:.6f} max dev {dev:.2e} loss {loss.item():.5f}/{L:.5f}")
    assert cos > 0.999 and dev < 2e-2 and lrel < 1e-2
    for a, b, name in ((0, 192, "W1"), (192, 256, "b1"), (256, 4352, "W2"), (4352, 4416, "b2"),
                       (4416, 4480, "W3"), (4480, 4481, "b3")):
        e = np.linalg.norm(gg[a:b] - g[a:b]) / np.linalg.norm(g[a:b])
        assert e < 3e-2, name
    grad2, _ = tr.grad_loss(dX, dS, dD)                  # fixed reduction order
    assert np.array_equal(grad2.cpu().numpy(), gg.astype(np.float32))


def test_adam_matches_oracle(cuda):
    import torch
    params = _params(4).astype(np.float64)
    dP, = _dev(params.astype(np.float32))
    tr = P.ptp.MlpTrainer(dP, lr=1e-3)
    rng = np.random.default_rng(12)
    p, m, v = params.astype(np.float32).astype(np.float64), np.zeros(W.N_PARAMS), np.zeros(W.N_PARAMS)
    for t in range(1, 6):
        g = rng.normal(0, 1e-2, W.N_PARAMS).astype(np.float32)
        tr.grad.copy_(torch.from_numpy(g))
        tr.adam()
        p, m, v = W.adam_step(p, g.astype(np.float64), m, v, t, lr=1e-3)
    got = dP.cpu().numpy().astype(np.float64)
    assert np.abs(got - p).max() < 1e-6 + 1e-6 * np.abs(p).max()


# ------------------------------------------------------------- features ---

@pytest.mark.parametrize("k", range(5))
def test_features_match_oracle(cuda, k):
    m = _meshes()[k]
    V, F, S = to_dev(m)
    plan = P.Plan(m.n, m.f, m.m, 1e-4)
    plan.prepare(V, F, S)
    X, scale = plan.warm_features()
    X, scale = X.cpu().numpy().astype(np.float64), scale.cpu().numpy().astype(np.float64)
    level, _, _, _ = O.toplesets(m.V, m.F, m.S)
    Xr, sr = W.features(m.V, m.F, m.S, level)
    reach = level >= 0
    say(f"[features] {m.name} n={m.n} unreachable {int((~reach).sum())}")
    assert np.array_equal(scale < 0, ~reach)
    assert np.allclose(scale[reach], sr[reach], rtol=2e-6, atol=0)
    assert np.allclose(X[reach, 0], Xr[reach, 0], rtol=2e-5, atol=1e-7)
    assert np.array_equal(X[reach, 1], Xr[reach, 1])
    c = np.abs(X[reach, 2] - Xr[reach, 2])
    say(f"  curvature max abs dev {c.max():.2e} (scale {np.abs(Xr[reach, 2]).max():.2e})")
    assert (c <= 1e-3 * np.abs(Xr[reach, 2]) + 2e-4).all()
    assert (X[~reach] == 0).all()


def test_predict_matches_oracle(cuda):
    import torch
    params = _params(5)
    for m in _meshes()[:3] + [_two_component_mesh()]:
        V, F, S = to_dev(m)
        plan = P.Plan(m.n, m.f, m.m, 1e-4)
        plan.prepare(V, F, S)
        dP, = _dev(params)
        up = torch.empty(m.n, dtype=torch.float32, device="cuda")
        plan.warm_predict(dP, up, inflate=1.05)
        got = up.cpu().numpy().astype(np.float64)
        level, _, _, _ = O.toplesets(m.V, m.F, m.S)
        ref = W.predict(params, m.V, m.F, m.S, level, inflate=1.05)
        fin = np.isfinite(ref) & (ref > 0)
        rel = np.abs(got[fin] - ref[fin]) / ref[fin]
        say(f"[predict] {m.name} max rel {rel.max():.2e}")
        assert rel.max() < 2e-2
        assert (got[m.S] == 0).all() and np.array_equal(np.isinf(got), np.isinf(ref))


# -------------------------------------------------------- certified run ---

def _plan(m, tol, **kw):
    V, F, S = to_dev(m)
    plan = P.Plan(m.n, m.f, m.m, tol, **kw)
    plan.prepare(V, F, S)
    return plan


def _run_warm(m, tol, w, **kw):
    import torch
    plan = _plan(m, tol, **kw)
    up = torch.from_numpy(np.ascontiguousarray(w, np.float32)).cuda()
    dist = torch.empty(m.n, dtype=torch.float32, device="cuda")
    plan.run_warm(up, dist)
    st = plan.stats()
    return dist.cpu().numpy(), st


def test_warm_from_no_bound_equals_plain(cuda):
    for m in _meshes()[:3]:
        g = gpu_run(m, 1e-4, want_order=False)
        for fill in (np.inf, -1.0, np.nan):
            d, st = _run_warm(m, 1e-4, np.full(m.n, fill))
            assert np.array_equal(d, g.dist), (m.name, fill)
            assert (st["iterations"], st["vertex_updates"], st["certify_rejected"]) == \
                   (g.iterations, g.updates, 0)


@pytest.mark.parametrize("k", range(5))
def test_warm_run_matches_oracle_and_plain(cuda, k):
    m = _meshes()[k]
    rng = np.random.default_rng(40 + k)
    dstar, _, _ = O.fixed_point(m.V, m.F, m.S)
    level, _, _, _ = O.toplesets(m.V, m.F, m.S)
    starts = {"scaled": 1.05 * dstar,
              "network": W.predict(_params(6), m.V, m.F, m.S, level),
              "noisy": dstar * rng.uniform(0.9, 1.2, m.n),
              "low": 0.7 * dstar}
    g = gpu_run(m, 1e-4, want_order=False)
    po = O.run(m.V, m.F, m.S, 1e-4)
    for name, w in starts.items():
        w = np.where(np.isfinite(w), w, np.inf).astype(np.float32)
        d, st = _run_warm(m, 1e-4, w)
        o = O.run_warm(m.V, m.F, m.S, 1e-4, w.astype(np.float64))
        e_or, _ = rel_errors(d, o.dist, m.S)
        e_pl, _ = rel_errors(d, g.dist, m.S)
        e_op, _ = rel_errors(d, po.dist, m.S)
        say(f"[warm] {m.name} {name}: K {st['iterations']}/{o.iterations} (plain {g.iterations}) "
            f"U {st['vertex_updates']}/{o.updates} (plain {g.updates}) rejected "
            f"{st['certify_rejected']}/{o.rejected} rounds {st['certify_rounds']} "
            f"err vs oracle warm {e_or:.1e} plain {e_pl:.1e} oracle plain {e_op:.1e}")
        assert st["status"] == P.PTP_OK
        assert max(e_or, e_pl, e_op) <= REL_TOL, name
        assert (d[m.S] == 0).all()
        assert np.array_equal(np.isinf(d), np.isinf(g.dist))
        if name == "scaled":
            assert st["certify_rejected"] == 0 and o.rejected == 0


@pytest.mark.parametrize("k", [0, 1, 2])
def test_certified_start_never_below_fixed_point(cuda, k):
    """With a cap of one iteration the output is the certified start except
    on V_1: it never lies below the fixed point."""
    m = _meshes()[k]
    rng = np.random.default_rng(70 + k)
    dstar, _, _ = O.fixed_point(m.V, m.F, m.S)
    for w in (0.7 * dstar, dstar * rng.uniform(0.8, 1.2, m.n), rng.uniform(0, 2, m.n)):
        d, st = _run_warm(m, 1e-4, w.astype(np.float32), max_iters=1)
        fin = np.isfinite(dstar)
        assert (d[fin] >= dstar[fin] * (1 - 2e-6) - 1e-7).all()
        assert st["certify_rounds"] >= 1


def test_warm_labels_unsupported_and_bad_args(cuda):
    import torch
    m = _meshes()[0]
    plan = _plan(m, 1e-4, want_labels=True)
    up = torch.full((m.n,), float("inf"), device="cuda")
    dist = torch.empty(m.n, device="cuda")
    with pytest.raises(P.PTPError) as e:
        plan.run_warm(up, dist)
    assert e.value.status == P.PTP_EUNSUPPORTED
    plan = _plan(m, 1e-4)
    dP, = _dev(_params(1))
    with pytest.raises(P.PTPError) as e:
        plan.warm_predict(dP, up, inflate=0.9)
    assert e.value.status == P.PTP_EINVAL
    lib = B.load()
    X, s, d = _dev(*_rows(10, 1))
    small = torch.empty(16, dtype=torch.float32, device="cuda")
    g = torch.empty(W.N_PARAMS, device="cuda")
    rc = lib.ptp_mlp_grad(B._ptr(dP), B._ptr(X), B._ptr(s), B._ptr(d), 10, B._ptr(small), 64,
                          B._ptr(g), None, B._stream(None))
    assert rc == P.PTP_ENOMEM


# ---------------------------------------------------------------- batch ---

def test_warm_batch_equals_single_and_graph_replay(cuda):
    import torch
    meshes = _meshes()
    params = _params(3)
    dP, = _dev(params)
    V, F, S, descs, out_len = P.concat(meshes)
    dV, dF, dS = (torch.from_numpy(x).cuda() for x in (V, F, S))
    b = P.Batch(descs, 1e-4)
    b.prepare(dV, dF, dS)
    up = torch.empty(out_len, device="cuda")
    dist = torch.empty(out_len, device="cuda")
    b.warm_predict(dP, up)
    b.run_warm(up, dist)
    rc, stats, status = b.stats()
    assert rc == P.PTP_OK
    ref_up, ref_d = up.cpu().numpy(), dist.cpu().numpy()
    for mm, dsc, st in zip(meshes, descs, stats):
        a, z = int(dsc.out_off), int(dsc.out_off) + mm.n
        plan = _plan(mm, 1e-4)
        u1 = torch.empty(mm.n, device="cuda")
        d1 = torch.empty(mm.n, device="cuda")
        plan.warm_predict(dP, u1)
        plan.run_warm(u1, d1)
        s1 = plan.stats()
        assert np.array_equal(u1.cpu().numpy(), ref_up[a:z]), mm.name
        assert np.array_equal(d1.cpu().numpy(), ref_d[a:z]), mm.name
        assert (s1["iterations"], s1["vertex_updates"], s1["certify_rejected"]) == \
               (st["iterations"], st["vertex_updates"], st["certify_rejected"])
    # predict + certified run captured in one graph, in place (upper = dist)
    d2 = torch.full_like(dist, -1.0)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    gph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(gph, stream=s):
            b.warm_predict(dP, d2, stream=s)
            b.run_warm(d2, d2, stream=s)
    for rep in range(3):
        d2.fill_(-1.0)
        torch.cuda.synchronize()
        gph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(d2.cpu().numpy(), ref_d), rep
        _ = (torch.ones(1000, device="cuda") * 2).sum().item()


def test_training_loss_falls_and_resume_is_exact(cuda, tmp_path):
    """The training loop on the library's kernels: 200 Adam steps on a fixed
    seed lower the loss on a fixed evaluation set; a run checkpointed at step
    100 (parameters, Adam moments, step, minibatch generator) and resumed
    ends bit-identical to the uninterrupted run."""
    import torch
    from paper_1810_08218_amd import train_warmstart as TW
    meshes = [I.training_mesh(t, seed=5) for t in range(6)]
    X, S, D = TW.dataset(meshes, log=lambda *a: None)
    ev0 = TW.evaluate(torch.from_numpy(TW.init_params(3)).cuda(), X, S, D)

    def fresh():
        p = torch.from_numpy(TW.init_params(3)).cuda()
        tr = P.ptp.MlpTrainer(p)
        g = torch.Generator(device="cuda")
        g.manual_seed(11)
        return tr, g

    tr, g = fresh()
    TW.train_steps(tr, X, S, D, g, 1, 200, 4096)
    ev = TW.evaluate(tr.params, X, S, D)
    say(f"  loss {ev0['loss']:.4f} -> {ev['loss']:.4f}; mean rel {ev0['mean_rel']:.3f} -> {ev['mean_rel']:.3f}")
    assert ev["loss"] < 0.5 * ev0["loss"]
    tr2, g2 = fresh()
    ck = str(tmp_path / "ckpt.npz")
    TW.train_steps(tr2, X, S, D, g2, 1, 100, 4096, checkpoint=ck, checkpoint_every=100)
    tr3, g3 = fresh()
    first = TW.load_checkpoint(ck, tr3, g3) + 1
    assert first == 101 and tr3.t == 100
    TW.train_steps(tr3, X, S, D, g3, first, 200, 4096)
    assert torch.equal(tr3.params, tr.params) and torch.equal(tr3.m, tr.m) and torch.equal(tr3.v, tr.v)
