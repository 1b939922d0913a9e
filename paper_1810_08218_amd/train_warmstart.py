"""Train the warm-start network on distances the library itself computes.

    python -m paper_1810_08218_amd.train_warmstart [--meshes 2000] [--steps 6000]
        [--out paper_1810_08218_amd/weights/warmstart_mlp.npz]

Data: ``inputs.training_mesh(t)`` for t < meshes (seed 5), solved by the
batched PTP at tol 1e-4 (targets) and passed through the feature kernels
(inputs); sources and unreachable vertices are left out.  Training: Adam
(lr 1e-3, betas 0.9 / 0.999) on minibatches of 65,536 rows drawn with a
seeded generator, loss = mean squared relative error (the loss of
``ptp_mlp_grad``), forward / backward / Adam in the library's kernels.  The
held-out meshes (seed 6) report the loss and the relative error of the
prediction at the end.  Everything runs on the GPU through the C ABI; the
only host work is mesh generation and bookkeeping.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import inputs as I
from . import ptp as B

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "weights", "warmstart_mlp.npz")
H = 64


def init_params(seed: int = 0) -> np.ndarray:
    """Seeded start: every weight and bias uniform in +-1/sqrt(fan_in)."""
    rng = np.random.default_rng(seed)
    parts = []
    for fi, fo in ((3, H), (H, H), (H, 1)):
        k = 1.0 / np.sqrt(fi)
        parts.append(rng.uniform(-k, k, fi * fo))
        parts.append(rng.uniform(-k, k, fo))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == B.MLP_PARAMS
    return p


def dataset(meshes, tol=1e-4, chunk=48, log=print):
    """(X [R, 3], scale [R], target [R]) device tensors over the meshes'
    reachable non-source vertices, solved in batches of `chunk` meshes."""
    import torch
    Xs, Ss, Ds = [], [], []
    for c0 in range(0, len(meshes), chunk):
        part = meshes[c0:c0 + chunk]
        V, F, S, descs, out_len = B.concat(part)
        dV, dF, dS = (torch.from_numpy(a).cuda() for a in (V, F, S))
        b = B.Batch(descs, tol)
        b.prepare(dV, dF, dS)
        dist = torch.empty(out_len, dtype=torch.float32, device="cuda")
        b.run(dist)
        rc, _, status = b.stats()
        if rc != B.PTP_OK:
            raise RuntimeError(f"training batch {c0}: status {status}")
        X, scale = b.warm_features()
        keep = (scale > 0) & (dist > 0) & torch.isfinite(dist)
        Xs.append(X[keep])
        Ss.append(scale[keep])
        Ds.append(dist[keep])
        log(f"  data meshes {c0}..{c0 + len(part) - 1}: {int(keep.sum())} rows")
    return torch.cat(Xs), torch.cat(Ss), torch.cat(Ds)


def evaluate(params, X, S, D, rows=1 << 20):
    """Mean and 95th-percentile relative error of the prediction, and the loss."""
    import torch
    n = min(rows, X.shape[0])
    pred = B.mlp_apply(params, X[:n].contiguous(), S[:n].contiguous())
    rel = ((pred - D[:n]) / D[:n]).abs()
    e = (pred - D[:n]) / torch.maximum(D[:n], S[:n])
    return {"mean_rel": float(rel.mean()), "p95_rel": float(rel.quantile(0.95)),
            "loss": float((e * e).mean())}


def train(meshes=2000, steps=6000, batch=65536, lr=1e-3, seed=0, out=DEFAULT_OUT, log=print):
    import torch
    t0 = time.time()
    log(f"[train] generating {meshes} training meshes")
    train_m = [I.training_mesh(t, seed=5) for t in range(meshes)]
    hold_m = [I.training_mesh(t, seed=6) for t in range(max(30, meshes // 20))]
    log(f"[train] {sum(m.n for m in train_m)} training vertices ({time.time() - t0:.1f} s)")
    X, S, D = dataset(train_m, log=log)
    Xh, Sh, Dh = dataset(hold_m, log=log)
    log(f"[train] rows {X.shape[0]} train, {Xh.shape[0]} held out ({time.time() - t0:.1f} s)")
    params = torch.from_numpy(init_params(seed)).cuda()
    tr = B.MlpTrainer(params, lr=lr)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    curve = []
    for step in range(1, steps + 1):
        idx = torch.randint(0, X.shape[0], (batch,), device="cuda", generator=gen)
        tr.step(X[idx].contiguous(), S[idx].contiguous(), D[idx].contiguous())
        if step % 500 == 0 or step == 1:
            loss = float(tr.loss.item())
            curve.append((step, loss))
            log(f"[train] step {step} loss {loss:.5f} ({time.time() - t0:.1f} s)")
    torch.cuda.synchronize()
    ev_train = evaluate(params, X, S, D)
    ev_hold = evaluate(params, Xh, Sh, Dh)
    log(f"[train] train {ev_train}  held out {ev_hold}")
    meta = {"meshes": meshes, "steps": steps, "batch": batch, "lr": lr, "seed": seed,
            "rows": int(X.shape[0]), "curve": curve, "train": ev_train, "held_out": ev_hold,
            "seconds": time.time() - t0}
    os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
    np.savez(out, params=params.cpu().numpy(), meta=np.array(json.dumps(meta)))
    log(f"[train] wrote {out}")
    return params, meta


def load_params(path: str = DEFAULT_OUT, device="cuda"):
    """The trained parameter vector as a float32 device tensor."""
    import torch
    with np.load(path, allow_pickle=False) as z:
        p = np.asarray(z["params"], np.float32)
    if p.size != B.MLP_PARAMS:
        raise ValueError(f"{path}: {p.size} parameters, expected {B.MLP_PARAMS}")
    return torch.from_numpy(p).to(device)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--meshes", type=int, default=2000)
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--batch", type=int, default=65536)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=DEFAULT_OUT)
    a = ap.parse_args(argv)

    def log(*x):
        print(*x, flush=True)

    train(a.meshes, a.steps, a.batch, a.lr, a.seed, a.out, log)
    return 0


if __name__ == "__main__":
    sys.exit(main())
