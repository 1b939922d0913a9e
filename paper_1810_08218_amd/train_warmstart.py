"""Train the warm-start network on distances the library itself computes.

    python -m paper_1810_08218_amd.train_warmstart [--meshes 2000] [--steps 6000]
        [--out paper_1810_08218_amd/weights/warmstart_mlp.npz]
        [--checkpoint ckpt.npz --checkpoint-every 1000] [--resume ckpt.npz]

Data: ``inputs.training_mesh(t)`` for t < meshes (seed 5), solved by the
batched PTP at tol 1e-4 (targets) and passed through the feature kernels
(inputs); sources and unreachable vertices are left out.  Training: Adam
(lr 1e-3, betas 0.9 / 0.999) on minibatches of 65,536 rows drawn with a
seeded generator, loss = mean squared relative error (the loss of
``ptp_mlp_grad``), forward / backward / Adam in the library's kernels.  The
held-out meshes (seed 6) report the loss and the relative error of the
prediction at the end.  A checkpoint holds the parameters, both Adam moments,
the step count and the state of the minibatch generator, so a run resumed
from it continues exactly as the uninterrupted run would.  Everything runs on the GPU through the C ABI; the
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


def save_checkpoint(path, trainer, gen, step, extra=None):
    """Parameters, Adam moments and step, minibatch generator state."""
    rec = {"params": trainer.params.cpu().numpy(), "adam_m": trainer.m.cpu().numpy(),
           "adam_v": trainer.v.cpu().numpy(), "adam_t": np.int64(trainer.t), "step": np.int64(step),
           "gen_state": gen.get_state().cpu().numpy()}
    if extra is not None:
        rec["meta"] = np.array(json.dumps(extra))
    tmp = path + ".tmp.npz"
    np.savez(tmp, **rec)
    os.replace(tmp, path)


def load_checkpoint(path, trainer, gen):
    """Restore a checkpoint into the trainer and generator; returns its step."""
    import torch
    with np.load(path, allow_pickle=False) as z:
        trainer.params.copy_(torch.from_numpy(np.asarray(z["params"], np.float32)))
        trainer.m.copy_(torch.from_numpy(np.asarray(z["adam_m"], np.float32)))
        trainer.v.copy_(torch.from_numpy(np.asarray(z["adam_v"], np.float32)))
        trainer.t = int(z["adam_t"])
        gen.set_state(torch.from_numpy(np.asarray(z["gen_state"], np.uint8)))
        return int(z["step"])


def train_steps(tr, X, S, D, gen, first, last, batch, log=None, every=500, t0=None, curve=None,
                checkpoint=None, checkpoint_every=0):
    """Adam steps first..last on seeded minibatches of the rows."""
    import torch
    for step in range(first, last + 1):
        idx = torch.randint(0, X.shape[0], (batch,), device="cuda", generator=gen)
        tr.step(X[idx].contiguous(), S[idx].contiguous(), D[idx].contiguous())
        if curve is not None and (step % every == 0 or step == 1):
            loss = float(tr.loss.item())
            curve.append((step, loss))
            if log:
                log(f"[train] step {step} loss {loss:.5f} ({time.time() - (t0 or 0):.1f} s)")
        if checkpoint and checkpoint_every and step % checkpoint_every == 0:
            save_checkpoint(checkpoint, tr, gen, step)


def train(meshes=2000, steps=6000, batch=65536, lr=1e-3, seed=0, out=DEFAULT_OUT, log=print,
          checkpoint=None, checkpoint_every=0, resume=None):
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
    first = 1
    if resume:
        first = load_checkpoint(resume, tr, gen) + 1
        log(f"[train] resumed from {resume} at step {first}")
    curve = []
    train_steps(tr, X, S, D, gen, first, steps, batch, log=log, t0=t0, curve=curve, checkpoint=checkpoint,
                checkpoint_every=checkpoint_every)
    torch.cuda.synchronize()
    ev_train = evaluate(params, X, S, D)
    ev_hold = evaluate(params, Xh, Sh, Dh)
    log(f"[train] train {ev_train}  held out {ev_hold}")
    meta = {"meshes": meshes, "steps": steps, "batch": batch, "lr": lr, "seed": seed,
            "rows": int(X.shape[0]), "curve": curve, "train": ev_train, "held_out": ev_hold,
            "seconds": time.time() - t0, "resumed_at": first if resume else None}
    os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
    np.savez(out, params=params.cpu().numpy(), meta=np.array(json.dumps(meta)))
    log(f"[train] wrote {out}")
    if checkpoint:
        save_checkpoint(checkpoint, tr, gen, steps, meta)
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
    ap.add_argument("--checkpoint", default=None, help="checkpoint file written during training")
    ap.add_argument("--checkpoint-every", type=int, default=1000)
    ap.add_argument("--resume", default=None, help="checkpoint to continue from")
    a = ap.parse_args(argv)

    def log(*x):
        print(*x, flush=True)

    train(a.meshes, a.steps, a.batch, a.lr, a.seed, a.out, log, checkpoint=a.checkpoint,
          checkpoint_every=a.checkpoint_every if a.checkpoint else 0, resume=a.resume)
    return 0


if __name__ == "__main__":
    sys.exit(main())
