"""Many source sets on one mesh in one batch (the meshes share the V and F
rows): every set's distances and labels equal those of a plan prepared for
that set alone, bit for bit, and two sets match the oracle."""
import numpy as np
import pytest

import oracle as O
import paper_1810_08218_amd as P
from gpu_util import rel_errors, say
from paper_1810_08218_amd import inputs as I

pytestmark = pytest.mark.gpu


def test_sixty_four_source_sets_share_rows(cuda):
    import torch
    base = I.noisy_icosphere(level=6, seed=4)
    rng = np.random.default_rng(41)
    meshes = []
    for k in range(64):
        m = int(rng.integers(1, 33))
        S = rng.choice(base.n, m, replace=False).astype(np.int32)
        meshes.append(I.Mesh(base.V, base.F, S, name=f"set{k}"))
    V, F, S, descs, out_len = P.concat(meshes, [None] + [0] * 63)
    assert V.shape[0] == base.n and F.shape[0] == base.f          # rows stored once
    dV, dF, dS = (torch.from_numpy(x).cuda() for x in (V, F, S))
    tol = 1e-4
    b = P.Batch(descs, tol, want_labels=True)
    b.prepare(dV, dF, dS)
    dist = torch.empty(out_len, dtype=torch.float32, device="cuda")
    lab = torch.empty(out_len, dtype=torch.int32, device="cuda")
    b.run(dist, lab)
    rc, stats, status = b.stats()
    assert rc == P.PTP_OK and all(s == P.PTP_OK for s in status)
    d_all, l_all = dist.cpu().numpy(), lab.cpu().numpy()
    for k, m in enumerate(meshes):
        plan = P.Plan(m.n, m.f, m.m, tol, want_labels=True)
        plan.prepare(dV, dF, torch.from_numpy(m.S).cuda())
        d1 = torch.empty(m.n, dtype=torch.float32, device="cuda")
        l1 = torch.empty(m.n, dtype=torch.int32, device="cuda")
        plan.run(d1, l1)
        st = plan.stats()
        o0 = int(descs[k].out_off)
        assert np.array_equal(d1.cpu().numpy(), d_all[o0:o0 + m.n]), m.name
        assert np.array_equal(l1.cpu().numpy(), l_all[o0:o0 + m.n]), m.name
        assert (st["iterations"], st["vertex_updates"]) == \
            (stats[k]["iterations"], stats[k]["vertex_updates"]), m.name
    for k in (0, 37):
        m = meshes[k]
        o = O.run(m.V, m.F, m.S, tol)
        o0 = int(descs[k].out_off)
        mx, mean = rel_errors(d_all[o0:o0 + m.n], o.dist, m.S)
        say(f"[sets] {m.name} m={m.m} K {stats[k]['iterations']}/{o.iterations} max rel {mx:.2e}")
        assert (stats[k]["iterations"], stats[k]["vertex_updates"]) == (o.iterations, o.updates)
        assert mx <= 1e-4
