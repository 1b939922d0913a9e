"""ptp_solve_noalloc (the workspace is the library's fixed device scratch,
for callers that cannot allocate) against ptp_solve with a caller workspace
(the same kernels): two calls in a row, the second on a smaller mesh, each
must give the distances, labels, iterations and updates of ptp_solve exactly,
and agree with the oracle to the distance tolerance.  A plan larger than the
scratch is refused with PTP_ENOMEM."""
import ctypes as C

import numpy as np
import pytest

import oracle as O
import paper_1810_08218_amd as P
from gpu_util import rel_errors, say, to_dev
from paper_1810_08218_amd import inputs as I
from paper_1810_08218_amd import ptp as B

pytestmark = pytest.mark.gpu


def _p(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def solve_with_workspace(plan, V, F, S, work, dist, label):
    """ptp_solve through the C ABI with a caller workspace."""
    import torch
    st = B.Stats()
    rc = P.load().ptp_solve(plan._h, _p(V), _p(F), _p(S), _p(work), work.numel(), _p(dist), _p(label),
                            C.byref(st), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    d = st.as_dict()
    d["status"] = rc
    return d


def solve_both(mesh, tol, labels):
    import torch
    V, F, S = to_dev(mesh)
    ref = P.Plan(mesh.n, mesh.f, mesh.m, tol, want_labels=labels)
    work = ref.workspace()
    d_ref = torch.empty(mesh.n, dtype=torch.float32, device="cuda")
    l_ref = torch.empty(mesh.n, dtype=torch.int32, device="cuda") if labels else None
    st_ref = solve_with_workspace(ref, V, F, S, work, d_ref, l_ref)
    plan = P.Plan(mesh.n, mesh.f, mesh.m, tol, want_labels=labels)
    d = torch.full((mesh.n,), -7.0, dtype=torch.float32, device="cuda")
    lab = torch.full((mesh.n,), -7, dtype=torch.int32, device="cuda") if labels else None
    say(f"[gpu] solve_noalloc {mesh.name} n={mesh.n} m={mesh.m} labels={labels} "
        f"workspace {plan.workspace_bytes()} of {P.load().ptp_noalloc_scratch_bytes()} bytes")
    st = plan.solve_noalloc(V, F, S, d, lab)
    out = (d.cpu().numpy(), lab.cpu().numpy() if labels else None, st,
           d_ref.cpu().numpy(), l_ref.cpu().numpy() if labels else None, st_ref)
    plan.close()
    ref.close()
    return out


@pytest.mark.parametrize("labels", [False, True])
def test_noalloc_equals_solve_two_calls(cuda, labels):
    tol = 1e-4
    big = I.batch_mesh(3)                                       # jittered 319 x 319 grid, 2 sources
    small = I.bumpy_icosphere(level=6, seed=11, n_sources=5)    # 40,962 vertices
    assert small.n < big.n
    for mesh in (big, small):
        d, lab, st, d_ref, l_ref, st_ref = solve_both(mesh, tol, labels)
        assert st["status"] == P.PTP_OK and st_ref["status"] == P.PTP_OK
        assert np.array_equal(d.view(np.uint32), d_ref.view(np.uint32))
        if labels:
            assert np.array_equal(lab, l_ref)
        for k in ("iterations", "n_toplesets", "vertex_updates", "reachable"):
            assert st[k] == st_ref[k], k
        o = O.run(mesh.V, mesh.F, mesh.S, tol)
        mx, _ = rel_errors(d, o.dist, mesh.S)
        say(f"  {mesh.name}: K={st['iterations']} (oracle {o.iterations}) max rel vs oracle {mx:.2e}")
        assert st["iterations"] == o.iterations
        assert mx <= 1e-4
        assert (d[mesh.S] == 0).all()


def test_noalloc_refuses_a_plan_beyond_the_scratch(cuda):
    import torch
    mesh = I.noisy_icosphere(level=8, seed=2)       # 655,362 vertices
    plan = P.Plan(mesh.n, mesh.f, mesh.m, 1e-4)
    assert plan.workspace_bytes() > P.load().ptp_noalloc_scratch_bytes()
    V, F, S = to_dev(mesh)
    d = torch.empty(mesh.n, dtype=torch.float32, device="cuda")
    with pytest.raises(P.PTPError) as e:
        plan.solve_noalloc(V, F, S, d)
    assert e.value.status == P.PTP_ENOMEM
    assert "fixed scratch" in str(e.value)
    plan.close()
