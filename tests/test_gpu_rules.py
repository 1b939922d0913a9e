"""GPU parity of the other band controllers and of the float64 run, and the
boundary's timing fields and one-call solve, against the CPU FP64 oracle.

* fixed half band [floor((k+1)/2), k] (paper Sec. 6): the schedule is fixed,
  so the retirement record, K and U must equal the oracle's exactly, and the
  distances agree within 1e-4;
* Jacobi to the fixed point: distances within 1e-4 of the oracle's fixed
  point (the float32 and float64 runs stop at their own last change, so K may
  differ by a few sweeps);
* float64 (paper Sec. 5.1 runs single and double precision): the same
  schedule as the oracle and distances within 1e-9 (both sides compute in
  float64 from the same float32 coordinates; the GPU uses the increment form
  of the update, the oracle the matrix form, which differ by rounding only).
"""
import ctypes as C

import numpy as np
import pytest

import oracle as O
import paper_1810_08218_amd as P
from gpu_util import check_labels, gpu_run, rel_errors, say, to_dev
from paper_1810_08218_amd import inputs as I

pytestmark = pytest.mark.gpu

F64_TOL = 1e-9


def _cases():
    return [I.flat_grid(64), I.noisy_icosphere(level=5, seed=7),
            I.bumpy_icosphere(level=5, seed=4, n_sources=12), I.batch_mesh(7), I.batch_mesh(300)]


@pytest.mark.parametrize("mesh", _cases(), ids=lambda m: m.name)
def test_fixed_half_band_parity(cuda, mesh):
    o = O.run(mesh.V, mesh.F, mesh.S, 1e-4, band_rule=1)
    g = gpu_run(mesh, 1e-4, labels=True, band_rule=P.BAND_FIXED_HALF)
    mx, mean = rel_errors(g.dist, o.dist, mesh.S)
    say(f"  K {g.iterations}/{o.iterations} rho {g.rho} U {g.updates}/{o.updates} max rel {mx:.2e}")
    assert g.iterations == o.iterations == max(1, 2 * o.rho - 3)
    assert g.updates == o.updates and np.array_equal(g.retire, o.retire_k)
    assert mx <= 1e-4
    n_lab, n_par = check_labels(mesh, g.label, g.parent, o.dist)
    say(f"  label mismatches {n_lab}, parent ties {n_par}")


@pytest.mark.parametrize("mesh", _cases(), ids=lambda m: m.name)
def test_jacobi_reaches_the_fixed_point(cuda, mesh):
    fp, lab, sweeps = O.fixed_point(mesh.V, mesh.F, mesh.S)
    g = gpu_run(mesh, 1e-4, labels=True, band_rule=P.BAND_JACOBI)
    mx, mean = rel_errors(g.dist, fp, mesh.S)
    say(f"  K {g.iterations} oracle sweeps {sweeps} rho {g.rho} max rel {mx:.2e} mean {mean:.2e}")
    assert g.status == P.PTP_OK
    assert mx <= 1e-4
    assert g.rho - 1 <= g.iterations
    n_lab, n_par = check_labels(mesh, g.label, g.parent, fp)
    say(f"  label mismatches {n_lab}, parent ties {n_par}")


@pytest.mark.parametrize("mesh", _cases() + [I.flat_grid(37, source=(20, 11))], ids=lambda m: m.name)
def test_float64_parity(cuda, mesh):
    tol = 1e-6 if mesh.name.startswith("grid") else 1e-4
    o = O.run(mesh.V, mesh.F, mesh.S, tol)
    g = gpu_run(mesh, tol, f64=True)
    assert g.dist.dtype == np.float64
    mx, mean = rel_errors(g.dist, o.dist, mesh.S)
    say(f"  K {g.iterations}/{o.iterations} U {g.updates}/{o.updates} max rel {mx:.2e} mean {mean:.2e}")
    assert np.array_equal(g.retire, o.retire_k)
    assert (g.iterations, g.updates) == (o.iterations, o.updates)
    assert mx <= F64_TOL
    assert (g.dist[mesh.S] == 0).all()
    assert np.array_equal(np.isinf(g.dist), np.isinf(o.dist))


def test_float64_rejects_labels(cuda):
    import torch
    m = I.flat_grid(8)
    V, F, S = to_dev(m)
    plan = P.Plan(m.n, m.f, m.m, 1e-4, want_labels=True)
    plan.prepare(V, F, S)
    with pytest.raises(P.PTPError) as e:
        plan.run_f64(torch.empty(m.n, dtype=torch.float64, device="cuda"))
    assert e.value.status == P.PTP_EUNSUPPORTED


def test_float64_batch_equals_single_plans(cuda):
    import torch
    meshes = [I.batch_mesh(t) for t in (7, 300, 301, 12)]
    V, F, S, descs, out_len = P.concat(meshes)
    b = P.Batch(descs, 1e-4)
    b.prepare(*(torch.from_numpy(x).cuda() for x in (V, F, S)))
    d = torch.empty(out_len, dtype=torch.float64, device="cuda")
    b.run_f64(d)
    rc, st, _ = b.stats()
    assert rc == P.PTP_OK
    for k, m in enumerate(meshes):
        g = gpu_run(m, 1e-4, f64=True, want_order=False)
        o0 = int(descs[k].out_off)
        assert np.array_equal(d[o0:o0 + m.n].cpu().numpy(), g.dist)
        assert st[k]["iterations"] == g.iterations


def test_stats_report_times(cuda):
    m = I.noisy_icosphere(level=6, seed=5)
    g = gpu_run(m, 1e-4)
    st = g.stats
    say(f"  ms_prepare {st['ms_prepare']:.3f} ms_run {st['ms_run']:.3f}")
    assert st["ms_prepare"] > 0 and st["ms_run"] > 0
    assert st["ms_mesh_begin"] == 0.0 and st["ms_mesh_end"] > 0
    assert st["ms_mesh_end"] <= st["ms_run"]


def test_solve_entry_point_equals_prepare_and_run(cuda):
    """ptp_solve (prepare + run + synchronise) called directly through the C
    ABI gives the prepare + run result bit for bit and fills the stats."""
    import torch
    m = I.bumpy_icosphere(level=5, seed=2, n_sources=6)
    ref = gpu_run(m, 1e-4, labels=True, want_order=False)
    lib = P.load()
    V, F, S = to_dev(m)
    plan = P.Plan(m.n, m.f, m.m, 1e-4, want_labels=True)
    work = plan.workspace()
    d = torch.empty(m.n, dtype=torch.float32, device="cuda")
    lab = torch.empty(m.n, dtype=torch.int32, device="cuda")
    st = P.ptp.Stats()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.ptp_solve(plan._h, C.c_void_p(V.data_ptr()), C.c_void_p(F.data_ptr()), C.c_void_p(S.data_ptr()),
                       C.c_void_p(work.data_ptr()), work.numel(), C.c_void_p(d.data_ptr()),
                       C.c_void_p(lab.data_ptr()), C.byref(st), stream)
    assert rc == P.PTP_OK
    assert np.array_equal(d.cpu().numpy(), ref.dist) and np.array_equal(lab.cpu().numpy(), ref.label)
    assert (st.iterations, st.vertex_updates) == (ref.iterations, ref.updates)
    assert st.ms_prepare > 0 and st.ms_run > 0
    # a bad workspace size is reported, not crashed on
    rc = lib.ptp_solve(plan._h, C.c_void_p(V.data_ptr()), C.c_void_p(F.data_ptr()), C.c_void_p(S.data_ptr()),
                       C.c_void_p(work.data_ptr()), 16, C.c_void_p(d.data_ptr()), C.c_void_p(lab.data_ptr()),
                       None, stream)
    assert rc == P.PTP_ENOMEM
