"""Pins of the warm-start oracle (features, network, loss gradient, Adam,
certified warm run) against what the mathematics fixes: textbook values,
identities, finite differences, library routines for the special cases
they cover (torch autograd and Adam on the CPU, torch's bfloat16 rounding),
closed forms of the features on flat and spherical meshes, and the reduction
of the warm run to the plain run."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import warm as W
from paper_1810_08218_amd import inputs as I


# ---------------------------------------------------------------- network ---

def test_bf16_rounding_nearest_even():
    ulp = 2.0 ** -7                       # bfloat16 spacing in [1, 2)
    cases = {1.0: 1.0,
             1.0 + ulp / 2: 1.0,          # tie -> even (1.0)
             1.0 + 1.5 * ulp: 1.0 + 2 * ulp,   # tie -> even (1 + 2 ulp)
             1.0 + ulp / 2 + 2.0 ** -20: 1.0 + ulp,
             -3.0: -3.0}
    for x, want in cases.items():
        assert W.bf16_round(np.float32(x)) == want, x
    torch = pytest.importorskip("torch")
    a = np.random.default_rng(0).normal(size=4096).astype(np.float32) * 10.0
    ref = torch.from_numpy(a).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(W.bf16_round(a), ref)


def test_gelu_textbook_values():
    assert W.gelu(np.array(0.0)) == 0.0
    assert abs(W.gelu(np.array(1.0)) - 0.8413447460685429) < 1e-15      # Phi(1)
    z = np.linspace(-6, 6, 101)
    assert np.allclose(W.gelu(z) - W.gelu(-z), z, atol=1e-14, rtol=0)   # Phi(z) + Phi(-z) = 1
    h = 1e-6
    fd = (W.gelu(z + h) - W.gelu(z - h)) / (2 * h)
    assert np.allclose(W.gelu_grad(z), fd, atol=1e-8)
    o = np.linspace(-30, 30, 61)
    assert np.allclose(W.softplus(o), np.log1p(np.exp(o)), rtol=1e-14)
    from scipy.special import expit
    assert np.allclose(W.sigmoid(o), expit(o), rtol=1e-14, atol=0)


def _batch(n=40, seed=3):
    rng = np.random.default_rng(seed)
    X = np.stack([rng.uniform(0, 3, n), rng.integers(0, 200, n) / 64.0, rng.normal(0, 0.05, n)], 1)
    s = rng.uniform(0.01, 0.1, n)
    d = s * 64 * X[:, 0] * rng.uniform(1.0, 1.3, n) + s * 0.1
    return X, s, d


def test_backward_matches_central_differences():
    params = W.init_params(1).astype(np.float64)
    X, s, d = _batch()
    L, g = W.loss_and_grad(params, X, s, d, round_weights=False)
    assert abs(L - W.loss_only(params, X, s, d, round_weights=False)) < 1e-14 * max(1, L)
    rng = np.random.default_rng(5)
    idx = np.concatenate([rng.choice(W.N_PARAMS, 120, replace=False),
                          [0, 191, 192, 255, 256, 4351, 4352, 4415, 4416, 4479, 4480]])
    for i in idx:
        h = 1e-4 * max(1.0, abs(params[i]))     # truncation ~h^2, rounding ~1e-16 L / h
        p1 = params.copy(); p1[i] += h
        p2 = params.copy(); p2[i] -= h
        fd = (W.loss_only(p1, X, s, d, False) - W.loss_only(p2, X, s, d, False)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * abs(g[i]) + 1e-10, (i, fd, g[i])


def test_backward_matches_torch_autograd_float64():
    torch = pytest.importorskip("torch")
    params = W.init_params(2).astype(np.float64)
    X, s, d = _batch(64, 4)
    L, g = W.loss_and_grad(params, X, s, d, round_weights=False)
    P = torch.tensor(params, dtype=torch.float64, requires_grad=True)
    W1 = P[0:192].view(3, 64); b1 = P[192:256]; W2 = P[256:4352].view(64, 64)
    b2 = P[4352:4416]; W3 = P[4416:4480]; b3 = P[4480]
    Xt, st, dt = (torch.tensor(a, dtype=torch.float64) for a in (X, s, d))
    h1 = torch.nn.functional.gelu(Xt @ W1 + b1)
    h2 = torch.nn.functional.gelu(h1 @ W2 + b2)
    o = h2 @ W3 + b3
    e = (64 * st * torch.nn.functional.softplus(o) - dt) / torch.maximum(dt, st)
    Lt = (e * e).mean()
    Lt.backward()
    assert abs(Lt.item() - L) < 1e-12 * max(1.0, L)
    assert np.allclose(P.grad.numpy(), g, rtol=1e-10, atol=1e-14)


def test_rounded_weights_gradient_is_straight_through():
    params = W.init_params(3).astype(np.float32).astype(np.float64)
    X, s, d = _batch()
    L1, g1 = W.loss_and_grad(params, X, s, d, round_weights=True)
    r = params.copy()
    for a, b in ((0, 192), (256, 4352), (4416, 4480)):
        r[a:b] = W.bf16_round(params[a:b])
    L2, g2 = W.loss_and_grad(r, X, s, d, round_weights=False)
    assert L1 == L2 and np.array_equal(g1, g2)


def test_adam_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(9)
    p = rng.normal(size=50)
    P = torch.tensor(p.copy(), requires_grad=True)
    opt = torch.optim.Adam([P], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(50)
    v = np.zeros(50)
    for t in range(1, 8):
        g = rng.normal(size=50)
        opt.zero_grad()
        P.grad = torch.tensor(g)
        opt.step()
        p, m, v = W.adam_step(p, g, m, v, t, lr=1e-2)
        assert np.allclose(P.detach().numpy(), p, rtol=1e-12, atol=1e-14)


# --------------------------------------------------------------- features ---

def test_mean_edge_on_right_isosceles_grid():
    s = 17
    m = I.flat_grid(s)
    h = 1.0 / (s - 1)
    assert abs(W.mean_edge(m.V, m.F) - h * (2 + math.sqrt(2)) / 3) < 1e-7


def test_curvature_flat_is_zero_sphere_is_minus_inverse_radius():
    m = I.flat_grid(12)
    Hc = W.mean_curvature(m.V, m.F)
    g = np.arange(144).reshape(12, 12)
    interior = g[1:-1, 1:-1].ravel()
    assert np.abs(Hc[interior]).max() < 1e-5          # float32 coordinates
    # regular icosahedron of circumradius R: five equilateral triangles per
    # vertex, every cotangent 1/sqrt(3), neighbours at cos(angle) = 1/sqrt(5);
    # the cotangent formula then gives |K| = 2 / R exactly, so H = -1 / R
    # with outward faces (K points inward)
    V0, F0 = I.icosphere64(0)
    for R in (1.0, 2.5):
        assert np.allclose(W.mean_curvature(V0 * R, F0), -1.0 / R, rtol=1e-12, atol=0)
    assert np.allclose(W.mean_curvature(V0, F0[:, [0, 2, 1]]), 1.0, rtol=1e-12, atol=0)
    # a finer icosphere approaches -1 / R (the cotangent formula is not exact
    # at the irregular vertices); exact scaling and orientation symmetry
    V, F = I.icosphere64(4)
    H1 = W.mean_curvature(V, F)
    assert abs(np.median(H1) + 1.0) < 0.02 and np.abs(H1 + 1.0).max() < 0.2
    assert np.allclose(W.mean_curvature(V * 2.5, F), H1 / 2.5, rtol=1e-12, atol=0)
    assert np.allclose(W.mean_curvature(V, F[:, [0, 2, 1]]), -H1, rtol=1e-12, atol=0)


def test_features_definition_pins():
    m = I.sphere(3, seed=4, n_sources=3)
    level, order, offs, rho = O.toplesets(m.V, m.F, m.S)
    X, scale = W.features(m.V, m.F, m.S, level)
    l = W.mean_edge(m.V, m.F)
    Vd = m.V.astype(np.float64)
    brute = np.min(np.linalg.norm(Vd[:, None, :] - Vd[m.S][None, :, :], axis=2), axis=1)
    assert np.allclose(X[:, 0] * 64 * l, brute, rtol=1e-12, atol=1e-15)
    assert np.array_equal(X[:, 1] * 64, level.astype(np.float64))
    assert (X[m.S, 0] == 0).all() and (scale == l).all()


# ------------------------------------------------------- certified warm run ---

@pytest.mark.parametrize("mesh", ["grid", "jgrid", "sphere"])
def test_warm_run_from_no_bound_is_the_plain_run(mesh):
    m = {"grid": lambda: I.flat_grid(24),
         "jgrid": lambda: I.Mesh(*I.jittered_grid(30, np.random.default_rng(2)), np.array([7, 500], np.int32)),
         "sphere": lambda: I.sphere(3, seed=1, n_sources=2)}[mesh]()
    p = O.run(m.V, m.F, m.S, 1e-5)
    for upper in (np.full(m.n, np.inf), np.full(m.n, -1.0), np.full(m.n, np.nan)):
        w = O.run_warm(m.V, m.F, m.S, 1e-5, upper)
        assert np.array_equal(w.dist, p.dist)
        assert (w.iterations, w.updates, w.rejected) == (p.iterations, p.updates, 0)
        assert np.array_equal(w.retire_k, p.retire_k)


def test_certification_soundness_and_result():
    """Certified starts stay above the fixed point whatever the input (too
    low, too high, noisy); the run from them reaches the plain result."""
    rng = np.random.default_rng(11)
    for m in (I.Mesh(*I.jittered_grid(28, rng), np.array([3], np.int32)),
              I.sphere(3, seed=5, n_sources=3), I.noisy_icosphere(level=3, seed=6)):
        dstar, _, _ = O.fixed_point(m.V, m.F, m.S)
        p = O.run(m.V, m.F, m.S, 1e-6)
        starts = {"scaled": 1.05 * dstar,
                  "low": 0.7 * dstar,
                  "noisy": dstar * rng.uniform(0.9, 1.2, m.n),
                  "random": rng.uniform(0, 3, m.n)}
        for name, w0 in starts.items():
            r = O.run_warm(m.V, m.F, m.S, 1e-6, w0)
            assert (r.certified >= dstar * (1 - 1e-12)).all(), name
            assert (r.certified[m.S] == 0).all()
            fin = np.isfinite(r.certified)
            assert np.array_equal(r.certified[fin], np.where(np.isin(np.arange(m.n), m.S), 0, w0)[fin])
            rel = np.abs(r.dist - p.dist) / np.maximum(p.dist, 1e-300)
            assert rel[np.isfinite(p.dist) & (p.dist > 0)].max() < 1e-4, name
            assert r.iterations >= r.rho - 1 or r.rho <= 1, name   # V_r retires no earlier than k = r + 1
        # an exact scaled bound loses nothing; a lone too-small value is withdrawn
        r = O.run_warm(m.V, m.F, m.S, 1e-6, 1.05 * dstar)
        assert r.rejected == 0
        w0 = 1.05 * dstar
        v = int(np.argmax(dstar))
        w0[v] = 0.5 * dstar[v]
        r = O.run_warm(m.V, m.F, m.S, 1e-6, w0)
        assert r.rejected >= 1 and np.isinf(r.certified[v])
