"""CPU FP64 oracle of the learned warm start: features, network, loss and
gradient, Adam.

TEST INFRASTRUCTURE ONLY, like the rest of this package: only ``tests/``, the
smoke check and the benchmark's CPU-baseline leg may import it.  Plain numpy
in float64, written from the definitions below; it shares nothing with the
HIP library.

The warm start is an extension of the method (the paper starts every
non-source vertex at +inf).  Its definitions:

Features of vertex v (caller order), for a mesh with mean edge length l =
mean over the triangles of their three edge lengths:
  f1(v)  = min over sources s of |x_v - x_s|   (Euclidean)
  hop(v) = topleset index r with v in V_r (Sec. 4.1), -1 if unreachable
  H(v)   = signed discrete mean curvature: K(v) = (1 / 2A) sum over incident
           triangles (v, a, b) of cot(angle at b)(x_a - x_v) + cot(angle at
           a)(x_b - x_v), A = a third of the incident triangle areas,
           H = |K| / 2 with the sign of K . n(v), n(v) = sum of the incident
           face normals (x_a - x_v) x (x_b - x_v); (a, b) follows the
           triangle's vertex order after v.  Degenerate triangles (zero area)
           add no cotangent term.
Network input x = (f1 / l / 64, hop / 64, H l), scale l.

Network: h1 = gelu(x W1 + b1), h2 = gelu(h1 W2 + b2), o = h2 . W3 + b3,
d^ = 64 l softplus(o); gelu(z) = z Phi(z) with the exact normal CDF.  The
parameter vector is [W1 (3x64) | b1 | W2 (64x64) | b2 | W3 | b3], matrices
input-major; the weight matrices are used rounded to bfloat16 (nearest
even), and the gradient treats that rounding as the identity.

Loss over rows i: L = mean_i ((d^_i - d_i) / max(d_i, l_i))^2.

Adam (bias-corrected): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

H = 64
N_PARAMS = 3 * H + H + H * H + H + H + 1


def bf16_round(a):
    """Round float32 values to the nearest bfloat16 (ties to even); returns
    float64.  Infinities and NaNs pass through."""
    x = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = x.view(np.uint32).astype(np.uint64)
    finite = (u & 0x7F800000) != 0x7F800000
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    r = np.where(finite, r, u >> 16)
    return (r.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def unpack(params):
    p = np.asarray(params, dtype=np.float64)
    if p.shape != (N_PARAMS,):
        raise ValueError(f"expected {N_PARAMS} parameters")
    o = 0
    W1 = p[o:o + 3 * H].reshape(3, H); o += 3 * H
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + H]; o += H
    b3 = p[o]
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, W3, [b3]]).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def softplus(o):
    return np.logaddexp(0.0, o)


def sigmoid(o):
    e = np.exp(-np.abs(o))
    return np.where(o >= 0, 1.0 / (1.0 + e), e / (1.0 + e))


def _weights(params, round_weights=True):
    W1, b1, W2, b2, W3, b3 = unpack(params)
    if round_weights:
        W1, W2, W3 = bf16_round(W1), bf16_round(W2), bf16_round(W3)
    return W1, b1, W2, b2, W3, b3


def forward(params, X, scale, round_weights=True):
    """d^ = 64 scale softplus(o(X)) for rows X[n, 3]; also returns o."""
    W1, b1, W2, b2, W3, b3 = _weights(params, round_weights)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1 + b1
    h1 = gelu(z1)
    z2 = h1 @ W2 + b2
    h2 = gelu(z2)
    o = h2 @ W3 + b3
    return 64.0 * np.asarray(scale, dtype=np.float64) * softplus(o), o


def loss_and_grad(params, X, scale, target, round_weights=True):
    """L = mean ((d^ - d) / max(d, scale))^2 and dL/dparams, by hand-derived
    backpropagation through the three layers."""
    W1, b1, W2, b2, W3, b3 = _weights(params, round_weights)
    X = np.asarray(X, dtype=np.float64)
    s = np.asarray(scale, dtype=np.float64)
    d = np.asarray(target, dtype=np.float64)
    n = X.shape[0]
    z1 = X @ W1 + b1
    h1 = gelu(z1)
    z2 = h1 @ W2 + b2
    h2 = gelu(z2)
    o = h2 @ W3 + b3
    den = np.maximum(d, s)
    e = (64.0 * s * softplus(o) - d) / den
    L = float(np.mean(e * e))
    go = 2.0 * e / den * 64.0 * s * sigmoid(o) / n          # dL/do
    gW3 = h2.T @ go
    gb3 = go.sum()
    gz2 = np.outer(go, W3) * gelu_grad(z2)
    gW2 = h1.T @ gz2
    gb2 = gz2.sum(axis=0)
    gz1 = (gz2 @ W2.T) * gelu_grad(z1)
    gW1 = X.T @ gz1
    gb1 = gz1.sum(axis=0)
    return L, pack(gW1, gb1, gW2, gb2, gW3, gb3)


def loss_only(params, X, scale, target, round_weights=True):
    dh, _ = forward(params, X, scale, round_weights)
    d = np.asarray(target, dtype=np.float64)
    e = (dh - d) / np.maximum(d, np.asarray(scale, dtype=np.float64))
    return float(np.mean(e * e))


def adam_step(params, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """Returns (params, m, v) after step t >= 1."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed=0):
    """Seeded initial parameters: uniform(+-1/sqrt(fan_in)) weights and
    biases (the usual default of a linear layer)."""
    rng = np.random.default_rng(seed)

    def lin(fi, fo):
        k = 1.0 / np.sqrt(fi)
        return rng.uniform(-k, k, (fi, fo)), rng.uniform(-k, k, fo)

    W1, b1 = lin(3, H)
    W2, b2 = lin(H, H)
    W3, b3 = lin(H, 1)
    return pack(W1, b1, W2, b2, W3[:, 0], b3[0]).astype(np.float32)


# ------------------------------------------------------------ features ---

def mean_edge(V, F):
    """Mean over the triangles of their three edge lengths (1 without faces)."""
    X = np.asarray(V, dtype=np.float64)
    F = np.asarray(F, dtype=np.int64).reshape(-1, 3)
    if F.shape[0] == 0:
        return 1.0
    e = [np.linalg.norm(X[F[:, (c + 1) % 3]] - X[F[:, c]], axis=1) for c in range(3)]
    lsum = float(np.sum(e[0]) + np.sum(e[1]) + np.sum(e[2]))
    return lsum / (3.0 * F.shape[0]) if lsum > 0 else 1.0


def mean_curvature(V, F):
    """Signed discrete mean curvature per vertex (definition in the module
    docstring), with plain loops over the triangles' corners."""
    X = np.asarray(V, dtype=np.float64)
    F = np.asarray(F, dtype=np.int64).reshape(-1, 3)
    n = X.shape[0]
    K = np.zeros((n, 3))
    nrm = np.zeros((n, 3))
    area = np.zeros(n)
    for c in range(3):
        v = F[:, c]
        a = F[:, (c + 1) % 3]
        b = F[:, (c + 2) % 3]
        pa = X[a] - X[v]
        pb = X[b] - X[v]
        q = np.cross(pa, pb)
        dbl = np.linalg.norm(q, axis=1)                       # twice the area
        np.add.at(nrm, v, q)
        np.add.at(area, v, dbl / 6.0)
        ok = dbl > 0
        safe = np.where(ok, dbl, 1.0)
        cot_a = np.einsum("ij,ij->i", X[v] - X[a], X[b] - X[a]) / safe   # angle at a
        cot_b = np.einsum("ij,ij->i", X[v] - X[b], X[a] - X[b]) / safe   # angle at b
        term = cot_b[:, None] * pa + cot_a[:, None] * pb
        np.add.at(K, v, np.where(ok[:, None], term, 0.0))
    Hc = np.zeros(n)
    has = area > 0
    Kn = K[has] / (2.0 * area[has])[:, None]
    h = 0.5 * np.linalg.norm(Kn, axis=1)
    sign = np.where(np.einsum("ij,ij->i", Kn, nrm[has]) < 0, -1.0, 1.0)
    Hc[has] = sign * h
    return Hc


def features(V, F, S, level):
    """Network inputs X[n, 3] and scale[n] (-1 where unreachable), given the
    topleset index per vertex (-1 unreachable)."""
    Xc = np.asarray(V, dtype=np.float64)
    S = np.asarray(S, dtype=np.int64)
    lvl = np.asarray(level)
    n = Xc.shape[0]
    l = mean_edge(V, F)
    f1 = np.full(n, np.inf)
    for s in S:
        f1 = np.minimum(f1, np.linalg.norm(Xc - Xc[s], axis=1))
    Hc = mean_curvature(V, F)
    X = np.stack([f1 / l / 64.0, lvl / 64.0, Hc * l], axis=1)
    scale = np.full(n, l)
    unreach = lvl < 0
    X[unreach] = 0.0
    scale[unreach] = -1.0
    return X, scale


def predict(params, V, F, S, level, inflate=1.05):
    """Warm-start upper bound in caller order: inflate * d^, 0 at the
    sources, +inf where unreachable."""
    X, scale = features(V, F, S, level)
    dh, _ = forward(params, X, np.where(scale > 0, scale, 0.0))
    w = inflate * dh
    w[np.asarray(level) < 0] = np.inf
    w[np.asarray(S, dtype=np.int64)] = 0.0
    return w
