"""NumPy FP64 oracle of the learned-weight network and of its training step.

TEST INFRASTRUCTURE (as the rest of ``oracle/``): only the tests, the smoke
check and the CPU-baseline leg of the benchmark may import it.

The learned variant (an extension of the method; the paper uses the
incremental-stencil weights of App. C) interpolates u at i+1/2 as a convex
combination of the three 3-point candidates of the fifth-order interpolation
from u_{i-2..i+2}:

    S_l = (3u_{i-2} - 10u_{i-1} + 15u_i)/8
    S_c = (-u_{i-1} + 6u_i + 3u_{i+1})/8
    S_r = (3u_i + 6u_{i+1} - u_{i+2})/8,     linear weights d = (1/16, 10/16, 5/16)

with omega_k proportional to d_k e^{tanh z_k} / (eps + beta_k)^2: the
network's logits z rescale each classical WENO5 weight (Jiang & Shu
smoothness indicators beta_k of x, eps = 1e-6) by a factor in [1/e, e], and
z = MLP(x) comes from a 5-32-32-3 perceptron with ReLU on the normalised
stencil x_j = (u_j - u_i) r, r = 1 / max_j |u_j - u_i|.

Training pairs come from a fine solution by injection: the coarse stencil is
every other fine node, and the label is the fine node at the coarse face
(nodes sit at cell centres, so the fine node 2j+1 lies exactly on the coarse
face j+1/2 between coarse nodes j and j+1).  The loss is the mean squared
error of the interpolated value in normalised units,
    t = (label - u_i) / max_j |u_j - u_i|.

This module computes in float64 throughout (no bfloat16 rounding): it is the
reference for the gradients of the float32 training kernels.  The rounded
inference used by the solver is the C oracle's ``orc_mlp_interp``.
"""
from __future__ import annotations

import numpy as np

NPARAM = 1347
SHAPES = (("W1", (5, 32)), ("b1", (32,)), ("W2", (32, 32)), ("b2", (32,)), ("W3", (32, 3)), ("b3", (3,)))
LIN = np.array([1.0 / 16.0, 10.0 / 16.0, 5.0 / 16.0])
# candidate interpolants as rows over the stencil u_{i-2..i+2}
CAND = np.array([[3.0, -10.0, 15.0, 0.0, 0.0],
                 [0.0, -1.0, 6.0, 3.0, 0.0],
                 [0.0, 0.0, 3.0, 6.0, -1.0]]) / 8.0


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    assert p.size == NPARAM
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = p[o:o + n].reshape(shp)
        o += n
    return out


def pack(d) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def init(seed: int, last_scale: float = 0.0) -> np.ndarray:
    """He-uniform hidden layers, zero biases; the last layer scaled by
    `last_scale` (0: the initial network gives the classical WENO5 weights)."""
    rng = np.random.default_rng(seed)
    d = {"W1": rng.uniform(-1, 1, (5, 32)) * np.sqrt(6.0 / 5.0), "b1": np.zeros(32),
         "W2": rng.uniform(-1, 1, (32, 32)) * np.sqrt(6.0 / 32.0), "b2": np.zeros(32),
         "W3": rng.uniform(-1, 1, (32, 3)) * np.sqrt(6.0 / 32.0) * last_scale, "b3": np.zeros(3)}
    return pack(d)


def normalise(u5):
    """x = (u - u_i) r with r = 1 / s, s = max |u - u_i| per row (x = 0 where s = 0)."""
    u5 = np.asarray(u5, dtype=np.float64)
    du = u5 - u5[..., 2:3]
    s = np.abs(du).max(axis=-1, keepdims=True)
    r = np.divide(1.0, s, out=np.zeros_like(s), where=s > 0)
    return du * r, s[..., 0]


EPS = 1e-6
BOUND = 1.0   # the network rescales each classical weight by at most e^{+-BOUND}


def beta(X):
    """Smoothness indicators of the three candidates (Jiang & Shu) of X (n, 5)."""
    x0, x1, x2, x3, x4 = (X[:, j] for j in range(5))
    return np.stack([13 / 12 * (x0 - 2 * x1 + x2) ** 2 + 0.25 * (x0 - 4 * x1 + 3 * x2) ** 2,
                     13 / 12 * (x1 - 2 * x2 + x3) ** 2 + 0.25 * (x1 - x3) ** 2,
                     13 / 12 * (x2 - 2 * x3 + x4) ** 2 + 0.25 * (3 * x2 - 4 * x3 + x4) ** 2], axis=1)


def prior(X):
    """ln of the classical WENO5 weights' numerators d_k / (eps + beta_k)^2."""
    return np.log(LIN) - 2.0 * np.log(EPS + beta(X))


def forward(p, X):
    """Logits, weights and the activations of a batch X (n, 5)."""
    q = unpack(p)
    a1 = X @ q["W1"] + q["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ q["W2"] + q["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ q["W3"] + q["b3"]
    zc = BOUND * np.tanh(z)
    y = zc + prior(X)
    y = y - y.max(axis=1, keepdims=True)
    e = np.exp(y)
    w = e / e.sum(axis=1, keepdims=True)
    return dict(a1=a1, h1=h1, a2=a2, h2=h2, z=z, w=w)


def predict(p, X):
    """Interpolated value of the normalised stencils: sum_k w_k S_k(x)."""
    f = forward(p, X)
    return (f["w"] * (X @ CAND.T)).sum(axis=1)


def interp(p, u5):
    """Learned interpolation of raw stencils (n, 5) in float64."""
    x, s = normalise(u5)
    u5 = np.asarray(u5, dtype=np.float64)
    w = forward(p, x)["w"]
    return (w * (u5 @ CAND.T)).sum(axis=1), w


def loss(p, X, T):
    r = predict(p, X) - T
    return float(np.mean(r * r))


def grad(p, X, T):
    """Gradient of `loss` by back-propagation."""
    q = unpack(p)
    f = forward(p, X)
    n = X.shape[0]
    S = X @ CAND.T                       # (n, 3) candidate values
    w = f["w"]
    yhat = (w * S).sum(axis=1)
    dy = 2.0 * (yhat - T) / n            # d loss / d yhat
    dw = dy[:, None] * S                 # d loss / d w_k
    dzc = w * (dw - (w * dw).sum(axis=1, keepdims=True))  # softmax Jacobian
    dz = dzc * BOUND * (1.0 - np.tanh(f["z"]) ** 2)
    g = {"W3": f["h2"].T @ dz, "b3": dz.sum(axis=0)}
    dh2 = dz @ q["W3"].T * (f["a2"] > 0)
    g["W2"] = f["h1"].T @ dh2
    g["b2"] = dh2.sum(axis=0)
    dh1 = dh2 @ q["W2"].T * (f["a1"] > 0)
    g["W1"] = X.T @ dh1
    g["b1"] = dh1.sum(axis=0)
    return pack(g)


def fd_grad(p, X, T, h=1e-6, idx=None):
    """Central finite differences of `loss` (all parameters or those in idx)."""
    p = np.asarray(p, dtype=np.float64)
    idx = range(NPARAM) if idx is None else idx
    out = np.zeros(NPARAM)
    for i in idx:
        e = np.zeros(NPARAM)
        e[i] = h
        out[i] = (loss(p + e, X, T) - loss(p - e, X, T)) / (2 * h)
    return out


def adam(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected), returning new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def samples_from_fine(f, keep_degenerate=False):
    """Training pairs from one fine field f (2n nodes, transmissive problem):
    for every coarse face j+1/2 with the whole coarse stencil j-2..j+2 inside,
    the stencil (f[2(j-2)], ..., f[2(j+2)]) and the label f[2j+1]; both
    orientations (the mirrored stencil f[2(j+3)], ..., f[2(j-1)] interpolates
    to the same face from the right), all left-biased pairs first.  Returns
    (X, T) in normalised units; stencils with s <= 1e-10 max |u_j| or a label
    beyond |t| = 4 (x = 0, t = 0: they add nothing to the loss or its
    gradient) are dropped unless keep_degenerate."""
    f = np.asarray(f, dtype=np.float64)
    c = f[0::2]
    n = c.size
    X, T = [], []
    for j in range(2, n - 2):
        u5 = c[j - 2:j + 3]
        X.append(u5)
        T.append(f[2 * j + 1])
    for j in range(1, n - 3):
        u5 = c[j - 1:j + 4][::-1]
        X.append(u5)
        T.append(f[2 * j + 1])
    if not X:
        return np.zeros((0, 5)), np.zeros(0)
    U = np.array(X)
    du = U - U[:, 2:3]
    s = np.abs(du).max(axis=1)
    # variations at round-off level carry no shape, and labels beyond [-4, 4]
    # in normalised units cannot be reached by any convex combination of the
    # candidates (|S_k| <= 3.5): such pairs are neutral
    live = s > 1e-10 * np.abs(U).max(axis=1)
    r = np.divide(1.0, s, out=np.zeros_like(s), where=live)
    live &= np.abs((np.array(T) - U[:, 2]) * r) <= 4.0
    r = np.where(live, r, 0.0)
    x = du * r[:, None]
    t = (np.array(T) - U[:, 2]) * r
    if keep_degenerate:
        return x, t
    return x[live], t[live]
