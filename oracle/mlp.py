"""FP64 reference of the per-level damping-weight network.

Test infrastructure only (see ``oracle/__init__``).

The paper damps its block Jacobi smoother with one fixed weight (0.5,
Section 4.1). The learned variant predicts a weight omega_l for every level
from eight cheap statistics of the scalar rows of A_l, with a multilayer
perceptron 8 -> 32 -> 32 -> 1 (tanh hidden units) whose output
omega = 0.2 + sigmoid(z) lies in (0.2, 1.2). It is trained by minimising the
mean squared error to measured per-level optimal weights with Adam.

Neither the features nor the network are in the paper: parity unpinned
against it. The functions below are pinned by central finite differences
(gradients), the closed form of Adam's first step, and closed-form feature
values on matrices whose rows are known.

Flat parameter layout (shared with the GPU library as a data format):
W1 (32 x 8, row-major), b1 (32), W2 (32 x 32, row-major), b2 (32),
W3 (32), b3 (1): 1377 values.
"""
from __future__ import annotations

import numpy as np

from .sparse import BlockCSR

NF, NH = 8, 32
SIZES = [("W1", (NH, NF)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NH,)), ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)
OMEGA_MIN, OMEGA_SPAN = 0.2, 1.0


# --------------------------------------------------------------------------
# row statistics
# --------------------------------------------------------------------------
def row_features(M: BlockCSR, level: int) -> np.ndarray:
    """Eight statistics of the scalar rows of a block matrix (each block
    row r of node i is the scalar row 3i + r; a scalar operator applied per
    component has the same rows three times, so its own rows are used).

    For a row with diagonal d and off-diagonal entries a_j (explicit zeros
    included in the count):
      rho = sum |a_j| / |d|  (Gershgorin ratio), sigma = (d + sum a_j) / d,
      tau = sqrt(sum a_j^2) / |d|, nz = stored entries.
    Features: mean rho, max rho, std rho (population), mean sigma, mean tau,
    mean nz / 64, level / 10, log10(unknowns) / 7 where unknowns = 3 * nodes.
    Rows with a zero diagonal count with rho = sigma = tau = 0.
    """
    br, bc = M.bshape
    rows = []
    for i in range(M.nrows):
        for r in range(br):
            d = 0.0
            off = []
            for k in range(M.indptr[i], M.indptr[i + 1]):
                j = M.indices[k]
                for c in range(bc):
                    v = float(M.vals[k, r, c])
                    if j == i and c == r:
                        d = v
                    else:
                        off.append(v)
            off = np.array(off)
            if d != 0.0:
                rho = np.abs(off).sum() / abs(d)
                sigma = (d + off.sum()) / d
                tau = np.sqrt((off ** 2).sum()) / abs(d)
            else:
                rho = sigma = tau = 0.0
            rows.append((rho, sigma, tau, len(off) + 1))
    a = np.array(rows, dtype=np.float64)
    rho = a[:, 0]
    return np.array([rho.mean(), rho.max(), np.sqrt(np.mean((rho - rho.mean()) ** 2)), a[:, 1].mean(),
                     a[:, 2].mean(), a[:, 3].mean() / 64.0, level / 10.0, np.log10(3.0 * M.nrows) / 7.0])


# --------------------------------------------------------------------------
# network
# --------------------------------------------------------------------------
def unflatten(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = theta[o:o + k].reshape(shape)
        o += k
    return out


def forward(theta: np.ndarray, X: np.ndarray):
    """omega for every row of X (n x 8) and the hidden activations."""
    p = unflatten(np.asarray(theta, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64)
    h1 = np.tanh(X @ p["W1"].T + p["b1"])
    h2 = np.tanh(h1 @ p["W2"].T + p["b2"])
    z = h2 @ p["W3"] + p["b3"][0]
    s = 1.0 / (1.0 + np.exp(-z))
    return OMEGA_MIN + OMEGA_SPAN * s, (X, h1, h2, s)


def loss(theta: np.ndarray, X: np.ndarray, y: np.ndarray) -> float:
    om, _ = forward(theta, X)
    return float(np.mean((om - y) ** 2))


def gradient(theta: np.ndarray, X: np.ndarray, y: np.ndarray) -> tuple[float, np.ndarray]:
    """Loss and its gradient by the chain rule through the three layers."""
    p = unflatten(np.asarray(theta, dtype=np.float64))
    om, (X, h1, h2, s) = forward(theta, X)
    n = X.shape[0]
    e = om - y
    dz = (2.0 / n) * e * OMEGA_SPAN * s * (1.0 - s)            # dL/dz per sample
    g = {"W3": dz @ h2, "b3": np.array([dz.sum()])}
    d2 = np.outer(dz, p["W3"]) * (1.0 - h2 ** 2)               # dL/d(pre-activation of layer 2)
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ p["W2"]) * (1.0 - h1 ** 2)
    g["W1"] = d1.T @ X
    g["b1"] = d1.sum(axis=0)
    flat = np.concatenate([g[name].ravel() for name, _ in SIZES])
    return float(np.mean(e ** 2)), flat


def adam_step(theta, grad, m, v, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (Kingma and Ba, 2015) with bias correction; t counts from 1."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad ** 2
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def train(theta, X, y, steps: int, lr: float):
    """Full-batch Adam from theta; returns the parameters and the loss before every step."""
    theta = np.array(theta, dtype=np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    hist = []
    for t in range(1, steps + 1):
        L, g = gradient(theta, X, y)
        hist.append(L)
        theta, m, v = adam_step(theta, g, m, v, t, lr)
    return theta, np.array(hist)
