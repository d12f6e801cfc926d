"""Pins of the oracle's damping-weight network and row features: finite
differences, Adam's closed-form first step, closed-form feature values."""
import numpy as np
import pytest

import synth
from oracle import mlp
from oracle.sparse import BlockCSR


def test_layout_size():
    assert mlp.NPARAM == 8 * 32 + 32 + 32 * 32 + 32 + 32 + 1 == synth.mlp_init().size


def test_gradient_matches_central_differences():
    theta = synth.mlp_init(1)
    X, y = synth.mlp_batch(13, 1)
    L, g = mlp.gradient(theta, X, y)
    assert abs(L - mlp.loss(theta, X, y)) < 1e-15
    h = 1e-6
    fd = np.empty_like(theta)
    for k in range(theta.size):
        e = np.zeros_like(theta)
        e[k] = h
        fd[k] = (mlp.loss(theta + e, X, y) - mlp.loss(theta - e, X, y)) / (2 * h)
    scale = np.abs(fd).max()
    assert np.abs(g - fd).max() < 1e-7 * scale, np.abs(g - fd).max() / scale
    # every layer receives a gradient (no dropped term)
    o = 0
    for name, shape in mlp.SIZES:
        k = int(np.prod(shape))
        assert np.abs(g[o:o + k]).max() > 0, name
        o += k


def test_adam_first_step_closed_form():
    theta = synth.mlp_init(2)
    g = np.linspace(-1.0, 1.0, theta.size)
    new, m, v = mlp.adam_step(theta, g, np.zeros_like(g), np.zeros_like(g), 1, 0.01)
    # t = 1: bias-corrected moments are g and g^2, so the step is lr * g / (|g| + eps)
    assert np.abs(new - (theta - 0.01 * g / (np.abs(g) + 1e-8))).max() < 1e-15
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g ** 2)


def test_adam_constant_gradient_moves_lr_per_step():
    # with a constant gradient the bias-corrected moments stay g, g^2: each step is lr * sign(g)
    theta = np.zeros(4)
    g = np.array([2.0, -3.0, 0.5, -0.25])
    m = v = np.zeros(4)
    for t in range(1, 6):
        theta, m, v = mlp.adam_step(theta, g, m, v, t, 0.1, eps=0.0)
    assert np.allclose(theta, -5 * 0.1 * np.sign(g), rtol=0, atol=1e-12)


def test_output_range_and_training_fits_a_network_target():
    X, _ = synth.mlp_batch(64, 3)
    teacher = synth.mlp_init(7)
    y, _ = mlp.forward(teacher, X)
    om, _ = mlp.forward(synth.mlp_init(0), X * 100.0)
    assert np.all(om > 0.2) and np.all(om < 1.2)
    theta, hist = mlp.train(synth.mlp_init(0), X, y, 400, 0.01)
    assert mlp.loss(theta, X, y) < 0.02 * hist[0]


def _scalar(indptr, indices, vals, n):
    return BlockCSR(np.array(indptr), np.array(indices), np.array(vals, dtype=float).reshape(-1, 1, 1), n)


def test_features_1d_laplacian_closed_form():
    n = 5
    indptr, indices, vals = [0], [], []
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                indices.append(j)
                vals.append(2.0 if i == j else -1.0)
        indptr.append(len(indices))
    f = mlp.row_features(_scalar(indptr, indices, vals, n), 2)
    # interior rows: rho 1, sigma 0, tau sqrt(2)/2, 3 entries; end rows: 0.5, 0.5, 0.5, 2 entries
    rho = np.array([0.5, 1, 1, 1, 0.5])
    expect = [rho.mean(), 1.0, rho.std(), (2 * 0.5) / 5, (3 * np.sqrt(2) / 2 + 2 * 0.5) / 5, (3 * 3 + 2 * 2) / 5 / 64,
              0.2, np.log10(15) / 7]
    assert np.allclose(f, expect, rtol=0, atol=1e-15)


def test_features_block_identity_and_scaling():
    n = 4
    vals = np.zeros((n, 3, 3))
    vals[:] = np.eye(3) * 7.0
    M = BlockCSR(np.arange(n + 1), np.arange(n), vals, n)
    f = mlp.row_features(M, 0)
    assert np.allclose(f, [0, 0, 0, 1, 0, 3 / 64, 0, np.log10(12) / 7], atol=1e-15)
    # the ratios are invariant under scaling the matrix
    rng = np.random.default_rng(0)
    A = rng.standard_normal((6, 6))
    A = A + A.T + 12 * np.eye(6)
    blocks = np.array([A[3 * i:3 * i + 3, 3 * j:3 * j + 3] for i in range(2) for j in range(2)])
    M2 = BlockCSR(np.array([0, 2, 4]), np.array([0, 1, 0, 1]), blocks, 2)
    M3 = BlockCSR(np.array([0, 2, 4]), np.array([0, 1, 0, 1]), -4.5 * blocks, 2)
    assert np.allclose(mlp.row_features(M2, 1), mlp.row_features(M3, 1), atol=1e-14)
    # dense recomputation of rho for the first row
    r0 = np.abs(A[0, 1:]).sum() / abs(A[0, 0])
    rows = [np.abs(np.delete(A[i], i)).sum() / abs(A[i, i]) for i in range(6)]
    assert abs(max(rows) - mlp.row_features(M2, 1)[1]) < 1e-14 and r0 in rows
