"""Pins of the FP64 learned-guess network: analytic gradient vs central
differences, architecture invariants, and the Adam step."""
import numpy as np
import pytest

from oracle import fem, mpnn
from workloads import unit_square, disc


def _graph(mesh):
    op = fem.Operators(mesh)
    return mpnn.Graph(op.xy, op.K), op


def test_layout_and_size():
    assert mpnn.n_params() == 32 * 5 + 32 + 3 * (2 * 32 * 32 + 32 * 3 + 32 + 32 * 64 + 32) + 33
    theta = mpnn.init_params(0)
    p = mpnn.unpack(theta)
    assert p["U2"].shape == (32, 64) and p["c"].shape == (1,)


def test_graph_edges_both_directions():
    g, op = _graph(disc(20, 30, seed=2))
    pairs = set(zip(g.src.tolist(), g.dst.tolist()))
    assert all((j, i) in pairs for i, j in pairs)
    assert len(pairs) == op.K.nnz - op.n
    np.testing.assert_allclose(g.deg, np.diff(op.K.indptr) - 1)


@pytest.mark.parametrize("mesh", [unit_square(6), disc(14, 20, seed=3)])
def test_gradient_matches_central_differences(mesh):
    g, op = _graph(mesh)
    rng = np.random.default_rng(1)
    theta = mpnn.init_params(4) + 0.05 * rng.standard_normal(mpnn.n_params())
    X = rng.standard_normal((g.n, 5))
    t = rng.standard_normal(g.n)
    L, grad = mpnn.loss_grad(theta, g, X, t)
    idx = rng.choice(theta.size, size=60, replace=False)
    eps = 1e-6
    for k in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += eps
        tm[k] -= eps
        fd = (mpnn.loss(tp, g, X, t) - mpnn.loss(tm, g, X, t)) / (2 * eps)
        assert abs(fd - grad[k]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9, (k, fd, grad[k])


def test_zero_decoder_returns_previous_increment():
    g, op = _graph(unit_square(5))
    theta = mpnn.init_params(0)
    p = mpnn.unpack(theta)
    p["w"][...] = 0.0
    p["c"][...] = 0.0
    rng = np.random.default_rng(0)
    hist = rng.standard_normal((4, g.n))
    b = rng.standard_normal(g.n)
    np.testing.assert_array_equal(mpnn.guess(theta, g, b, hist), hist[0])


def test_scale_equivariance():
    """Inputs are normalised: scaling b and the history by the same factor
    scales the guess by that factor."""
    g, op = _graph(disc(16, 24, seed=5))
    theta = mpnn.init_params(3)
    rng = np.random.default_rng(2)
    hist = rng.standard_normal((4, g.n))
    b = rng.standard_normal(g.n)
    np.testing.assert_allclose(mpnn.guess(theta, g, 7.5 * b, 7.5 * hist),
                               7.5 * mpnn.guess(theta, g, b, hist), rtol=1e-12, atol=1e-12)


def test_adam_first_step_moves_by_lr_times_sign():
    rng = np.random.default_rng(0)
    theta = rng.standard_normal(50)
    grad = rng.standard_normal(50)
    m, v = np.zeros(50), np.zeros(50)
    t0 = theta.copy()
    mpnn.adam_step(theta, grad, m, v, 1, lr=1e-3)
    # bias-corrected first step: |delta| = lr * |g| / (|g| + eps) ~= lr
    np.testing.assert_allclose(t0 - theta, 1e-3 * np.sign(grad), rtol=1e-4)


def test_training_reduces_loss_on_a_fixed_sample():
    g, op = _graph(unit_square(7))
    rng = np.random.default_rng(3)
    X = rng.standard_normal((g.n, 5))
    t = 0.3 * X[:, 1] - 0.2 * X[:, 2] + 0.1 * X[:, 0]
    theta = mpnn.init_params(1)
    m, v = np.zeros_like(theta), np.zeros_like(theta)
    L0 = mpnn.loss(theta, g, X, t)
    for k in range(1, 201):
        _, gr = mpnn.loss_grad(theta, g, X, t)
        mpnn.adam_step(theta, gr, m, v, k, lr=3e-3)
    assert mpnn.loss(theta, g, X, t) < 0.1 * L0
