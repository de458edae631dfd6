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
@pytest.mark.parametrize("tscale", [0.5, 20.0])
def test_gradient_matches_central_differences(mesh, tscale):
    """Both branches of the per-sample normaliser max(1, mean t^2)."""
    g, op = _graph(mesh)
    rng = np.random.default_rng(1)
    theta = mpnn.init_params(4) + 0.05 * rng.standard_normal(mpnn.n_params())
    X = rng.standard_normal((g.n, 5))
    t = tscale * rng.standard_normal(g.n)
    L, grad = mpnn.loss_grad(theta, g, X, t)
    idx = rng.choice(theta.size, size=60, replace=False)
    eps = 1e-6
    for k in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += eps
        tm[k] -= eps
        fd = (mpnn.loss(tp, g, X, t) - mpnn.loss(tm, g, X, t)) / (2 * eps)
        assert abs(fd - grad[k]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9, (k, fd, grad[k])
    # the normaliser: a sample with large targets weighs as one with rms 1
    y, _ = mpnn.forward(theta, g, X)
    want = np.mean((y - t) ** 2) / max(1.0, np.mean(t * t))
    assert L == pytest.approx(want, rel=1e-14)


def test_zero_decoder_returns_quadratic_extrapolation():
    g, op = _graph(unit_square(5))
    theta = mpnn.init_params(0)
    p = mpnn.unpack(theta)
    p["w"][...] = 0.0
    p["c"][...] = 0.0
    rng = np.random.default_rng(0)
    hist = rng.standard_normal((4, g.n))
    b = rng.standard_normal(g.n)
    np.testing.assert_allclose(mpnn.guess(theta, g, b, hist),
                               3 * hist[0] - 3 * hist[1] + hist[2], rtol=1e-13, atol=1e-13)


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


def _readout_net(rows, weights):
    """Parameters whose output is y = sum_k weights[k] relu(x . rows[k]):
    encoder rows as given, zero residual updates, linear decoder."""
    theta = mpnn.init_params(0)
    p = mpnn.unpack(theta)
    p["We"][...] = 0.0
    p["ce"][...] = 0.0
    for k, r in enumerate(rows):
        p["We"][k] = r
    for r in range(mpnn.ROUNDS):
        p[f"U{r}"][...] = 0.0
        p[f"v{r}"][...] = 0.0
    p["w"][...] = 0.0
    p["w"][:len(weights)] = weights
    p["c"][...] = 0.0
    return theta


def _e(k):
    v = np.zeros(mpnn.NFEAT)
    v[k] = 1.0
    return v


def _history(n, seed, order=2):
    """phi at t = 0, -1, -2, -3 of a per-node polynomial in t; returns the
    history and phi at t = 1."""
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((order + 1, n))
    at = lambda t: sum(c[k] * (0.5 * t) ** k for k in range(order + 1))  # noqa: E731
    return np.stack([at(t) for t in (0.0, -1.0, -2.0, -3.0)]), at(1.0)


def test_extrapolation_features_are_exact_for_polynomial_histories():
    """Zero output continues a history that is quadratic in time exactly;
    y = e / s (the input column of the last extrapolation error) continues a
    cubic history exactly.  Rounding aside, the guess is then independent of
    b."""
    g, op = _graph(disc(16, 24, seed=7))
    b = np.random.default_rng(2).standard_normal(g.n)
    hist, nxt = _history(g.n, 1, order=2)
    zero = _readout_net([], [])
    np.testing.assert_allclose(mpnn.guess(zero, g, b, hist), nxt, rtol=1e-11, atol=1e-11)
    hist, nxt = _history(g.n, 2, order=3)
    cubic = _readout_net([_e(2), -_e(2)], [1.0, -1.0])
    np.testing.assert_allclose(mpnn.guess(cubic, g, b, hist), nxt, rtol=1e-11, atol=1e-11)
    # and the quadratic extrapolation alone misses the cubic term
    assert np.linalg.norm(mpnn.guess(zero, g, b, hist) - nxt) > 1e-2 * np.linalg.norm(nxt)
    X, q, s = mpnn.features(g, b, hist)
    np.testing.assert_allclose(mpnn.target(q, s, nxt), X[:, 2], rtol=1e-10, atol=1e-10)


@pytest.mark.parametrize("with_natural", [False, True])
def test_residual_feature_is_one_richardson_step(with_natural):
    """y = omega rho / s gives q + omega (b - K q) on the solver's system:
    free rows couple to free columns only, phi = 0 rows are identity
    rows."""
    mesh = unit_square(7)
    op = fem.Operators(mesh)
    nat = np.zeros(op.n, bool)
    if with_natural:
        nat[np.isclose(op.xy[:, 0], 1.0)] = True
    g = mpnn.Graph(op.xy, op.K, nat if with_natural else None)
    hist = np.random.default_rng(3).standard_normal((4, op.n))
    b = np.random.default_rng(4).standard_normal(op.n)
    omega = 0.25
    net = _readout_net([_e(1), -_e(1)], [omega, -omega])
    Kd = op.K.toarray()
    f = ~nat
    q = 3 * hist[0] - 3 * hist[1] + hist[2]
    want = q.copy()
    want[f] += omega * (b[f] - Kd[np.ix_(f, f)] @ q[f])
    want[nat] += omega * (b[nat] - q[nat])
    np.testing.assert_allclose(mpnn.guess(net, g, b, hist), want, rtol=1e-12, atol=1e-12)


def test_scale_fallbacks():
    """s = rms(e), floored at 1e-12 rms(phi^n) (a history quadratic in time
    has e = 0 up to rounding); without a history, rms(b) / hbar^2."""
    g, op = _graph(unit_square(6))
    rng = np.random.default_rng(5)
    b = rng.standard_normal(g.n)
    r = rng.standard_normal((4, g.n))
    rms = lambda v: np.linalg.norm(v) / np.sqrt(g.n)  # noqa: E731
    quad = np.stack([r[0], r[0] - r[1] + r[2], r[0] - 2 * r[1] + 4 * r[2],
                     r[0] - 3 * r[1] + 9 * r[2]])
    first = np.stack([r[0], 0 * r[0], 0 * r[0], 0 * r[0]])
    cases = [
        (r, rms(r[0] - 3 * r[1] + 3 * r[2] - r[3])),
        (first, rms(r[0])),
        (quad, 1e-12 * rms(r[0])),
        (np.zeros((4, g.n)), rms(b) / g.hbar ** 2),
    ]
    for hist, want in cases:
        _, _, s = mpnn.features(g, b, hist)
        assert s == pytest.approx(want, rel=1e-10)
