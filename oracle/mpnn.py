"""FP64 reference of the learned initial guess for the coarse Poisson solve.

Oracle (test infrastructure only).  The paper solves Eq. 23 from scratch every
step; the library can start its PCG from a guess predicted by a small
message-passing network on the coarse mesh, and keeps the plain previous-step
guess whenever the network's initial residual is worse.  This module is the
plain FP64 definition of that network, its loss, its gradient (written out by
the chain rule) and one Adam step; the tests check the gradient against
central differences and the GPU kernels against this module.

Network (hidden width H = 32, R = 3 rounds), on the coarse node graph (edges
= off-diagonal slots of the coarse stiffness matrix, both directions):
  history  q = 3 phi^n - 3 phi^{n-1} + phi^{n-2} (quadratic extrapolation in
           time), e = phi^n - 3 phi^{n-1} + 3 phi^{n-2} - phi^{n-3} (the error
           the same extrapolation made for phi^n), d_1 = phi^n - phi^{n-1},
           d_2 = phi^n - 2 phi^{n-1} + phi^{n-2}
  residual rho = b - K q, K the solver's coarse operator (Eq. 23 with the
           phi = 0 rows and columns replaced by identity)
  scales   s_b = rms(b) (1 if zero); s = max(rms(e), 1e-12 rms(phi^n)) (the
           floor keeps s above the rounding level of e), or s_b / hbar^2 if
           that is zero (the coarse Poisson solution scales like b / h^2);
           s_k = rms(d_k) (1 if zero)
  input    x_i = [b_i / s_b, rho_i / s, e_i / s, d_1,i / s_1, d_2,i / s_2]
           The network refines the FP64 extrapolation q in units of its
           expected error, so a BF16 network never has to resolve the small
           step-to-step change of phi against phi itself; K t = rho / s holds
           for the target t below.
  edges    e_ij = [(x_j - x_i) / hbar, (y_j - y_i) / hbar, |x_j - x_i| / hbar],
           hbar = mean coarse edge length
  encoder  h_i = relu(W_e x_i + c_e)
  round r  p_i = A_r h_i,  q_i = B_r h_i
           m_ij = relu(p_i + q_j + C_r e_ij + d_r)
           a_i = (1 / deg_i) sum_{j in N(i)} m_ij
           h_i <- h_i + relu(U_r [h_i; a_i] + v_r)
  decoder  y_i = w . h_i + c
  guess    g_i = q_i + s y_i
  loss     L = (1/N) sum_i (y_i - t_i)^2 / max(1, (1/N) sum_i t_i^2),
           t_i = (phi^{n+1}_i - q_i) / s; the per-sample normaliser bounds
           the weight of steps whose history is dominated by the solver
           noise of the previous solves (then e is tiny and t large)
Flat parameter order: W_e (H x 5), c_e (H), then per round A (H x H), B (H x H),
C (H x 3), d (H), U (H x 2H), v (H), then w (H), c (1); matrices row-major
(output x input).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

H = 32
ROUNDS = 3
NFEAT = 5
EFEAT = 3


def layout():
    """[(name, shape)] in flat order."""
    out = [("We", (H, NFEAT)), ("ce", (H,))]
    for r in range(ROUNDS):
        out += [(f"A{r}", (H, H)), (f"B{r}", (H, H)), (f"C{r}", (H, EFEAT)), (f"d{r}", (H,)),
                (f"U{r}", (H, 2 * H)), (f"v{r}", (H,))]
    out += [("w", (H,)), ("c", (1,))]
    return out


def n_params():
    return int(sum(np.prod(s) for _, s in layout()))


def unpack(theta):
    """Views of the flat parameter vector by name."""
    p, off = {}, 0
    for name, shape in layout():
        k = int(np.prod(shape))
        p[name] = theta[off:off + k].reshape(shape)
        off += k
    return p


def init_params(seed=0):
    """Uniform fan-in initialisation; the residual updates and the decoder
    start small so that the first guesses stay close to phi^n."""
    rng = np.random.default_rng(seed)
    theta = np.zeros(n_params())
    p = unpack(theta)
    for name, shape in layout():
        if len(shape) == 2:
            lim = np.sqrt(6.0 / shape[1])
            if name.startswith("U"):
                lim *= 0.1
            p[name][...] = rng.uniform(-lim, lim, size=shape)
    p["w"][...] = rng.uniform(-0.01, 0.01, size=H)
    return theta


class Graph:
    """Directed edges (i -> j) of the coarse node graph, grouped by i with j
    ascending, their features, and the solver's coarse operator (K with the
    rows and columns of `natural` nodes, where phi = 0, replaced by
    identity)."""

    def __init__(self, xy, K, natural=None):
        A = K.tocsr()
        A.sort_indices()
        if natural is not None and np.any(natural):
            keep = sp.diags((~np.asarray(natural, bool)).astype(np.float64))
            self.op = (keep @ A @ keep + sp.diags(np.asarray(natural, np.float64))).tocsr()
        else:
            self.op = A
        n = A.shape[0]
        rows = np.repeat(np.arange(n), np.diff(A.indptr))
        keep = rows != A.indices
        self.n = n
        self.src = rows[keep]
        self.dst = A.indices[keep]
        self.deg = np.bincount(self.src, minlength=n).astype(np.float64)
        d = xy[self.dst] - xy[self.src]
        length = np.hypot(d[:, 0], d[:, 1])
        self.hbar = float(length.mean())
        self.e = np.stack([d[:, 0], d[:, 1], length], axis=1) / self.hbar


def rms(v):
    return float(np.sqrt(np.mean(v * v)))


def features(g: Graph, b, hist):
    """Node inputs [N, 5], the extrapolation q and the scale s (hist: phi^n,
    ..., phi^{n-3})."""
    b = np.asarray(b, np.float64)
    p0, p1, p2, p3 = [np.asarray(h, np.float64) for h in hist[:4]]
    q = 3.0 * p0 - 3.0 * p1 + p2
    e = p0 - 3.0 * p1 + 3.0 * p2 - p3
    d1 = p0 - p1
    d2 = p0 - 2.0 * p1 + p2
    sb = rms(b) or 1.0
    s = max(rms(e), 1e-12 * rms(p0)) or sb / g.hbar ** 2
    s1 = rms(d1) or 1.0
    s2 = rms(d2) or 1.0
    rho = b - g.op @ q
    X = np.stack([b / sb, rho / s, e / s, d1 / s1, d2 / s2], axis=1)
    return X, q, s


def relu(z):
    return np.maximum(z, 0.0)


def forward(theta, g: Graph, X):
    """Output y [N] and the cache of every intermediate."""
    p = unpack(theta)
    cache = {"X": X}
    z0 = X @ p["We"].T + p["ce"]
    h = relu(z0)
    cache["z0"] = z0
    for r in range(ROUNDS):
        P = h @ p[f"A{r}"].T
        Q = h @ p[f"B{r}"].T
        S = P[g.src] + Q[g.dst] + g.e @ p[f"C{r}"].T + p[f"d{r}"]
        M = relu(S)
        a = np.zeros_like(h)
        np.add.at(a, g.src, M)
        a = a / g.deg[:, None]
        Z = np.concatenate([h, a], axis=1) @ p[f"U{r}"].T + p[f"v{r}"]
        cache[r] = (h, S, a, Z)
        h = h + relu(Z)
    cache["h"] = h
    y = h @ p["w"] + p["c"][0]
    return y, cache


def loss(theta, g, X, t):
    y, _ = forward(theta, g, X)
    return float(np.mean((y - t) ** 2) / max(1.0, np.mean(t * t)))


def backward(theta, g: Graph, cache, dy):
    """Gradient of sum_i dy_i y_i with respect to theta (flat)."""
    p = unpack(theta)
    grad = np.zeros_like(theta)
    G = unpack(grad)
    h = cache["h"]
    G["w"][...] = dy @ h
    G["c"][0] = dy.sum()
    dh = np.outer(dy, p["w"])
    for r in reversed(range(ROUNDS)):
        h_in, S, a, Z = cache[r]
        dZ = dh * (Z > 0)
        G[f"U{r}"][...] = dZ.T @ np.concatenate([h_in, a], axis=1)
        G[f"v{r}"][...] = dZ.sum(axis=0)
        dha = dZ @ p[f"U{r}"]
        dh_in = dh + dha[:, :H]
        da = dha[:, H:]
        dM = (da / g.deg[:, None])[g.src]
        dS = dM * (S > 0)
        G[f"C{r}"][...] = dS.T @ g.e
        G[f"d{r}"][...] = dS.sum(axis=0)
        dP = np.zeros_like(h_in)
        np.add.at(dP, g.src, dS)
        dQ = np.zeros_like(h_in)
        np.add.at(dQ, g.dst, dS)
        G[f"A{r}"][...] = dP.T @ h_in
        G[f"B{r}"][...] = dQ.T @ h_in
        dh = dh_in + dP @ p[f"A{r}"] + dQ @ p[f"B{r}"]
    dz0 = dh * (cache["z0"] > 0)
    G["We"][...] = dz0.T @ cache["X"]
    G["ce"][...] = dz0.sum(axis=0)
    return grad


def loss_grad(theta, g, X, t):
    """Loss and its gradient (normalised mean squared error on the correction)."""
    y, cache = forward(theta, g, X)
    n = y.shape[0]
    w = 1.0 / max(1.0, float(np.mean(t * t)))
    L = float(np.mean((y - t) ** 2)) * w
    return L, backward(theta, g, cache, 2.0 * w * (y - t) / n)


def adam_step(theta, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba) in place; step counts from 1."""
    m[...] = b1 * m + (1 - b1) * grad
    v[...] = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    theta[...] = theta - lr * mh / (np.sqrt(vh) + eps)


def target(q, s, phi_next):
    """Normalised training target of a solved phi^{n+1}."""
    return (np.asarray(phi_next, np.float64) - q) / s


def guess(theta, g, b, hist):
    X, q, s = features(g, b, hist)
    y, _ = forward(theta, g, X)
    return q + s * y
