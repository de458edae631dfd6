"""Pins of the oracle's P1 element matrices and assembled operators against
closed forms, brute-force quadrature and exact identities (Sect. 2.1, Eqs. 17-20)."""
import numpy as np
import pytest

from oracle import fem
from workloads import unit_square, disc, channel_cylinder


def _quad_points(xy3, n=4):
    """Brute-force quadrature on a triangle: split it into n^2 congruent
    sub-triangles and apply the edge-midpoint rule (exact for quadratics) on
    each, so every integrand below (at most quadratic) is integrated exactly."""
    a, b, c = xy3
    area = 0.5 * abs((b[0] - a[0]) * (c[1] - a[1]) - (c[0] - a[0]) * (b[1] - a[1]))
    subs = []
    for i in range(n):
        for j in range(n - i):
            subs.append([(i, j), (i + 1, j), (i, j + 1)])
            if i + j < n - 1:
                subs.append([(i + 1, j), (i + 1, j + 1), (i, j + 1)])
    pts = []
    for s in subs:
        s = np.array(s, float) / n
        for k in range(3):
            pts.append(0.5 * (s[k] + s[(k + 1) % 3]))
    s = np.array(pts)
    w = np.full(len(s), area / len(s))
    xy = a + s[:, 0:1] * (b - a) + s[:, 1:2] * (c - a)
    lam = np.stack([1 - s[:, 0] - s[:, 1], s[:, 0], s[:, 1]], 1)   # barycentric = shape functions
    return xy, lam, w


TRIS = [
    np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]),
    np.array([[0.3, -0.2], [1.7, 0.4], [0.1, 1.3]]),
    np.array([[2.0, 1.0], [2.5, 1.1], [2.2, 1.9]]),
]


def test_reference_triangle_closed_forms():
    """Textbook values on the reference triangle (0,0),(1,0),(0,1)."""
    xy = TRIS[0]
    tri = np.array([[0, 1, 2]])
    area, b, c = fem.element_geometry(xy, tri)
    assert area[0] == 0.5
    M = fem.element_mass(area)[0]
    np.testing.assert_allclose(M, np.array([[2, 1, 1], [1, 2, 1], [1, 1, 2]]) / 24.0, rtol=0, atol=1e-17)
    K = fem.element_stiffness(area, b, c)[0]
    np.testing.assert_allclose(K, [[1.0, -0.5, -0.5], [-0.5, 0.5, 0.0], [-0.5, 0.0, 0.5]], atol=1e-16)
    dx, dy = fem.element_divergence(b, c)
    # grad psi = (-1,-1), (1,0), (0,1); int psi_i = 1/6
    np.testing.assert_allclose(dx[0], np.tile([-1, 1, 0], (3, 1)) / 6.0, atol=1e-17)
    np.testing.assert_allclose(dy[0], np.tile([-1, 0, 1], (3, 1)) / 6.0, atol=1e-17)


@pytest.mark.parametrize("t", range(len(TRIS)))
def test_element_matrices_vs_quadrature(t):
    xy = TRIS[t]
    tri = np.array([[0, 1, 2]])
    area, b, c = fem.element_geometry(xy, tri)
    q, lam, w = _quad_points(xy)
    grad = np.stack([b[0], c[0]], 1) / (2 * area[0])                # [3,2]
    M_q = np.einsum("qi,qj,q->ij", lam, lam, w)
    np.testing.assert_allclose(fem.element_mass(area)[0], M_q, rtol=1e-12)
    K_q = (grad @ grad.T) * area[0]
    np.testing.assert_allclose(fem.element_stiffness(area, b, c)[0], K_q, rtol=1e-12)
    dx, dy = fem.element_divergence(b, c)
    np.testing.assert_allclose(dx[0], np.einsum("qi,q->i", lam, w)[:, None] * grad[None, :, 0], rtol=1e-12)
    np.testing.assert_allclose(dy[0], np.einsum("qi,q->i", lam, w)[:, None] * grad[None, :, 1], rtol=1e-12)
    rng = np.random.default_rng(t)
    wx, wy = rng.normal(size=3), rng.normal(size=3)
    N = fem.element_convection(area, b, c, wx[None], wy[None])[0]
    whx, why = lam @ wx, lam @ wy                                     # w_h at quadrature points
    N_q = np.einsum("qi,q,qj->ij", lam, w, whx[:, None] * grad[None, :, 0] + why[:, None] * grad[None, :, 1])
    np.testing.assert_allclose(N, N_q, rtol=1e-11, atol=1e-14)


MESHES = {
    "square9": lambda: unit_square(9),
    "disc": lambda: disc(24, 60, seed=3),
}


@pytest.mark.parametrize("name", list(MESHES))
def test_assembly_invariants(name):
    m = MESHES[name]()
    op = fem.Operators(m)
    n = op.n
    one = np.ones(n)
    # K annihilates constants; M integrates to the domain area
    assert np.abs(op.K @ one).max() < 1e-12
    assert abs(one @ (op.M @ one) - op.area.sum()) < 1e-13
    assert abs(op.lumped.sum() - op.area.sum()) < 1e-13
    # symmetry and P1 mass identity M_ii = sum_{j != i} M_ij
    assert abs(op.K - op.K.T).max() < 1e-14
    offd = (op.M @ one) - op.M.diagonal()
    np.testing.assert_allclose(op.M.diagonal(), offd, rtol=1e-13)
    # G = -D^T
    assert abs(op.Gx + op.Dx.T).max() == 0.0
    # 1^T D U equals the boundary flux of the P1 trace (trapezoid rule per edge)
    rng = np.random.default_rng(0)
    U = rng.normal(size=(2, n))
    flux = 0.0
    xy = op.xy
    for (p, q) in m["bedge"]:
        t = xy[q] - xy[p]
        nrm = np.array([t[1], -t[0]])            # outward for a ccw boundary
        flux += 0.5 * ((U[:, p] + U[:, q]) @ nrm)
    assert abs(one @ op.div(U) - flux) < 1e-11


def _interior(m):
    b = np.zeros(m["xy"].shape[0], bool)
    b[m["bedge"].ravel()] = True
    return ~b


@pytest.mark.parametrize("name", list(MESHES))
def test_linear_fields_exact(name):
    """Exactness on linear data: gradient, divergence, Laplacian, convection."""
    m = MESHES[name]()
    op = fem.Operators(m)
    x, y = op.xy[:, 0], op.xy[:, 1]
    inner = _interior(m)
    p = 0.3 + 1.7 * x - 0.9 * y
    gp = op.grad(p)
    np.testing.assert_allclose(gp[0][inner], 1.7 * op.lumped[inner], rtol=1e-12)
    np.testing.assert_allclose(gp[1][inner], -0.9 * op.lumped[inner], rtol=1e-12)
    # divergence-free linear velocity
    u = np.stack([0.2 + 0.5 * x + 1.3 * y, -0.7 - 0.4 * x - 0.5 * y])
    assert np.abs(op.div(u)).max() < 1e-14
    # Laplacian of a linear function vanishes at interior nodes
    assert np.abs((op.K @ p)[inner]).max() < 1e-12
    # convection of a linear field by a constant velocity
    wx, wy = np.full_like(x, 0.6), np.full_like(x, -1.1)
    N = op.convection(wx, wy)
    np.testing.assert_allclose(N @ p, (0.6 * 1.7 + 1.1 * 0.9) * op.lumped, rtol=1e-12, atol=1e-15)


def test_channel_mesh_valid():
    m = channel_cylinder(h=0.03)
    op = fem.Operators(m)
    assert np.all(op.area > 0)
    assert abs(op.area.sum() - (2.2 * 0.41 - np.pi * 0.05 ** 2)) < 2e-3


@pytest.mark.parametrize("name", list(MESHES) + ["channel"])
def test_wathen_mass_matrix_spectrum(name):
    """Wathen's bound for P1 triangles: the eigenvalues of D^-1 M (D = diag M)
    lie in [1/2, 2], also for the principal submatrix left after removing
    boundary rows and columns (Rayleigh quotients over a subspace)."""
    m = MESHES[name]() if name in MESHES else channel_cylinder(h=0.06)
    op = fem.Operators(m)
    M = op.M.toarray()
    d = np.diag(M)
    lam = np.linalg.eigvalsh(M / np.sqrt(np.outer(d, d)))
    assert lam.min() >= 0.5 - 1e-12 and lam.max() <= 2.0 + 1e-12
    inner = _interior(m)
    Mi = M[np.ix_(inner, inner)]
    di = np.diag(Mi)
    lam = np.linalg.eigvalsh(Mi / np.sqrt(np.outer(di, di)))
    assert lam.min() >= 0.5 - 1e-12 and lam.max() <= 2.0 + 1e-12
