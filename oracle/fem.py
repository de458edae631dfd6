"""P1/P1 Galerkin matrices (Sect. 2.1, Eqs. 17-20).

Oracle (test infrastructure only).  Each global matrix is the sum of element
matrices written out from their definitions on a triangle e with
counter-clockwise vertices (x_i, y_i), i = 0, 1, 2:

  |e| = area,  grad psi_i = (b_i, c_i) / (2|e|),
  b_i = y_j - y_k,  c_i = x_k - x_j  for (i, j, k) a cyclic permutation,
  int_e psi_i psi_j = |e| (1 + delta_ij) / 12.

  M (mass)         M_ij = int psi_i psi_j
  K (stiffness)    K_ij = int grad psi_i . grad psi_j   (L_v = nu K, L_p = -K)
  D (divergence)   (D U)_i = int psi_i div u_h          (two blocks Dx, Dy)
  G (gradient)     G = -D^T, i.e. (G P)_i = -int p_h div(psi_i)
  N(w) (convection) N_ij = int psi_i (w_h . grad psi_j)
  B (boundary mass) B_ij = int_{Gamma_N} psi_i psi_j ds  (natural edges only;
                    on an edge of length L: L/3 on the diagonal, L/6 off it)

Readings: L_p is taken as -K so that Eq. 18 reads K Phi = -(3/(2 dt)) D U
(the weak form of Eq. 12 with the natural condition Eq. 13); D is the strong
divergence and G its negative transpose, which makes the outflow the
traction-free (do-nothing) condition of Eq. 11.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from workloads.meshes import NATURAL


def element_geometry(xy, tri):
    """Per-element area and gradient coefficients b, c ([T,3] each)."""
    x = xy[tri, 0]
    y = xy[tri, 1]
    b = np.stack([y[:, 1] - y[:, 2], y[:, 2] - y[:, 0], y[:, 0] - y[:, 1]], axis=1)
    c = np.stack([x[:, 2] - x[:, 1], x[:, 0] - x[:, 2], x[:, 1] - x[:, 0]], axis=1)
    area = 0.5 * ((x[:, 1] - x[:, 0]) * (y[:, 2] - y[:, 0])
                  - (x[:, 2] - x[:, 0]) * (y[:, 1] - y[:, 0]))
    return area, b, c


def element_mass(area):
    """[T,3,3]: |e| (1 + delta_ij) / 12."""
    base = (np.ones((3, 3)) + np.eye(3)) / 12.0
    return area[:, None, None] * base[None]


def element_stiffness(area, b, c):
    """[T,3,3]: (b_i b_j + c_i c_j) / (4 |e|)."""
    return (b[:, :, None] * b[:, None, :] + c[:, :, None] * c[:, None, :]) / (4.0 * area[:, None, None])


def element_divergence(b, c):
    """([T,3,3], [T,3,3]): int psi_i d(psi_j)/dx = b_j / 6, same for y with c_j."""
    dx = np.repeat(b[:, None, :] / 6.0, 3, axis=1)
    dy = np.repeat(c[:, None, :] / 6.0, 3, axis=1)
    return dx, dy


def element_convection(area, b, c, wx, wy):
    """[T,3,3]: int psi_i (w_h . grad psi_j) with w_h the P1 interpolant of the
    nodal velocity (wx, wy) given per element vertex ([T,3] each).

    int psi_i w_h = sum_k w_k |e| (1 + delta_ik) / 12, and grad psi_j is
    constant, so N_ij = (b_j, c_j) . sum_k w_k (1 + delta_ik) / 24.
    """
    mass_w = (np.ones((3, 3)) + np.eye(3))        # (1 + delta_ik)
    sx = wx @ mass_w.T                             # sx[:, i] = sum_k (1+d_ik) wx_k
    sy = wy @ mass_w.T
    return (sx[:, :, None] * b[:, None, :] + sy[:, :, None] * c[:, None, :]) / 24.0


def edge_mass(xy, edges):
    """[E,2,2]: int_e psi_a psi_b ds on straight edges (a, b) of length L,
    L (1 + delta_ab) / 6 (the 1-D P1 mass matrix)."""
    d = xy[edges[:, 1]] - xy[edges[:, 0]]
    length = np.hypot(d[:, 0], d[:, 1])
    base = (np.ones((2, 2)) + np.eye(2)) / 6.0
    return length[:, None, None] * base[None]


def assemble_edges(edges, n, emat):
    """Sum edge matrices [E,2,2] into an n x n CSR matrix."""
    rows = np.repeat(edges, 2, axis=1).ravel()
    cols = np.tile(edges, (1, 2)).ravel()
    return sp.coo_matrix((emat.ravel(), (rows, cols)), shape=(n, n)).tocsr()


def assemble(tri, n, emat):
    """Sum element matrices [T,3,3] into an n x n CSR matrix."""
    rows = np.repeat(tri, 3, axis=1).ravel()
    cols = np.tile(tri, (1, 3)).ravel()
    return sp.coo_matrix((emat.ravel(), (rows, cols)), shape=(n, n)).tocsr()


class Operators:
    """All constant matrices of one mesh."""

    def __init__(self, mesh: dict):
        self.xy = np.asarray(mesh["xy"], np.float64)
        self.tri = np.asarray(mesh["tri"], np.int64)
        self.n = self.xy.shape[0]
        self.area, self.b, self.c = element_geometry(self.xy, self.tri)
        if np.any(self.area <= 0):
            raise ValueError("mesh has a clockwise or degenerate triangle")
        self.M = assemble(self.tri, self.n, element_mass(self.area))
        self.K = assemble(self.tri, self.n, element_stiffness(self.area, self.b, self.c))
        ex, ey = element_divergence(self.b, self.c)
        self.Dx = assemble(self.tri, self.n, ex)
        self.Dy = assemble(self.tri, self.n, ey)
        self.Gx = -self.Dx.T.tocsr()
        self.Gy = -self.Dy.T.tocsr()
        # boundary mass on the natural (traction) edges: the traction data
        # t_N of Eqs. 4, 8 and 11 enters the momentum right-hand side as B T
        bedge = np.asarray(mesh.get("bedge", np.zeros((0, 2))), np.int64).reshape(-1, 2)
        btag = np.asarray(mesh.get("btag", np.zeros(0)), np.int64)
        nat = bedge[btag == NATURAL]
        self.B = assemble_edges(nat, self.n, edge_mass(self.xy, nat))
        # lumped mass m_i = sum over incident elements of |e| / 3
        self.lumped = np.bincount(self.tri.ravel(), weights=np.repeat(self.area / 3.0, 3),
                                  minlength=self.n)

    def convection(self, wx, wy):
        """N(w) for nodal velocity w = (wx, wy)."""
        e = element_convection(self.area, self.b, self.c, wx[self.tri], wy[self.tri])
        return assemble(self.tri, self.n, e)

    def div(self, u):
        """D U for u of shape [2, n]."""
        return self.Dx @ u[0] + self.Dy @ u[1]

    def grad(self, p):
        """G P, shape [2, n]."""
        return np.stack([self.Gx @ p, self.Gy @ p])
