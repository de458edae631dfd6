"""Nested mesh hierarchy and the transfer operators (Sect. 2.2).

Oracle (test infrastructure only).

* Refinement: every triangle (a, b, c) is split into four by its edge
  midpoints, so a mesh with N elements refined k times has 4^k N elements and
  the spaces are nested, V_1 c V_2 c V_3 c V_4.
* Node numbering convention (shared with the library's C-ABI as an interface,
  not as code).  Each refinement keeps the parent level's nodes and appends
  the midpoint of every edge in first-encounter order over (triangle, local
  edge (0,1), (1,2), (2,0)); children of (a, b, c) with midpoints m_ab, m_bc,
  m_ca are (a, m_ab, m_ca), (m_ab, b, m_bc), (m_ca, m_bc, c), (m_ab, m_bc,
  m_ca), in that order; boundary edge e = (p, q) becomes (p, m), (m, q) with
  e's tag.  The finest mesh is then renumbered: the coarse nodes keep 0..N_c-1
  and the new nodes follow, stably sorted by their owner, the coarse
  triangle that is the ancestor of the triangle that first created them, so
  that the nodes of one coarse triangle are contiguous (the library's
  neighbour gathers stay local in memory).  Intermediate levels keep the
  level-by-level numbering.
* Restriction is pure injection: the coarse value at a coarse node is the fine
  value at the coincident fine node.  With the numbering above that node has
  the same index.
* Prolongation is linear interpolation: a new midpoint node takes the mean of
  its two parent-edge end values.  Applied level by level, k times.
* No boundary snapping (the paper's nested spaces need none).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from workloads.meshes import DIRICHLET, NATURAL


def refine_once(xy, tri, bedge, btag):
    """One level of 4:1 refinement.  Returns (xy, tri, bedge, btag, ends,
    creator), where ends[m - n_parent] = (a, b) are the parent edge ends of
    new node m and creator[m - n_parent] the parent triangle that first
    encountered that edge."""
    xy = np.asarray(xy, np.float64)
    tri = np.asarray(tri, np.int64)
    bedge = np.asarray(bedge, np.int64)
    n = xy.shape[0]
    t = tri.shape[0]
    loc = np.stack([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]], axis=1).reshape(-1, 2)
    lo = loc.min(axis=1)
    hi = loc.max(axis=1)
    key = lo * n + hi
    uniq, first, inv = np.unique(key, return_index=True, return_inverse=True)
    # number the distinct edges by their first appearance in (triangle, local edge) order
    order = np.argsort(first, kind="stable")
    rank = np.empty_like(order)
    rank[order] = np.arange(order.size)
    mid = (n + rank[inv]).reshape(t, 3)
    ends = np.stack([loc[first[order], 0], loc[first[order], 1]], axis=1)
    new_xy = np.concatenate([xy, 0.5 * (xy[ends[:, 0]] + xy[ends[:, 1]])])

    a, b, c = tri[:, 0], tri[:, 1], tri[:, 2]
    mab, mbc, mca = mid[:, 0], mid[:, 1], mid[:, 2]
    kids = np.stack([
        np.stack([a, mab, mca], 1),
        np.stack([mab, b, mbc], 1),
        np.stack([mca, mbc, c], 1),
        np.stack([mab, mbc, mca], 1),
    ], axis=1).reshape(-1, 3)

    bkey = bedge.min(axis=1) * n + bedge.max(axis=1)
    pos = np.searchsorted(uniq, bkey)
    if np.any(pos >= uniq.size) or np.any(uniq[np.minimum(pos, uniq.size - 1)] != bkey):
        raise ValueError("boundary edge is not an edge of the mesh")
    bm = n + rank[pos]
    new_bedge = np.stack([np.stack([bedge[:, 0], bm], 1),
                          np.stack([bm, bedge[:, 1]], 1)], axis=1).reshape(-1, 2)
    new_btag = np.repeat(np.asarray(btag), 2)
    creator = first[order] // 3
    return new_xy, kids, new_bedge, new_btag, ends, creator


class Hierarchy:
    """Coarse mesh plus k uniform refinements."""

    def __init__(self, coarse: dict, levels: int):
        if not 0 <= levels <= 3:
            raise ValueError("levels must be 0..3")
        self.levels = levels
        xy, tri = np.asarray(coarse["xy"], np.float64), np.asarray(coarse["tri"], np.int64)
        bedge, btag = np.asarray(coarse["bedge"], np.int64), np.asarray(coarse["btag"], np.int64)
        self.meshes = [dict(xy=xy, tri=tri, bedge=bedge, btag=btag)]
        self.ends = []          # ends[l]: parent pairs of the nodes added at refinement l+1
        owner = np.full(xy.shape[0], -1, np.int64)   # coarse triangle that created a node
        for l in range(levels):
            xy, tri, bedge, btag, ends, creator = refine_once(xy, tri, bedge, btag)
            # level-l triangle t descends from coarse triangle t // 4^l
            owner = np.concatenate([owner, creator >> (2 * l)])
            self.meshes.append(dict(xy=xy, tri=tri, bedge=bedge, btag=btag))
            self.ends.append(ends)
        nc = self.meshes[0]["xy"].shape[0]
        nf = xy.shape[0]
        # canonical fine numbering: coarse nodes first, then the new nodes
        # stably sorted by owner; canon[levelwise id] = canonical id
        self.canon = np.arange(nf)
        if levels:
            order = nc + np.argsort(owner[nc:], kind="stable")
            self.canon[order] = np.arange(nc, nf)
            self.owner = np.empty(nf, np.int64)
            self.owner[self.canon] = owner
            fine = self.meshes[-1]
            fxy = np.empty_like(fine["xy"])
            fxy[self.canon] = fine["xy"]
            self.meshes[-1] = dict(xy=fxy, tri=self.canon[fine["tri"]],
                                   bedge=self.canon[fine["bedge"]], btag=fine["btag"])
        else:
            self.owner = owner

    @property
    def coarse(self):
        return self.meshes[0]

    @property
    def fine(self):
        return self.meshes[-1]

    def restrict(self, uf):
        """Injection R: fine nodal values -> coarse nodal values (Eq. 22)."""
        nc = self.coarse["xy"].shape[0]
        return np.asarray(uf)[..., :nc].copy()

    def prolong(self, phic):
        """Linear prolongation P applied k times (Eq. 24), level by level in
        the level-wise numbering, then put in the canonical fine order."""
        phi = np.asarray(phic, np.float64).copy()
        for ends in self.ends:
            phi = np.concatenate([phi, 0.5 * (phi[ends[:, 0]] + phi[ends[:, 1]])])
        out = np.empty_like(phi)
        out[self.canon] = phi
        return out

    def prolongation_matrix(self):
        """P = P_k ... P_1 as an explicit N_f x N_c sparse matrix: each level
        keeps the parent nodes and adds every midpoint with weights 1/2, 1/2."""
        nc = self.coarse["xy"].shape[0]
        P = sp.identity(nc, format="csr")
        for ends in self.ends:
            n, m = P.shape[0], ends.shape[0]
            rows = np.concatenate([np.arange(n), n + np.arange(m), n + np.arange(m)])
            cols = np.concatenate([np.arange(n), ends[:, 0], ends[:, 1]])
            vals = np.concatenate([np.ones(n), np.full(m, 0.5), np.full(m, 0.5)])
            Pl = sp.coo_matrix((vals, (rows, cols)), shape=(n + m, n)).tocsr()
            P = (Pl @ P).tocsr()
        inv = np.empty_like(self.canon)
        inv[self.canon] = np.arange(self.canon.size)
        return P[inv].tocsr()


def boundary_nodes(mesh: dict, tag: int) -> np.ndarray:
    """Sorted nodes lying on a boundary edge with the given tag."""
    sel = mesh["btag"] == tag
    return np.unique(mesh["bedge"][sel].ravel())


def dirichlet_nodes(mesh):
    """Velocity-Dirichlet set: every node on a Dirichlet edge (walls win at
    junctions with the outflow)."""
    return boundary_nodes(mesh, DIRICHLET)


def natural_nodes(mesh):
    """phi = 0 set (Eq. 14): every node on a natural (traction-free) edge."""
    return boundary_nodes(mesh, NATURAL)
