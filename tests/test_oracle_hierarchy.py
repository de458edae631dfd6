"""Pins of the oracle's mesh hierarchy and transfer operators (Sect. 2.2)."""
import json
import os

import numpy as np
import pytest

from oracle import fem
from oracle.hierarchy import Hierarchy, dirichlet_nodes, natural_nodes
from workloads import unit_square, disc, channel_cylinder, NATURAL

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_fig1_node_element_counts():
    """A disc mesh with the paper's coarsest Poisson mesh size refines to the
    sizes printed in the caption of Fig. 1 (and Table 7's fine mesh)."""
    g = json.load(open(os.path.join(GOLDEN, "fig1_counts.json")))
    h = Hierarchy(disc(96, 1105, seed=0), 2)
    lv = g["levels"]
    assert h.meshes[0]["xy"].shape[0] == lv[0]["nodes"]
    assert h.meshes[0]["tri"].shape[0] == lv[0]["elements"]
    assert h.meshes[1]["xy"].shape[0] == lv[1]["nodes"]
    assert h.meshes[1]["tri"].shape[0] == lv[1]["elements"]
    assert h.meshes[2]["tri"].shape[0] == lv[2]["elements"]


def test_refined_square_is_structured_square():
    """4:1 refinement of the n x n right-triangle mesh gives the (2n-1) x (2n-1)
    mesh with the same diagonal orientation (same node set, same triangle set)."""
    h = Hierarchy(unit_square(5), 2)
    ref = unit_square(17)
    f = h.fine
    key = lambda xy: np.round(xy * 16).astype(int) @ np.array([1, 1000])
    kf, kr = key(f["xy"]), key(ref["xy"])
    assert sorted(kf) == sorted(kr)
    m = {k: i for i, k in enumerate(kr)}
    tf = {tuple(sorted(m[k] for k in kf[t])) for t in f["tri"]}
    tr = {tuple(sorted(t)) for t in ref["tri"]}
    assert tf == tr


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_refinement_geometry(levels):
    h = Hierarchy(disc(20, 30, seed=1), levels)
    c, f = fem.Operators(h.coarse), fem.Operators(h.fine)
    assert f.tri.shape[0] == 4 ** levels * c.tri.shape[0]
    assert np.all(f.area > 0)
    # children of coarse triangle t are fine triangles t*4^k ... (t+1)*4^k - 1
    np.testing.assert_allclose(f.area.reshape(-1, 4 ** levels).sum(1), c.area, rtol=1e-13)
    # node count V' = V + E per level
    for a, b in zip(h.meshes[:-1], h.meshes[1:]):
        e = {tuple(sorted(p)) for t in a["tri"] for p in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0]))}
        assert b["xy"].shape[0] == a["xy"].shape[0] + len(e)
    # coarse nodes keep their index and coordinates
    np.testing.assert_array_equal(f.xy[: c.n], c.xy)


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_transfer_operators(levels):
    h = Hierarchy(disc(20, 30, seed=2), levels)
    P = h.prolongation_matrix()
    nc = h.coarse["xy"].shape[0]
    rng = np.random.default_rng(levels)
    phic = rng.normal(size=nc)
    # R P = I (injection after prolongation), P 1 = 1
    np.testing.assert_array_equal(h.restrict(h.prolong(phic)), phic)
    np.testing.assert_allclose(h.prolong(np.ones(nc)), 1.0, rtol=0, atol=1e-15)
    # prolongation is exact on linear functions
    xc, xf = h.coarse["xy"], h.fine["xy"]
    lin = lambda xy: 0.7 - 1.3 * xy[:, 0] + 2.1 * xy[:, 1]
    np.testing.assert_allclose(h.prolong(lin(xc)), lin(xf), atol=1e-14)
    # matrix form equals the level-by-level form
    np.testing.assert_allclose(P @ phic, h.prolong(phic), atol=1e-15)
    # P's rows hold at most 3 nonzeros (the coarse triangle's vertices), dyadic weights
    assert np.diff(P.indptr).max() <= 3
    np.testing.assert_array_equal(P.data * 2 ** levels, np.round(P.data * 2 ** levels))


@pytest.mark.parametrize("levels", [1, 2])
def test_galerkin_identities(levels):
    """Nested P1 spaces: coarse operators equal the Galerkin products."""
    h = Hierarchy(disc(24, 40, seed=4), levels)
    C, F = fem.Operators(h.coarse), fem.Operators(h.fine)
    P = h.prolongation_matrix()
    np.testing.assert_allclose((P.T @ F.K @ P).toarray(), C.K.toarray(), atol=1e-12)
    np.testing.assert_allclose((P.T @ F.M @ P).toarray(), C.M.toarray(), atol=1e-15)
    np.testing.assert_allclose((P.T @ F.Dx @ P).toarray(), C.Dx.toarray(), atol=1e-14)
    np.testing.assert_allclose((P.T @ F.Dy @ P).toarray(), C.Dy.toarray(), atol=1e-14)


def test_boundary_sets():
    m = unit_square(5, tags={"left": NATURAL})
    h = Hierarchy(m, 1)
    d = dirichlet_nodes(h.fine)
    n = natural_nodes(h.fine)
    xy = h.fine["xy"]
    # every boundary node is in one of the sets; corners on the left side are in both
    on_b = (xy[:, 0] == 0) | (xy[:, 0] == 1) | (xy[:, 1] == 0) | (xy[:, 1] == 1)
    assert set(np.where(on_b)[0]) == set(d) | set(n)
    assert set(n) == set(np.where(xy[:, 0] == 0)[0])
    both = set(d) & set(n)
    assert {tuple(xy[i]) for i in both} == {(0.0, 0.0), (0.0, 1.0)}


def test_channel_boundary_tags_inherited():
    h = Hierarchy(channel_cylinder(h=0.05), 2)
    f = h.fine
    nat = natural_nodes(f)
    assert np.all(np.isclose(f["xy"][nat, 0], 2.2))
    assert f["bedge"].shape[0] == 4 * h.coarse["bedge"].shape[0]


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_fine_numbering_groups_nodes_by_owner_coarse_triangle(levels):
    """Canonical fine order: coarse nodes first, then the new nodes grouped by
    the coarse triangle that created them; every new node lies in that
    triangle (closed), and the fine mesh is the same point and triangle set as
    the level-by-level refinement."""
    m = disc(20, 30, seed=6)
    h = Hierarchy(m, levels)
    nc = h.coarse["xy"].shape[0]
    own = h.owner[nc:]
    assert np.all(np.diff(own) >= 0) and own.min() >= 0
    xy = h.fine["xy"][nc:]
    t = h.coarse["tri"][own]
    A, B, C = (h.coarse["xy"][t[:, k]] for k in range(3))
    det = (B[:, 0] - A[:, 0]) * (C[:, 1] - A[:, 1]) - (C[:, 0] - A[:, 0]) * (B[:, 1] - A[:, 1])
    l1 = ((xy[:, 0] - A[:, 0]) * (C[:, 1] - A[:, 1]) - (C[:, 0] - A[:, 0]) * (xy[:, 1] - A[:, 1])) / det
    l2 = ((B[:, 0] - A[:, 0]) * (xy[:, 1] - A[:, 1]) - (xy[:, 0] - A[:, 0]) * (B[:, 1] - A[:, 1])) / det
    tol = 1e-12
    assert np.all(l1 >= -tol) and np.all(l2 >= -tol) and np.all(l1 + l2 <= 1 + tol)
    # distinct points; triangles keep their order (those of coarse triangle T
    # are T*4^k ... (T+1)*4^k - 1) and orientation
    key = np.round(h.fine["xy"] * 2 ** 30).astype(np.int64)
    assert len({tuple(k) for k in key}) == h.fine["xy"].shape[0]
    F, c = fem.Operators(h.fine), fem.Operators(h.coarse)
    assert np.all(F.area > 0)
    np.testing.assert_allclose(F.area.reshape(-1, 4 ** levels).sum(1), c.area, rtol=1e-13)
