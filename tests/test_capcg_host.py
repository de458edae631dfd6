"""Host checks of the tiling behind the s-step coarse PCG (no GPU): the
library's planner cuts the coarse nodes into tiles that own at most 512 nodes
each and whose depth-4 graph neighbourhoods hold at most 1024 nodes; the
checks recompute ownership and neighbourhood sizes with scipy's graph search,
independently of the planner.  Also the argument checks of the solver
option."""
import os

import numpy as np
import pytest
import scipy.sparse as sp

from workloads import unit_square, channel_cylinder, disc, NATURAL

S, OWN_MAX, EXT_MAX, ELL_MAX = 4, 512, 1024, 7680


@pytest.fixture(scope="module")
def N():
    from paper_1812_00185_amd import _native as N

    if not os.path.exists(N.LIB_PATH):
        from paper_1812_00185_amd.build import build

        build()
    N.load()
    return N


MESHES = {
    "square_9": lambda: unit_square(9),
    "square_natural_33": lambda: unit_square(33, tags={"left": NATURAL}),
    "square_257": lambda: unit_square(257),
    "disc": lambda: disc(30, 200, seed=3),
    "channel": lambda: channel_cylinder(0.02),
}


def graph(mesh):
    """CSR node graph of the mesh (every triangle edge, both directions, and
    the diagonal first in each row: the library's convention)."""
    tri = np.asarray(mesh["tri"], np.int64)
    n = mesh["xy"].shape[0]
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    A = sp.coo_matrix((np.ones(2 * len(e)), (np.r_[e[:, 0], e[:, 1]], np.r_[e[:, 1], e[:, 0]])),
                      shape=(n, n)).tocsr()
    A.sort_indices()
    rowptr, col = [0], []
    for i in range(n):
        col += [i] + list(A.indices[A.indptr[i]:A.indptr[i + 1]])
        rowptr.append(len(col))
    return np.array(rowptr, np.int32), np.array(col, np.int32), mesh["xy"], A


def depth_sizes(A, own_sets, s):
    """Nodes within graph distance s of each own set (boolean matrix powers)."""
    A = (A + sp.eye(A.shape[0])).astype(np.int8).tocsr()
    out = []
    for own in own_sets:
        v = np.zeros(A.shape[0], bool)
        v[own] = True
        for _ in range(s):
            v = v | (A @ v.astype(np.int8) > 0)
        out.append(int(v.sum()))
    return out


@pytest.mark.parametrize("name", sorted(MESHES))
def test_tiles_cover_and_fit(N, name):
    rowptr, col, xy, K = graph(MESHES[name]())
    n = rowptr.size - 1
    perm, own_off, info = N.ca_plan_host(rowptr, col, xy)
    print(f"[plan] {name}: n={n} {info}", flush=True)
    assert np.array_equal(np.sort(perm), np.arange(n))
    assert own_off[0] == 0 and own_off[-1] == n and np.all(np.diff(own_off) >= 1)
    sizes = np.diff(own_off)
    assert sizes.max() == info["max_own"] <= OWN_MAX
    assert info["ntiles"] == sizes.size >= -(-n // OWN_MAX)
    own_sets = [perm[own_off[t]:own_off[t + 1]] for t in range(info["ntiles"])]
    ext = depth_sizes(K, own_sets, S)
    assert max(ext) == info["max_ext"] <= EXT_MAX
    rows = depth_sizes(K, own_sets, S - 1)
    assert max(rows) * info["width"] <= ELL_MAX
    assert all(e >= o.size for e, o in zip(ext, own_sets))
    assert info["width"] == int(np.diff(rowptr).max())
    # each tile's own nodes in ascending node order
    assert all(np.all(np.diff(o) > 0) for o in own_sets)


def test_square_257_tiles_are_compact(N):
    """On the 257 x 257 pressure mesh the bisection gives tiles of about
    512 nodes whose neighbourhoods are close to those of square patches."""
    rowptr, col, xy, K = graph(unit_square(257))
    perm, own_off, info = N.ca_plan_host(rowptr, col, xy)
    assert info["ntiles"] == -(-66049 // OWN_MAX)
    # a square patch of 512 nodes (22.6 x 22.6) grows to about 31 x 31 = 961
    assert info["max_ext"] <= 1100


def test_planner_rejects_bad_graphs(N):
    rowptr, col, xy, _ = graph(unit_square(5))
    bad = col.copy()
    bad[3] = rowptr.size + 7
    with pytest.raises(N.CGPError):
        N.ca_plan_host(rowptr, bad, xy)
    empty_row = rowptr.copy()
    empty_row[1] = 0
    with pytest.raises(N.CGPError):
        N.ca_plan_host(empty_row, col, xy)
    nan_xy = np.array(xy, np.float64)
    nan_xy[4, 1] = np.nan
    with pytest.raises(N.CGPError):
        N.ca_plan_host(rowptr, col, nan_xy)


def test_option_requires_fp64():
    from paper_1812_00185_amd import CGP
    from paper_1812_00185_amd._native import CGPError

    with pytest.raises(CGPError):
        CGP(unit_square(9), 1, 1e-3, 1e-2, precision="mixed", precond="jacobi_s4", device="cpu")
    g = CGP(unit_square(33), 1, 1e-3, 1e-2, precond="jacobi_s4", device="cpu")
    assert g.sizes.workspace_bytes > 0
