"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every entry point include/cgp.h declares, and its host set-up (mesh
validation, refinement, numbering, boundary sets) matches the oracle."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle.hierarchy import Hierarchy, dirichlet_nodes, natural_nodes
from workloads import unit_square, channel_cylinder, disc, NATURAL

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cgp.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1812_00185_amd import _native as N

    if not os.path.exists(N.LIB_PATH):
        from paper_1812_00185_amd.build import build

        build()
    return N.load()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cgp_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol(lib):
    from paper_1812_00185_amd import _native as N

    names = declared_functions()
    assert "cgp_project_step" in names and len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == {s[0] for s in N.SIGNATURES}


def _create(lib, mesh, levels, **kw):
    from paper_1812_00185_amd import _native as N

    xy = np.ascontiguousarray(mesh["xy"], np.float64)
    tri = np.ascontiguousarray(mesh["tri"], np.int32)
    be = np.ascontiguousarray(mesh["bedge"], np.int32)
    bt = np.ascontiguousarray(mesh["btag"], np.int32)
    m = N.Mesh(xy.shape[0], tri.shape[0], bt.shape[0],
               xy.ctypes.data_as(C.POINTER(C.c_double)), tri.ctypes.data_as(C.POINTER(C.c_int32)),
               be.ctypes.data_as(C.POINTER(C.c_int32)), bt.ctypes.data_as(C.POINTER(C.c_int32)))
    p = dict(chi=0, precision=0, restrict_mode=0, dt=1e-3, nu=1e-2, pcg_tol=1e-8, inner_tol=1e-5,
             mom_tol=1e-12, mass_tol=1e-12, max_iter=100, mom_max_iter=100, mass_max_iter=100,
             max_outer=5, mass_mode=0, coarse_precond=0, scheme=0)
    p.update(kw)
    prob = N.Problem(m, levels, p["chi"], p["precision"], p["restrict_mode"], p["dt"], p["nu"],
                     p["pcg_tol"], p["inner_tol"], p["mom_tol"], p["mass_tol"], p["max_iter"],
                     p["mom_max_iter"], p["mass_max_iter"], p["max_outer"], p["mass_mode"],
                     p["coarse_precond"], p["scheme"])
    ctx = C.c_void_p()
    rc = lib.cgp_create(C.byref(prob), C.byref(ctx))
    return rc, ctx


@pytest.mark.parametrize("name,mesh,k", [
    ("square", unit_square(9, tags={"left": NATURAL}), 2),
    ("disc", disc(30, 80, seed=1), 3),
    ("channel", channel_cylinder(0.05), 2),
    ("square_k0", unit_square(5), 0),
])
def test_host_hierarchy_matches_oracle(lib, name, mesh, k):
    from paper_1812_00185_amd import _native as N

    rc, ctx = _create(lib, mesh, k)
    assert rc == 0, lib.cgp_last_error()
    try:
        sz = N.Sizes()
        assert lib.cgp_query(ctx, C.byref(sz)) == 0
        h = Hierarchy(mesh, k)
        f = h.fine
        assert sz.n_fine == f["xy"].shape[0] and sz.n_fine_tris == f["tri"].shape[0]
        assert sz.n_coarse == mesh["xy"].shape[0]
        assert sz.n_natural_coarse == natural_nodes(h.coarse).size
        xy = np.empty(2 * sz.n_fine)
        assert lib.cgp_fine_nodes(ctx, xy.ctypes.data_as(C.POINTER(C.c_double))) == 0
        assert np.array_equal(xy.reshape(-1, 2), f["xy"])          # bit-exact numbering
        d = np.empty(sz.n_dirichlet, np.int32)
        assert lib.cgp_dirichlet_nodes(ctx, d.ctypes.data_as(C.POINTER(C.c_int32))) == 0
        assert np.array_equal(d, dirichlet_nodes(f))
        # CSR graph size: N + 2 E (each undirected edge twice)
        e = {tuple(sorted(p)) for t in f["tri"] for p in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0]))}
        assert sz.nnz_fine == sz.n_fine + 2 * len(e)
        assert sz.workspace_bytes > 8 * sz.nnz_fine
    finally:
        lib.cgp_destroy(ctx)


def test_structured_2049_sizes(lib):
    """The 2049 x 2049 workload: 4,198,401 nodes and 29,372,417 nonzeros."""
    from paper_1812_00185_amd import _native as N

    rc, ctx = _create(lib, unit_square(257), 3)
    assert rc == 0
    sz = N.Sizes()
    lib.cgp_query(ctx, C.byref(sz))
    lib.cgp_destroy(ctx)
    assert (sz.n_fine, sz.nnz_fine, sz.n_coarse, sz.nnz_coarse) == (4198401, 29372417, 66049, 460289)


def test_mesh_errors(lib):
    from paper_1812_00185_amd import _native as N

    base = unit_square(3)
    bad = {k: v.copy() for k, v in base.items()}
    bad["tri"][0] = bad["tri"][0][[0, 2, 1]]                      # clockwise
    assert _create(lib, bad, 1)[0] == N.CGP_ERR_MESH
    assert b"clockwise" in lib.cgp_last_error()
    dup = {k: v.copy() for k, v in base.items()}
    dup["tri"] = np.concatenate([dup["tri"], dup["tri"][:1]])     # duplicate triangle
    assert _create(lib, dup, 1)[0] == N.CGP_ERR_MESH
    miss = {k: v.copy() for k, v in base.items()}
    miss["bedge"], miss["btag"] = miss["bedge"][1:], miss["btag"][1:]   # untagged boundary edge
    assert _create(lib, miss, 1)[0] == N.CGP_ERR_MESH
    tag = {k: v.copy() for k, v in base.items()}
    tag["btag"][0] = 7
    assert _create(lib, tag, 1)[0] == N.CGP_ERR_MESH
    assert _create(lib, base, 4)[0] == N.CGP_ERR_INVALID
    assert _create(lib, base, 1, dt=0.0)[0] == N.CGP_ERR_INVALID
    assert _create(lib, base, 1, chi=2)[0] == N.CGP_ERR_INVALID
    assert _create(lib, base, 1, mass_mode=4)[0] == N.CGP_ERR_INVALID
    assert _create(lib, base, 1, scheme=2)[0] == N.CGP_ERR_INVALID
    assert _create(lib, base, 1, scheme=1, chi=1)[0] == N.CGP_ERR_INVALID
    assert b"rotational" in lib.cgp_last_error()
    rc, ctx = _create(lib, base, 1, scheme=1)
    assert rc == 0
    lib.cgp_destroy(ctx)
    for mode in (N.CGP_MASS_LUMPED_P, N.CGP_MASS_LUMPED):
        rc, ctx = _create(lib, base, 1, chi=1, mass_mode=mode)
        assert rc == 0
        lib.cgp_destroy(ctx)
    rc, ctx = _create(lib, base, 1)
    assert rc == 0
    # device calls before cgp_assemble are rejected without touching the GPU
    assert lib.cgp_restrict(ctx, None, None, None) == N.CGP_ERR_INVALID
    assert lib.cgp_assemble(ctx, None, 0, None, 0, None) == N.CGP_ERR_WORKSPACE
    # the page-locked host buffer is the caller's too: its size is reported,
    # and a missing one is rejected before any device work
    sz = N.Sizes()
    assert lib.cgp_query(ctx, C.byref(sz)) == 0 and sz.host_bytes >= 64
    assert lib.cgp_extrapolate(ctx, None, None, None) == N.CGP_ERR_INVALID
    lib.cgp_destroy(ctx)
    lib.cgp_destroy(None)
