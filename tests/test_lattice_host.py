"""Host checks of the lattice mass operator (no GPU): the library's stencil
code (the same functions the Chebyshev kernel runs) against the oracle's
assembled P1 mass matrix, on structured and unstructured coarse meshes and
every coarsening level."""
import ctypes as C
import os

import numpy as np
import pytest

from oracle.fem import Operators
from oracle.hierarchy import Hierarchy
from workloads import unit_square, channel_cylinder, disc, NATURAL


@pytest.fixture(scope="module")
def N():
    from paper_1812_00185_amd import _native as N

    if not os.path.exists(N.LIB_PATH):
        from paper_1812_00185_amd.build import build

        build()
    N.load()
    return N


CASES = [
    ("square_k0", lambda: unit_square(9), 0),
    ("square_k1", lambda: unit_square(9, tags={"left": NATURAL}), 1),
    ("square_k2", lambda: unit_square(17), 2),
    ("square_k3", lambda: unit_square(33), 3),
    ("disc_k2", lambda: disc(30, 120, seed=2), 2),
    ("disc_k3", lambda: disc(30, 80, seed=1), 3),
    ("channel_k2", lambda: channel_cylinder(0.05), 2),
]


@pytest.mark.parametrize("name,meshf,k", CASES, ids=[c[0] for c in CASES])
def test_lattice_mass_apply_matches_assembled(N, name, meshf, k):
    from paper_1812_00185_amd.solver import CGP

    mesh = meshf()
    g = CGP(mesh, k, 1e-3, 1e-2, device="cpu")
    try:
        M = Operators(Hierarchy(mesh, k).fine).M.tocsr()
        M.sort_indices()
        rp = np.ascontiguousarray(M.indptr, np.int32)
        col = np.ascontiguousarray(M.indices, np.int32)
        val = np.ascontiguousarray(M.data, np.float64)
        x = np.random.default_rng(k + 3).standard_normal(g.nf)
        y, d = np.empty(g.nf), np.empty(g.nf)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        rc = g.lib.cgp_lattice_mass_apply_host(
            g.ctx, rp.ctypes.data_as(ip), col.ctypes.data_as(ip), val.ctypes.data_as(dp),
            x.ctypes.data_as(dp), y.ctypes.data_as(dp), d.ctypes.data_as(dp))
        assert rc == 0, g.lib.cgp_last_error()
        ref = M @ x
        err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
        derr = np.max(np.abs(d - M.diagonal()) / M.diagonal())
        print(f"[lattice] {name}: N_f={g.nf} rel err {err:.2e} diag {derr:.2e}")
        assert err < 1e-13 and derr < 1e-12
    finally:
        g.close()
