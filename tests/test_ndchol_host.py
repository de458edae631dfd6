"""Host checks of the nested-dissection factor preconditioner of the coarse
solve (no GPU): the library's host routine runs the ordering, the symbolic and
numeric factorisation and the level-by-level triangular solves that the
device kernels run, on the coarse stiffness matrices of the oracle; the
result must solve the system.  Also the oracle's exact coarse solve against
properties that fix it."""
import ctypes as C
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle.cgp import OracleCGP
from oracle.fem import Operators
from oracle.hierarchy import natural_nodes
from workloads import unit_square, channel_cylinder, disc, NATURAL, get_workload


@pytest.fixture(scope="module")
def N():
    from paper_1812_00185_amd import _native as N

    if not os.path.exists(N.LIB_PATH):
        from paper_1812_00185_amd.build import build

        build()
    N.load()
    return N


MESHES = {
    "square_natural": lambda: unit_square(33, tags={"left": NATURAL}),
    "square_neumann": lambda: unit_square(65),
    "disc_neumann": lambda: disc(30, 200, seed=3),
    "channel": lambda: channel_cylinder(0.05),
}


def coarse_system(mesh):
    C_ = Operators(mesh)
    K = C_.K.tocsr()
    K.sort_indices()
    nat = natural_nodes(mesh)
    skip = np.zeros(K.shape[0], np.uint8)
    skip[nat] = 1
    if nat.size == 0:
        skip[-1] = 1          # the library pins the last node of a pure Neumann problem
    return K, C_.xy, skip


@pytest.mark.parametrize("name", sorted(MESHES))
def test_host_factor_solves_the_system(N, name):
    K, xy, skip = coarse_system(MESHES[name]())
    n = K.shape[0]
    free = np.flatnonzero(skip == 0)
    r = np.random.default_rng(7).standard_normal(n)
    z, info = N.ndchol_solve_host(K.indptr, K.indices, K.data, xy, skip, r)
    Kf = K[free][:, free]
    res = np.linalg.norm(Kf @ z[free] - r[free]) / np.linalg.norm(r[free])
    assert res < 1e-12, res
    assert np.all(z[skip == 1] == 0.0)
    ref = spla.spsolve(Kf.tocsc(), r[free])
    assert np.linalg.norm(z[free] - ref) / np.linalg.norm(ref) < 1e-10
    assert info["n_factored"] == free.size
    assert 1 <= info["height"] <= 2 * int(np.log2(n)) + 2
    assert info["max_front"] <= 8192 and info["g_entries"] > 0
    print(f"[ndchol] {name}: n={n} {info} residual {res:.1e}")


def test_host_factor_is_linear_and_exact_on_the_range(N):
    """Solving K z = K x recovers x on the factored unknowns (any x)."""
    K, xy, skip = coarse_system(MESHES["square_natural"]())
    free = skip == 0
    x = np.random.default_rng(3).standard_normal(K.shape[0])
    x[~free] = 0.0
    z, _ = N.ndchol_solve_host(K.indptr, K.indices, K.data, xy, skip, K @ x)
    assert np.linalg.norm(z - x) / np.linalg.norm(x) < 1e-11


def test_host_factor_rejects_indefinite_and_bad_input(N):
    K, xy, skip = coarse_system(MESHES["square_natural"]())
    bad = K.copy()
    bad.data = -bad.data
    with pytest.raises(N.CGPError, match="pivot"):
        N.ndchol_solve_host(bad.indptr, bad.indices, bad.data, xy, skip, np.ones(K.shape[0]))
    col = K.indices.copy()
    col[3] = K.shape[0]
    with pytest.raises(N.CGPError, match="out of range"):
        N.ndchol_solve_host(K.indptr, col, K.data, xy, skip, np.ones(K.shape[0]))


def test_host_factor_single_node_and_tiny(N):
    K = sp.csr_matrix(np.array([[2.0, -1.0], [-1.0, 2.0]]))
    z, info = N.ndchol_solve_host(K.indptr, K.indices, K.data, np.array([0.0, 0, 1, 0]),
                                  np.zeros(2, np.uint8), np.array([1.0, 0.0]))
    assert np.allclose(z, [2 / 3, 1 / 3], rtol=0, atol=1e-15)
    assert info["n_supernodes"] == 1 and info["height"] == 1


def test_context_reports_factor_structure(N):
    """cgp_create orders the coarse unknowns on the host: phi = 0 nodes are
    not unknowns and the pure Neumann problem pins one node."""
    from paper_1812_00185_amd.solver import CGP

    for mesh, expect in ((unit_square(17, tags={"left": NATURAL}), 17 * 17 - 17),
                         (unit_square(17), 17 * 17 - 1)):
        g = CGP(mesh, 1, 1e-3, 1e-2, precond="ndchol", device="cpu")
        assert g.ndchol["n_factored"] == expect and g.ndchol["height"] >= 2
        g.close()
    g = CGP(unit_square(17), 1, 1e-3, 1e-2, device="cpu")
    assert g.ndchol["n_factored"] == 0
    g.close()
    # the mixed-precision form keeps the same factor structure (FP32 values)
    g = CGP(unit_square(17), 1, 1e-3, 1e-2, precision="mixed", precond="ndchol", device="cpu")
    assert g.ndchol["n_factored"] == 17 * 17 - 1
    g.close()
    with pytest.raises(N.CGPError, match="requires precision"):
        CGP(unit_square(9), 1, 1e-3, 1e-2, precision="mixed", precond="jacobi_s4", device="cpu")


# ---------------------------------------------------------------- oracle pins

def _oracle(mesh, coarse):
    return OracleCGP(mesh, 1, 1e-3, 1e-2, 0, pcg_tol=1e-14, coarse=coarse)


@pytest.mark.parametrize("name", ["square_neumann", "square_natural"])
def test_oracle_exact_coarse_solves_eq23(name):
    """The exact coarse solve satisfies K_c phi = b on every unknown (the
    pinned row too, as b is compatible), and agrees with the independent
    Jacobi-PCG run to 1e-14."""
    mesh = MESHES[name]()
    o = _oracle(mesh, "exact")
    rng = np.random.default_rng(11)
    b = rng.standard_normal(o.nc)
    b[o.nat_c] = 0.0
    if o.pure_neumann:
        b -= b.mean()
    phi, info = o.poisson(b, np.zeros(o.nc))
    f = o.phi_free
    res = np.linalg.norm(o.Kc_ff @ phi[f] - b[f]) / np.linalg.norm(b[f])
    assert res < 1e-12, res
    phi_cg, _ = _oracle(mesh, "pcg").poisson(b, np.zeros(o.nc))
    assert np.linalg.norm(phi - phi_cg) / np.linalg.norm(phi) < 1e-10


def test_oracle_exact_coarse_independent_of_pin():
    """Pure Neumann: after the mean removal the result does not depend on
    which unknown was pinned."""
    o = _oracle(MESHES["disc_neumann"](), "exact")
    assert o.pure_neumann
    b = np.random.default_rng(5).standard_normal(o.nc)
    b -= b.mean()
    a, _ = o.poisson(b, np.zeros(o.nc))
    c, _ = o.poisson(b, np.zeros(o.nc), pin=0)
    assert np.linalg.norm(a - c) / np.linalg.norm(a) < 1e-11
    m = o.C.lumped
    assert abs(m @ a) < 1e-12 * np.linalg.norm(a) * m.sum()
