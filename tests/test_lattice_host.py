"""Host checks of the lattice mass operator (no GPU): the library's stencil
code (the same functions the Chebyshev kernel runs) against the oracle's
assembled P1 mass matrix, on structured and unstructured coarse meshes and
every coarsening level."""
import ctypes as C
import os

import numpy as np
import pytest
from scipy.sparse.linalg import spsolve

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


# ------------------------------------------------------- paired Chebyshev steps

def _cheb_coefs(iters):
    """(ca_j, cb_j), j < iters, of the three-term Chebyshev recurrence on the
    interval [1/2, 2] (the mass solves of Eqs. 25-26)."""
    theta, delta = 1.25, 0.75
    sigma = theta / delta
    rho = 1.0 / sigma
    out = []
    for j in range(iters):
        ca, cb = 0.0, 1.0 / theta
        if j > 0:
            rn = 1.0 / (2.0 * sigma - rho)
            ca, cb, rho = rn * rho, 2.0 * rn / delta, rn
        out.append((ca, cb))
    return out


PAIR_CASES = [
    # (name, coarse mesh, nr); triangle counts not multiples of the 12 per
    # block, odd (143 triangles) and even first edge nodes, natural
    # boundaries, unstructured
    ("square9_nr3", lambda: unit_square(9), 3),
    ("square6_nr2", lambda: unit_square(6, tags={"left": NATURAL}), 2),
    ("disc_nr3", lambda: disc(30, 80, seed=1), 3),
    ("disc_odd_nr2", lambda: disc(25, 60, seed=4), 2),
    ("disc_odd_nr3", lambda: disc(25, 60, seed=4), 3),
]


@pytest.mark.parametrize("name,meshf,nr", PAIR_CASES, ids=[c[0] for c in PAIR_CASES])
def test_cheb_pairs_match_step_by_step(N, name, meshf, nr):
    """A whole mass solve as the library launches it on lattice size 8 --
    step pairs of a step on the coarse-edge and vertex nodes, the two-step
    kernel on the interior nodes, a step on the edge and vertex nodes --
    emulated on the host with every index checked and the iterates starting
    as NaN, equals the step-by-step sequence bit for bit, and both equal the
    Chebyshev recurrence
    x_{j+1} = x_j + ca (x_j - x_{j-1}) + cb D^-1 (b - M x_j) with the
    oracle's assembled mass matrix (velocity components held at 0 on
    Dirichlet nodes), for odd and even step counts."""
    from paper_1812_00185_amd.solver import CGP

    mesh = meshf()
    g = CGP(mesh, 3, 1e-3, 1e-2, device="cpu")
    try:
        M = Operators(Hierarchy(mesh, 3).fine).M.tocsr()
        M.sort_indices()
        rp = np.ascontiguousarray(M.indptr, np.int32)
        col = np.ascontiguousarray(M.indices, np.int32)
        val = np.ascontiguousarray(M.data, np.float64)
        rng = np.random.default_rng(len(name) + nr)
        n = g.nf
        b = rng.standard_normal((n, nr))
        di = 1.0 / M.diagonal()
        mask = np.zeros((n, nr), bool)
        mask[g.dirichlet_nodes, :2] = True
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)

        def lib_solve(iters, pairs, mixed=0):
            x = np.empty((n, nr))
            rc = g.lib.cgp_lattice_cheb_solve_host(
                g.ctx, rp.ctypes.data_as(ip), col.ctypes.data_as(ip), val.ctypes.data_as(dp),
                nr, b.ctypes.data_as(dp), iters, pairs, mixed, x.ctypes.data_as(dp))
            assert rc == 0, g.lib.cgp_last_error()
            return x

        for iters in (1, 2, 3, 4, 5, 6, 27):
            cf = _cheb_coefs(iters)
            xp, x = np.zeros((n, nr)), np.zeros((n, nr))
            for ca, cb in cf:
                xn = x + ca * (x - xp) + (cb * di)[:, None] * (b - M @ x)
                xn[mask] = 0.0
                xp, x = x, xn
            got = lib_solve(iters, 1)
            steps = lib_solve(iters, 0)
            assert np.all(np.isfinite(got)), f"{iters} steps: a value read before it was written"
            assert np.array_equal(got, steps), f"{iters} steps: pairs differ from single steps"
            err = np.abs(got - x).max() / np.abs(x).max()
            print(f"[cheb pairs] {name}: N_f={n} coarse triangles {len(mesh['tri'])} "
                  f"{iters} steps {err:.1e}")
            # rounding: the stencil sums in another order than the CSR product
            assert err < 1e-13
            assert np.all(got[mask] == 0.0)

        # the mixed-precision form (two float-stored solves of 15 steps, the
        # FP64 residual of the first as the second's right-hand side) against
        # the exact solution; 27 FP64 steps for comparison
        free = ~mask
        exact = np.zeros((n, nr))
        for d in range(nr):
            f = free[:, d]
            exact[f, d] = spsolve(M[f][:, f].tocsc(), b[f, d])
        scale = np.abs(exact).max()
        mix = lib_solve(15, 1, 1)
        assert np.array_equal(mix, lib_solve(15, 0, 1)), "mixed: pairs differ from single steps"
        e_mix = np.abs(mix - exact).max() / scale
        e64 = np.abs(lib_solve(27, 1) - exact).max() / scale
        print(f"[cheb mixed] {name}: vs exact {e_mix:.1e} (FP64, 27 steps: {e64:.1e})")
        assert np.all(mix[mask] == 0.0)
        assert e_mix < 1e-11 and e64 < 1e-11
    finally:
        g.close()


def test_cheb_solve_host_rejects_other_lattice_sizes(N):
    from paper_1812_00185_amd.solver import CGP

    g = CGP(unit_square(9), 2, 1e-3, 1e-2, device="cpu")
    try:
        z = np.zeros(3 * g.nf)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        i = np.zeros(g.nc + 1, np.int32)
        rc = g.lib.cgp_lattice_cheb_solve_host(
            g.ctx, i.ctypes.data_as(ip), i.ctypes.data_as(ip), z.ctypes.data_as(dp), 3,
            z.ctypes.data_as(dp), 5, 1, 0, z.ctypes.data_as(dp))
        assert rc != 0 and b"lattice size 8" in g.lib.cgp_last_error()
    finally:
        g.close()


# ------------------------------------------------ correction right-hand sides

RHS_CASES = [
    ("square_k1_natural", lambda: unit_square(9, tags={"left": NATURAL}), 1, 1),
    ("square_k2", lambda: unit_square(17), 2, 0),
    ("square_k3", lambda: unit_square(9), 3, 1),
    ("square_k3_natural", lambda: unit_square(9, tags={"left": NATURAL}), 3, 1),
    ("disc_k3", lambda: disc(30, 80, seed=1), 3, 1),
    ("channel_k2", lambda: channel_cylinder(0.08), 2, 1),
    ("square_k0", lambda: unit_square(9), 0, 1),
]


@pytest.mark.parametrize("name,meshf,k,chi", RHS_CASES, ids=[c[0] for c in RHS_CASES])
def test_lattice_correction_rhs_matches_assembled(N, name, meshf, k, chi):
    """The right-hand sides of Eqs. 25-26 as the library forms them on the
    lattice layout (geometry from the coarse triangles, interior stencils
    from coefficient differences, edge and vertex nodes triangle by
    triangle) against the oracle's assembled G = -D^T and D on the fine mesh,
    for arbitrary (not prolonged) phi_f and U~, natural boundaries
    included."""
    from paper_1812_00185_amd.solver import CGP

    mesh = meshf()
    dt, nu = 1e-3, 1e-2
    g = CGP(mesh, k, dt, nu, chi=chi, device="cpu")
    try:
        F = Operators(Hierarchy(mesh, k).fine)
        rng = np.random.default_rng(k + 11 * chi + len(name))
        phi = rng.standard_normal(g.nf)
        ut = rng.standard_normal((2, g.nf))
        dp = C.POINTER(C.c_double)
        hier = Hierarchy(mesh, k)
        phic = rng.standard_normal(g.nc)
        # arbitrary phi_f; then phi_f = P phi_c given as phi_c (the step's form)
        for label, pf, pc in (("phi_f", phi, None), ("phi_c", hier.prolong(phic), phic)):
            rhs = np.empty((g.nf, 3))
            rc = g.lib.cgp_lattice_correct_rhs_host(
                g.ctx, pf.ctypes.data_as(dp) if pc is None else None,
                None if pc is None else pc.ctypes.data_as(dp),
                np.ascontiguousarray(ut).ctypes.data_as(dp), rhs.ctypes.data_as(dp))
            assert rc == 0, g.lib.cgp_last_error()
            ref_u = -(2.0 / 3.0) * dt * F.grad(pf)
            ref_u[:, g.dirichlet_nodes] = 0.0
            ref_p = -nu * F.div(ut) if chi else np.zeros(g.nf)
            eu = np.abs(rhs[:, :2].T - ref_u).max() / np.abs(ref_u).max()
            ep = np.abs(rhs[:, 2] - ref_p).max() / max(np.abs(ref_p).max(), 1e-300)
            print(f"[corr rhs] {name} ({label}): N_f={g.nf} velocity {eu:.1e} pressure {ep:.1e}")
            assert eu < 1e-13
            assert (ep < 1e-13) if chi else np.all(rhs[:, 2] == 0.0)
            assert np.all(rhs[g.dirichlet_nodes, :2] == 0.0)
    finally:
        g.close()


# ------------------------------------------------------------ momentum rows

MOM_CASES = [
    ("square_k1", lambda: unit_square(9), 1, False),
    ("square_k3", lambda: unit_square(9), 3, False),
    ("square_k3_traction", lambda: unit_square(9, tags={"left": NATURAL}), 3, True),
    ("disc_k2", lambda: disc(30, 120, seed=2), 2, False),
    ("disc_k3", lambda: disc(30, 80, seed=1), 3, False),
    ("channel_k2_traction", lambda: channel_cylinder(0.08), 2, True),
]


@pytest.mark.parametrize("name,meshf,k,trac", MOM_CASES, ids=[c[0] for c in MOM_CASES])
def test_lattice_momentum_rows_match_assembled(N, name, meshf, k, trac):
    """The momentum rows of Eq. 21 as the library assembles them on the
    lattice layout (fine-triangle coefficients from the coarse triangles, no
    coordinate, side or column index read) against the oracle's assembled
    matrix, right-hand side, initial guess and initial residual, on every row of a fine node
    other than the coarse vertices (those keep the side-based assembly):
    random fields, pressure, forcing, Dirichlet values and, on natural
    boundaries, traction."""
    from oracle.cgp import OracleCGP
    from paper_1812_00185_amd.solver import CGP

    mesh = meshf()
    dt, nu = 1e-3, 1e-2
    g = CGP(mesh, k, dt, nu, chi=1, device="cpu")
    o = OracleCGP(mesh, k, dt, nu, 1)
    try:
        n = g.nf
        assert np.array_equal(o.dir, g.dirichlet_nodes)
        rng = np.random.default_rng(k + len(name))
        Up, U, F = (rng.standard_normal((2, n)) for _ in range(3))
        P = rng.standard_normal(n)
        uD = rng.standard_normal((2, o.dir.size))
        T = rng.standard_normal((2, n)) if trac else None
        A, rhs_o, w = o.momentum_system(Up, U, P, uD, F, T)
        A = A.tocsr()
        x0_o = w.copy()
        x0_o[:, o.dir] = uD
        nnz = int(g.sizes.nnz_fine)
        rowptr = np.empty(n + 1, np.int32)
        col = np.empty(nnz, np.int32)
        aval = np.empty(nnz)
        rhs = np.empty((2, n))
        x0 = np.empty((2, n))
        r0 = np.empty((2, n))
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        arr = lambda a: None if a is None else np.ascontiguousarray(a).ctypes.data_as(dp)
        rc = g.lib.cgp_lattice_momentum_host(
            g.ctx, arr(Up), arr(U), arr(P), arr(uD), arr(F), arr(T), rowptr.ctypes.data_as(ip),
            col.ctypes.data_as(ip), aval.ctypes.data_as(dp), rhs.ctypes.data_as(dp),
            x0.ctypes.data_as(dp), r0.ctypes.data_as(dp))
        assert rc == 0, g.lib.cgp_last_error()
        rows = np.arange(g.nc, n)
        assert rows.size > 0
        lo, hi = rowptr[g.nc], rowptr[n]
        ri = np.repeat(np.arange(n), np.diff(rowptr))[lo:hi]
        ref = np.asarray(A[ri, col[lo:hi]]).ravel()
        assert np.array_equal(x0[:, rows], x0_o[:, rows])
        # Dirichlet rows (identity, boundary values) exactly; free rows to
        # rounding, scaled by the free rows' own magnitudes
        dirrow = np.zeros(n, bool)
        dirrow[o.dir] = True
        fr = ~dirrow[ri]
        assert np.array_equal(aval[lo:hi][~fr], ref[~fr])
        rf = rows[~dirrow[rows]]
        assert np.array_equal(rhs[:, rows[dirrow[rows]]], rhs_o[:, rows[dirrow[rows]]])
        ea = np.abs(aval[lo:hi][fr] - ref[fr]).max() / np.abs(ref[fr]).max()
        er = np.abs(rhs[:, rf] - rhs_o[:, rf]).max() / np.abs(rhs_o[:, rf]).max()
        # the initial residual the assembly forms for BiCGSTAB: rhs - A x0 with
        # the oracle's matrix and guess (zero on Dirichlet rows)
        res_o = np.stack([rhs_o[d] - A @ x0_o[d] for d in range(2)])
        assert np.all(r0[:, rows[dirrow[rows]]] == 0.0)
        e0 = np.abs(r0[:, rf] - res_o[:, rf]).max() / np.abs(rhs_o[:, rf]).max()
        print(f"[mom rows] {name}: N_f={n}, free rows {rf.size}: A {ea:.1e} rhs {er:.1e} "
              f"r0 {e0:.1e}")
        assert ea < 1e-13 and er < 1e-13 and e0 < 1e-13
        # the coarse-vertex rows are left to the side-based kernel
        assert np.all(np.isnan(aval[:lo])) and np.all(np.isnan(rhs[:, :g.nc]))
    finally:
        g.close()
