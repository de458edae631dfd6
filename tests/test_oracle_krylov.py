"""Pins of the oracle's Krylov solvers against direct solves."""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spl

from oracle import fem
from oracle.cgp import OracleCGP
from oracle.krylov import pcg_jacobi, bicgstab_jacobi
from workloads import unit_square, disc, get_workload, NATURAL


def test_pcg_matches_direct_spd():
    m = unit_square(17, tags={"left": NATURAL})
    op = fem.Operators(m)
    free = np.setdiff1d(np.arange(op.n), np.where(m["xy"][:, 0] == 0)[0])
    K = op.K[free][:, free].tocsr()
    rng = np.random.default_rng(0)
    b = rng.normal(size=free.size)
    x_d = spl.spsolve(K.tocsc(), b)
    for tol in (1e-6, 1e-10):
        x, info = pcg_jacobi(K, b, tol=tol)
        assert info.converged and info.res <= tol
        true = np.linalg.norm(b - K @ x) / np.linalg.norm(b)
        assert true <= 10 * tol
        # error bound ||x - x*|| <= ||K^-1|| ||r||
        lam_min = spl.eigsh(K, k=1, sigma=0, which="LM", return_eigenvectors=False)[0]
        assert np.linalg.norm(x - x_d) <= 1.01 * true * np.linalg.norm(b) / lam_min


def test_pcg_pure_neumann_vs_bordered_direct():
    """Singular K with b in range(K): compare with the bordered (Lagrange
    multiplier) system that fixes the mean."""
    m = disc(30, 80, seed=5)
    op = fem.Operators(m)
    K = op.K
    rng = np.random.default_rng(1)
    b = rng.normal(size=op.n)
    b -= b.mean()
    x, info = pcg_jacobi(K, b, tol=1e-12)
    assert info.converged
    one = np.ones((op.n, 1))
    B = sp.bmat([[K, sp.csr_matrix(one)], [sp.csr_matrix(one.T), None]]).tocsc()
    xd = spl.spsolve(B, np.concatenate([b, [0.0]]))[:-1]
    np.testing.assert_allclose(x - x.mean(), xd - xd.mean(), atol=1e-9 * np.abs(xd).max())


def test_pcg_zero_rhs_and_good_guess():
    op = fem.Operators(unit_square(9))
    K = (op.K + op.M).tocsr()
    x, info = pcg_jacobi(K, np.zeros(op.n))
    assert info.iters == 0 and not x.any()
    b = np.ones(op.n)
    xs = spl.spsolve(K.tocsc(), b)
    x, info = pcg_jacobi(K, b, x0=xs, tol=1e-8)
    assert info.iters == 0


def test_bicgstab_matches_splu_on_momentum_matrix():
    w = get_workload("tg33_k1").with_(coarse_n=9, levels=1)
    ora = OracleCGP(w.coarse_mesh(), w.levels, w.dt, w.nu, w.chi)
    Um, U0, P0 = w.initial_fields(ora.fine_xy)
    uD = w.dirichlet_values(ora.fine_xy[ora.dir], w.dt)
    A, rhs, wv = ora.momentum_system(Um, U0, P0, uD)
    assert abs(A - A.T).max() > 0          # genuinely nonsymmetric
    lu = spl.splu(A.tocsc())
    for d in range(2):
        x, info = bicgstab_jacobi(A, rhs[d], x0=wv[d], tol=1e-12)
        assert info.converged
        xd = lu.solve(rhs[d])
        assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)
        # Dirichlet rows reproduce the boundary data exactly up to the tolerance
        np.testing.assert_allclose(x[ora.dir], uD[d], atol=1e-11)
