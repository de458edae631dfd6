"""Krylov solvers used by the oracle (test infrastructure only).

The paper solves every system with ILU(0)-GMRES(m) (Sect. 2.3); the library
replaces that with diagonally (Jacobi) preconditioned CG for the symmetric
systems and BiCGSTAB for the momentum system.  The oracle runs the same two
algorithms in FP64, written out plainly, with the same stopping rule:

  stop when ||r_k||_2 <= tol * ||b||_2 with r_k the recursively updated
  residual (relative to ||b||, not ||r_0||, so a better initial guess pays).

A zero right-hand side returns the zero vector after 0 iterations.
"""
from __future__ import annotations

import numpy as np


class SolveInfo:
    def __init__(self, iters, converged, res):
        self.iters = iters
        self.converged = converged
        self.res = res

    def __repr__(self):
        return f"SolveInfo(iters={self.iters}, converged={self.converged}, res={self.res:.3e})"


def pcg_jacobi(A, b, x0=None, tol=1e-10, maxit=10000):
    """Jacobi-preconditioned conjugate gradients for symmetric A (positive
    definite, or semi-definite with b in range(A))."""
    b = np.asarray(b, np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, np.float64)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros_like(b), SolveInfo(0, True, 0.0)
    dinv = 1.0 / A.diagonal()
    r = b - A @ x
    rnorm = np.linalg.norm(r)
    if rnorm <= tol * bnorm:
        return x, SolveInfo(0, True, rnorm / bnorm)
    z = dinv * r
    p = z.copy()
    rho = r @ z
    for k in range(1, maxit + 1):
        q = A @ p
        alpha = rho / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        rnorm = np.linalg.norm(r)
        if rnorm <= tol * bnorm:
            return x, SolveInfo(k, True, rnorm / bnorm)
        z = dinv * r
        rho_new = r @ z
        beta = rho_new / rho
        rho = rho_new
        p = z + beta * p
    return x, SolveInfo(maxit, False, rnorm / bnorm)


def bicgstab_jacobi(A, b, x0=None, tol=1e-12, maxit=1000):
    """Right-Jacobi-preconditioned BiCGSTAB (van der Vorst) for nonsymmetric A,
    shadow residual r^ = r_0.  The stopping test is also applied to the
    half-step residual s, in which case x + alpha p^ is returned."""
    b = np.asarray(b, np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, np.float64)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros_like(b), SolveInfo(0, True, 0.0)
    dinv = 1.0 / A.diagonal()
    r = b - A @ x
    rnorm = np.linalg.norm(r)
    if rnorm <= tol * bnorm:
        return x, SolveInfo(0, True, rnorm / bnorm)
    rhat = r.copy()
    rho_old = alpha = omega = 1.0
    p = np.zeros_like(b)
    v = np.zeros_like(b)
    for k in range(1, maxit + 1):
        rho = rhat @ r
        beta = (rho / rho_old) * (alpha / omega)
        p = r + beta * (p - omega * v)
        phat = dinv * p
        v = A @ phat
        alpha = rho / (rhat @ v)
        s = r - alpha * v
        snorm = np.linalg.norm(s)
        if snorm <= tol * bnorm:
            # half-step convergence (also guards t = 0 below)
            return x + alpha * phat, SolveInfo(k, True, snorm / bnorm)
        shat = dinv * s
        t = A @ shat
        omega = (t @ s) / (t @ t)
        x = x + alpha * phat + omega * shat
        r = s - omega * t
        rho_old = rho
        rnorm = np.linalg.norm(r)
        if rnorm <= tol * bnorm:
            return x, SolveInfo(k, True, rnorm / bnorm)
    return x, SolveInfo(maxit, False, rnorm / bnorm)
