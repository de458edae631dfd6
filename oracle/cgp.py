"""The CGP incremental pressure-projection time step (Sect. 2.2, Eqs. 21-26).

Oracle (test infrastructure only).  One step maps (U^{n-1}, U^n, P^n, Phi_c^n)
to (U^{n+1}, P^{n+1}, Phi_c^{n+1}):

  1. momentum (Eq. 21):
       (3/2 M + dt N(w) + dt nu K) U~ = -dt G P^n + dt M F + 2 M U^n - 1/2 M U^{n-1},
       w = 2 U^n - U^{n-1} (extrapolated convecting velocity, Eq. 9);
       Dirichlet rows replaced by U~ = u_D(t^{n+1}) (Eq. 10); the traction
       t_N(t^{n+1}) of Eq. 11 on the natural edges adds dt B T to the
       right-hand side (B the P1 boundary mass matrix of those edges, T the
       nodal traction), so that the weak form's natural condition is
       -p^n n + nu grad(u~) n = t_N (the boundary part of -G P^n supplies
       -p^n n).
  2.-3. restriction and coarse Poisson (Eqs. 22-23):
       K_c Phi_c = -(3/(2 dt)) Dbar U~, with Phi_c = 0 at natural-boundary
       nodes (Eq. 14, rows and columns removed) and the natural condition of
       Eq. 13 elsewhere.  Dbar is the divergence of the coarsened mesh derived
       from inner products with the coarse shape functions (Sect. 2.2); two
       readings are provided:
         'galerkin' (default): the coarse shape functions tested against the
             fine velocity, (Dbar U~)_I = int psi_I^c div u~_f = (P^T D_f U~)_I;
         'inject': the fine velocity injected onto the coarse nodes first
             (Eq. 22, U~_c = R U~) and the coarse-mesh divergence D_c applied.
       Only the first keeps the fine velocity error independent of the
       coarsening level, as the paper reports (Table 1); the second grows
       without bound for two coarsening levels in the rotational form.
  4. prolongation (Eq. 24): Phi_f = P Phi_c.
  5. velocity (Eq. 25): M U^{n+1} = M U~ - (2/3) dt G Phi_f, solved as
       M dU = -(2/3) dt G Phi_f on the non-Dirichlet nodes, dU = 0 on Dirichlet
       nodes, U^{n+1} = U~ + dU.
  6. pressure: chi = 0 takes the algebraic update of Eq. 16,
       P^{n+1} = P^n + Phi_f (Sect. 2.3);
     chi = 1 solves Eq. 26 with the consistent mass matrix:
       M dp = -nu D U~,  P^{n+1} = P^n + Phi_f + dp.

Non-incremental form (scheme='nonincremental', the "NCGP" the paper compares
with, Sect. 2.3): the momentum equation has no pressure term, the coarse
Poisson problem of Eq. 23 is solved for the pressure itself (same right-hand
side and scaling), the velocity correction is Eq. 25, and P^{n+1} = Phi_f;
it has no rotational form (chi = 0).

Readings where the paper is silent:
  * the linear solvers are Jacobi-PCG (symmetric) and Jacobi-BiCGSTAB
    (momentum) with ||r|| <= tol ||b||; the momentum solve starts from w with
    the Dirichlet values of Eq. 10 imposed (so the Dirichlet rows' residual is
    zero throughout and the shadow residual lives on the free rows), the
    Poisson solve from the previous step's Phi_c (zero at the first step);
    with coarse='exact' the coarse system is solved directly instead (the
    limit of a PCG whose preconditioner is an exact factorisation of K_c);
  * when no boundary is natural the coarse Poisson problem is pure Neumann:
    the right-hand side is projected onto mean zero (Euclidean mean) before the
    solve, and the lumped-mass-weighted mean of Phi_c is removed after it;
  * at a node shared by Dirichlet and natural edges the velocity is Dirichlet
    and Phi = 0;
  * 1/Re is written nu.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import Operators
from .hierarchy import Hierarchy, dirichlet_nodes, natural_nodes
from .krylov import SolveInfo, bicgstab_jacobi, pcg_jacobi


@dataclass
class State:
    U_prev: np.ndarray          # [2, N_f]
    U: np.ndarray               # [2, N_f]
    P: np.ndarray               # [N_f]
    phi_hist: np.ndarray        # [4, N_c], most recent first
    step: int = 0


@dataclass
class StepResult:
    state: State
    U_tilde: np.ndarray
    b_c: np.ndarray
    phi_c: np.ndarray
    phi_f: np.ndarray
    stats: dict = field(default_factory=dict)


def _rows_to_identity(A, rows):
    """Replace the given rows of A by identity rows."""
    n = A.shape[0]
    keep = np.ones(n)
    keep[rows] = 0.0
    put = np.zeros(n)
    put[rows] = 1.0
    return (sp.diags(keep) @ A + sp.diags(put)).tocsr()


MASS_MODES = ("consistent", "lumped_p", "lumped")


class OracleCGP:
    def __init__(self, coarse_mesh, levels, dt, nu, chi, pcg_tol=1e-8,
                 mom_tol=1e-12, mass_tol=1e-12, max_iter=20000, restrict="galerkin",
                 mass="consistent", coarse="pcg", scheme="incremental"):
        if restrict not in ("galerkin", "inject"):
            raise ValueError("restrict must be 'galerkin' or 'inject'")
        if scheme not in ("incremental", "nonincremental"):
            raise ValueError("scheme must be 'incremental' or 'nonincremental'")
        if scheme == "nonincremental" and chi != 0:
            raise ValueError("the non-incremental scheme has no rotational form (chi = 0)")
        # 'incremental': the paper's method (Eqs. 21-26); 'nonincremental': the
        # CGP form it is compared with (Sect. 2.3): no pressure in the momentum
        # equation, the coarse Poisson problem solved for the pressure itself,
        # P^{n+1} = Phi_f
        self.scheme = scheme
        if coarse not in ("pcg", "exact"):
            raise ValueError("coarse must be 'pcg' or 'exact'")
        # 'pcg': Jacobi-PCG to pcg_tol from the guess; 'exact': the exact
        # solution of the coarse system (what PCG preconditioned by an exact
        # factorisation of K_c returns, to rounding)
        self.coarse_solver = coarse
        if mass not in MASS_MODES:
            raise ValueError(f"mass must be one of {MASS_MODES}")
        self.restrict_mode = restrict
        # 'consistent': Eqs. 25 and 26 with the consistent M (the paper's
        # choice); 'lumped_p': the rotational pressure update with the lumped
        # mass matrix, Eq. 27; 'lumped': Eq. 27 and the velocity correction of
        # Eq. 25 with the lumped mass matrix as well
        self.mass_mode = mass
        self.hier = Hierarchy(coarse_mesh, levels)
        self.dt, self.nu, self.chi = float(dt), float(nu), int(chi)
        self.pcg_tol, self.mom_tol, self.mass_tol = pcg_tol, mom_tol, mass_tol
        self.max_iter = max_iter
        self.F = Operators(self.hier.fine)
        self.C = Operators(self.hier.coarse)
        self.nf = self.F.n
        self.nc = self.C.n
        self.dir = dirichlet_nodes(self.hier.fine)
        self.vel_free = np.setdiff1d(np.arange(self.nf), self.dir)
        self.nat_c = natural_nodes(self.hier.coarse)
        self.phi_free = np.setdiff1d(np.arange(self.nc), self.nat_c)
        self.pure_neumann = self.nat_c.size == 0
        self.Kc_ff = self.C.K[self.phi_free][:, self.phi_free].tocsr()
        self.M_ff = self.F.M[self.vel_free][:, self.vel_free].tocsr()
        self.A_const = (1.5 * self.F.M + (self.dt * self.nu) * self.F.K).tocsr()
        self.P = self.hier.prolongation_matrix()

    # ---- inputs --------------------------------------------------------
    @property
    def fine_xy(self):
        return self.F.xy

    def initial_state(self, U_prev, U, P):
        return State(np.array(U_prev, np.float64), np.array(U, np.float64),
                     np.array(P, np.float64), np.zeros((4, self.nc)))

    # ---- the six steps ---------------------------------------------------
    def momentum_system(self, U_prev, U, P, uD, F=None, T=None):
        """Matrix and right-hand sides of Eq. 21 with the Dirichlet rows set;
        T: nodal traction [2, N_f] on the natural edges (Eq. 11), or None
        (traction free)."""
        dt = self.dt
        w = 2.0 * U - U_prev
        A = (self.A_const + dt * self.F.convection(w[0], w[1])).tocsr()
        A = _rows_to_identity(A, self.dir)
        M = self.F.M
        GP = self.F.grad(P)
        rhs = np.empty((2, self.nf))
        for d in range(2):
            r = 2.0 * (M @ U[d]) - 0.5 * (M @ U_prev[d])
            if self.scheme == "incremental":
                r = r - dt * GP[d]
            if F is not None:
                r = r + dt * (M @ F[d])
            if T is not None:
                r = r + dt * (self.F.B @ T[d])
            r[self.dir] = uD[d]
            rhs[d] = r
        return A, rhs, w

    def momentum(self, U_prev, U, P, uD, F=None, T=None):
        A, rhs, w = self.momentum_system(U_prev, U, P, uD, F, T)
        # initial guess: w, with the Dirichlet values of Eq. 10 imposed
        x0 = w.copy()
        x0[:, self.dir] = uD
        Ut = np.empty_like(rhs)
        its = []
        for d in range(2):
            Ut[d], info = bicgstab_jacobi(A, rhs[d], x0=x0[d], tol=self.mom_tol,
                                          maxit=self.max_iter)
            its.append(info.iters)
        return Ut, its

    def restrict_rhs(self, Ut):
        """b_c = -(3/(2 dt)) Dbar U~ (Eqs. 22-23), phi = 0 rows zeroed,
        mean removed for the pure Neumann problem."""
        if self.restrict_mode == "galerkin":
            div_c = self.P.T @ self.F.div(Ut)
        else:
            div_c = self.C.div(self.hier.restrict(Ut))
        b = -(1.5 / self.dt) * div_c
        b[self.nat_c] = 0.0
        if self.pure_neumann:
            b = b - b.mean()
        return b

    def poisson(self, b, guess, pin=None):
        phi = np.zeros(self.nc)
        if self.coarse_solver == "exact":
            x, info = self.exact_coarse(b[self.phi_free], pin)
        else:
            x, info = pcg_jacobi(self.Kc_ff, b[self.phi_free], x0=guess[self.phi_free],
                                 tol=self.pcg_tol, maxit=self.max_iter)
        phi[self.phi_free] = x
        if self.pure_neumann:
            m = self.C.lumped
            phi = phi - (m @ phi) / m.sum()
        return phi, info

    def exact_coarse(self, b, pin=None):
        """Direct solve of K_c x = b on the phi-free unknowns.  K_c is
        singular in the pure Neumann case (constants are its null space and b
        has zero sum): one unknown (`pin`, default the last) is then fixed to
        0, which selects one solution; the mean removal in poisson() makes the
        result independent of that choice."""
        K = self.Kc_ff
        n = K.shape[0]
        x = np.zeros(n)
        if self.pure_neumann:
            pin = n - 1 if pin is None else pin
            keep = np.setdiff1d(np.arange(n), [pin])
            x[keep] = spla.spsolve(K[keep][:, keep].tocsc(), b[keep])
        else:
            x = spla.spsolve(K.tocsc(), b)
        nb = np.linalg.norm(b)
        res = np.linalg.norm(b - K @ x) / nb if nb > 0 else 0.0
        return x, SolveInfo(1, True, res)

    def velocity_correction(self, Ut, phi_f):
        """Eq. 25: M dU = -(2/3) dt G phi_f on the non-Dirichlet rows (dU = 0
        on the Dirichlet set); M consistent, or lumped (diagonal of row sums)
        in mass mode 'lumped'."""
        rhs = -(2.0 / 3.0) * self.dt * self.F.grad(phi_f)
        U = Ut.copy()
        its = []
        f = self.vel_free
        for d in range(2):
            if self.mass_mode == "lumped":
                U[d][f] += rhs[d][f] / self.F.lumped[f]
                its.append(0)
                continue
            du, info = pcg_jacobi(self.M_ff, rhs[d][f], tol=self.mass_tol, maxit=self.max_iter)
            U[d][f] += du
            its.append(info.iters)
        return U, its

    def pressure_update(self, P, phi_f, Ut):
        """chi = 0: P + phi_f (Eq. 16, algebraic form).  chi = 1: P + phi_f + dp
        with M dp = -nu D U~ (Eq. 26 / 20, consistent M) or dp = M_L^-1 (-nu D U~)
        with the lumped M_L (Eq. 27)."""
        if self.scheme == "nonincremental":
            return phi_f.copy(), 0
        if self.chi == 0:
            return P + phi_f, 0
        rhs = -self.nu * self.F.div(Ut)
        if self.mass_mode in ("lumped_p", "lumped"):
            return P + phi_f + rhs / self.F.lumped, 0
        dp, info = pcg_jacobi(self.F.M, rhs, tol=self.mass_tol, maxit=self.max_iter)
        return P + phi_f + dp, info.iters

    def step(self, st: State, uD, F=None, guess=None, T=None) -> StepResult:
        Ut, mom_its = self.momentum(st.U_prev, st.U, st.P, uD, F, T)
        b = self.restrict_rhs(Ut)
        g = st.phi_hist[0] if guess is None else guess
        phi_c, pinfo = self.poisson(b, g)
        phi_f = self.hier.prolong(phi_c)
        U_new, mass_its = self.velocity_correction(Ut, phi_f)
        P_new, p_its = self.pressure_update(st.P, phi_f, Ut)
        hist = np.concatenate([phi_c[None], st.phi_hist[:-1]])
        new = State(st.U.copy(), U_new, P_new, hist, st.step + 1)
        stats = dict(mom_iters=mom_its, pcg_iters=pinfo.iters, pcg_res=pinfo.res,
                     pcg_converged=pinfo.converged, mass_iters=mass_its,
                     prot_iters=p_its)
        return StepResult(new, Ut, b, phi_c, phi_f, stats)

    # ---- diagnostics -----------------------------------------------------
    def l2(self, e):
        """Discrete L2 norm sqrt(e^T M e); vector fields sum over components."""
        e = np.atleast_2d(e)
        return float(np.sqrt(sum(ei @ (self.F.M @ ei) for ei in e)))

    def mean_free(self, p):
        m = self.F.lumped
        return p - (m @ p) / m.sum()


def build(workload):
    return OracleCGP(workload.coarse_mesh(), workload.levels, workload.dt, workload.nu,
                     workload.chi, workload.pcg_tol, workload.mom_tol, workload.mass_tol,
                     workload.max_iter, workload.restrict, workload.mass,
                     "exact" if workload.precond == "ndchol" else "pcg", workload.scheme)


def run(workload, steps=None, record=None, F=None):
    """Run a workload from its initial fields (its forcing and traction data
    when it has them, else F); returns (oracle, final state, per-step stats,
    recorded StepResults at the requested step numbers)."""
    ora = build(workload)
    Um, U0, P0 = workload.initial_fields(ora.fine_xy)
    st = ora.initial_state(Um, U0, P0)
    xy_dir = ora.fine_xy[ora.dir]
    nsteps = workload.steps if steps is None else steps
    recs = {}
    allstats = []
    for n in range(nsteps):
        t = (n + 1) * workload.dt
        uD = workload.dirichlet_values(xy_dir, t)
        Fw = workload.forcing(ora.fine_xy, t)
        res = ora.step(st, uD, F if Fw is None else Fw,
                       T=workload.traction(ora.fine_xy, t))
        st = res.state
        allstats.append(res.stats)
        if record is not None and (n + 1) in record:
            recs[n + 1] = res
    return ora, st, allstats, recs
