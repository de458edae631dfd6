"""The synthetic workloads: coarse mesh, coarsening level, time step, viscosity,
scheme and solver settings, initial fields and boundary data.

Each entry describes a problem only; how it is discretised and solved is up to
the caller (the HIP library or the CPU oracle).
"""
from __future__ import annotations

from dataclasses import dataclass, replace
from functools import lru_cache

import numpy as np

from . import flows
from .meshes import NATURAL, unit_square, channel_cylinder, disc

FP64 = 0
MIXED = 1


@dataclass(frozen=True)
class Workload:
    name: str
    mesh: str                  # 'square' | 'channel' | 'disc'
    coarse_n: int              # nodes per side of the coarse square mesh (square only)
    levels: int                # coarsening level k: fine = k uniform 4:1 refinements
    dt: float
    nu: float
    steps: int
    chi: int                   # 0 standard, 1 rotational
    flow: str                  # 'taylor_green' | 'cavity' | 'channel' | 'jobelin_disc' | 'jobelin_open'
    precision: int = FP64
    pcg_tol: float = 1e-8
    inner_tol: float = 1e-5
    mom_tol: float = 1e-12
    mass_tol: float = 1e-12
    max_iter: int = 20000
    restrict: str = "galerkin"     # 'galerkin' | 'inject'
    mass: str = "consistent"       # 'consistent' | 'lumped_p' (Eq. 27) | 'lumped'
    precond: str = "jacobi"        # coarse PCG preconditioner: 'jacobi' | 'ndchol' (exact factor)
    scheme: str = "incremental"    # 'incremental' (the method) | 'nonincremental' (NCGP, chi = 0)
    lid_speed: float = 1.0
    channel_h: float = 0.0082
    seed: int = 0
    phase: tuple = (0.0, 0.0)      # Taylor-Green shift (x0, y0): u(x - x0, y - y0, t)
    natural: tuple = ()            # square sides tagged NATURAL ('left', ...); others DIRICHLET

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)

    # ---- input data -----------------------------------------------------
    def coarse_mesh(self) -> dict:
        if self.mesh == "square":
            return _square(self.coarse_n, tuple(self.natural))
        if self.mesh == "channel":
            return _channel(self.channel_h, self.seed)
        if self.mesh == "disc":
            return _disc(self.seed)
        raise ValueError(self.mesh)

    def initial_fields(self, xy: np.ndarray):
        """(U^{-1}, U^0, P^0): Taylor-Green takes the exact fields at t=-dt and
        t=0; the impulsively started flows start from rest."""
        n = xy.shape[0]
        if self.flow == "taylor_green":
            x, y = self._shifted(xy)
            um, vm, _ = flows.taylor_green(x, y, -self.dt, self.nu)
            u0, v0, p0 = flows.taylor_green(x, y, 0.0, self.nu)
            return np.stack([um, vm]), np.stack([u0, v0]), p0
        if self.flow in ("jobelin_disc", "jobelin_open"):
            fn = flows.jobelin_disc if self.flow == "jobelin_disc" else flows.jobelin_open
            um, vm, _ = fn(xy[:, 0], xy[:, 1], -self.dt)
            u0, v0, p0 = fn(xy[:, 0], xy[:, 1], 0.0)
            return np.stack([um, vm]), np.stack([u0, v0]), p0
        z = np.zeros(n)
        return np.stack([z, z]), np.stack([z, z]), z.copy()

    def dirichlet_values(self, xy_dir: np.ndarray, t: float) -> np.ndarray:
        """[2, n_dir] velocity at the Dirichlet nodes at time t."""
        x, y = xy_dir[:, 0], xy_dir[:, 1]
        if self.flow == "taylor_green":
            u, v, _ = flows.taylor_green(*self._shifted(xy_dir), t, self.nu)
        elif self.flow == "cavity":
            u, v = flows.cavity_lid(x, y, self.lid_speed)
        elif self.flow == "channel":
            u, v = flows.channel_inflow(x, y)
        elif self.flow == "jobelin_disc":
            u, v, _ = flows.jobelin_disc(x, y, t)
        elif self.flow == "jobelin_open":
            u, v, _ = flows.jobelin_open(x, y, t)
        else:
            raise ValueError(self.flow)
        return np.stack([u, v])

    def exact(self, xy: np.ndarray, t: float):
        if self.flow in ("jobelin_disc", "jobelin_open"):
            fn = flows.jobelin_disc if self.flow == "jobelin_disc" else flows.jobelin_open
            u, v, p = fn(xy[:, 0], xy[:, 1], t)
            return np.stack([u, v]), p
        if self.flow != "taylor_green":
            return None
        u, v, p = flows.taylor_green(*self._shifted(xy), t, self.nu)
        return np.stack([u, v]), p

    def forcing(self, xy: np.ndarray, t: float):
        """[2, N] nodal body force at time t, or None (zero)."""
        if self.flow == "jobelin_disc":
            return np.stack(flows.jobelin_disc_forcing(xy[:, 0], xy[:, 1], t, self.nu))
        if self.flow == "jobelin_open":
            return np.stack(flows.jobelin_open_forcing(xy[:, 0], xy[:, 1], t, self.nu))
        return None

    def traction(self, xy: np.ndarray, t: float):
        """[2, N] nodal traction t_N = -p n + nu grad(u) n of the exact
        solution on the natural sides at time t (zero at every other node),
        or None (traction free)."""
        if self.flow != "jobelin_open" or not self.natural:
            return None
        return flows.jobelin_open_traction(xy, t, self.nu, self.natural)

    def _shifted(self, xy):
        """Coordinates shifted by the Taylor-Green phase (a translated exact
        solution is still one)."""
        return xy[:, 0] - self.phase[0], xy[:, 1] - self.phase[1]


@lru_cache(maxsize=8)
def _square_cached(n, natural):
    return unit_square(n, {s: NATURAL for s in natural})


def _square(n, natural=()):
    m = _square_cached(n, natural)
    return {k: v.copy() for k, v in m.items()}


@lru_cache(maxsize=2)
def _disc_cached(seed):
    return disc(96, 1105, 0.5, seed)


def _disc(seed):
    m = _disc_cached(seed)
    return {k: v.copy() for k, v in m.items()}


@lru_cache(maxsize=2)
def _channel_cached(h, seed):
    return channel_cylinder(h, seed)


def _channel(h, seed):
    m = _channel_cached(h, seed)
    return {k: v.copy() for k, v in m.items()}


# The five workloads.  Sizes follow the problem statement: unit-square meshes
# with n x n nodes, a channel with a cylinder, levels of 4:1 coarsening.
WORKLOADS = {
    # 33x33 fine / 17x17 pressure mesh, Taylor-Green, standard scheme, FP64 PCG 1e-10
    "tg33_k1": Workload("tg33_k1", "square", 17, 1, 1e-3, 0.01, 100, 0, "taylor_green",
                        FP64, pcg_tol=1e-10),
    # 257x257 fine lid-driven cavity Re=100, coarsening 0..3, both schemes
    **{f"cavity257_k{k}_chi{c}_{p}": Workload(
        f"cavity257_k{k}_chi{c}_{p}", "square", (256 >> k) + 1, k, 5e-3, 0.01, 500, c,
        "cavity", FP64 if p == "fp64" else MIXED, pcg_tol=1e-8)
       for k in range(4) for c in (0, 1) for p in ("fp64", "mixed")},
    # channel minus cylinder, 2 levels, Re=20, rotational, mixed
    "channel_k2": Workload("channel_k2", "channel", 0, 2, 1e-3, 1e-3, 1000, 1, "channel",
                           MIXED, pcg_tol=1e-8),
    # learned-guess cavity (config-2 mesh, k=1 pressure mesh 129x129)
    "cavity257_k1_learned": Workload("cavity257_k1_learned", "square", 129, 1, 5e-3, 0.01,
                                     1000, 0, "cavity", MIXED, pcg_tol=1e-8),
    # the paper's Jobelin vortex in the circle of radius 1/2 (Re = 10, dt = 0.01,
    # t = 1): coarse mesh of 1201 nodes / 2304 triangles (Fig. 1), k = 2.  The
    # projected field is nearly solenoidal (|b_c| ~ 1e-3 |U~|), so the momentum
    # solve runs to 1e-15: at 1e-12 its stopping error is visible in Phi
    **{f"jobelin_disc_chi{c}": Workload(f"jobelin_disc_chi{c}", "disc", 0, 2, 1e-2, 0.1, 100, c,
                                        "jobelin_disc", FP64, pcg_tol=1e-10, mom_tol=1e-15)
       for c in (0, 1)},
    # the paper's Jobelin vortex with an open boundary (Sect. 3.2): unit
    # square, natural (traction) boundary on x = 0, Dirichlet elsewhere,
    # Re = 10, dt = 0.01, t = 1, standard scheme; the paper's finest mesh
    # has 16384 elements and coarsens up to k = 2: 65x65 fine nodes
    # (8192 triangles) here, with the exact solution's forcing and traction
    **{f"jobelin_open_k{k}": Workload(f"jobelin_open_k{k}", "square", (64 >> k) + 1, k, 1e-2,
                                      0.1, 100, 0, "jobelin_open", FP64, pcg_tol=1e-10,
                                      mom_tol=1e-14, natural=("left",))
       for k in range(3)},
    # the paper's Taylor-Green case (Sect. 3.1): Re = 10, dt = 0.00125, t = 1
    # (800 steps), velocity Dirichlet data of the exact solution on every
    # side; 129x129 fine nodes (32768 triangles), coarsening k = 0..3
    **{f"tg_re10_k{k}_chi{c}": Workload(f"tg_re10_k{k}_chi{c}", "square", (128 >> k) + 1, k,
                                        0.00125, 0.1, 800, c, "taylor_green", FP64,
                                        pcg_tol=1e-10)
       for k in range(4) for c in (0, 1)},
    # 2049x2049 Taylor-Green, 3 levels (257x257 pressure mesh), rotational
    "tg2049_k3_fp64": Workload("tg2049_k3_fp64", "square", 257, 3, 2e-4, 0.005, 200, 1,
                               "taylor_green", FP64, pcg_tol=1e-8),
    "tg2049_k3_mixed": Workload("tg2049_k3_mixed", "square", 257, 3, 2e-4, 0.005, 200, 1,
                                "taylor_green", MIXED, pcg_tol=1e-8),
}


def get_workload(name: str) -> Workload:
    return WORKLOADS[name]
