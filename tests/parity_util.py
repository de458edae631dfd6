"""Helpers shared by the parity tests (not a test module).

The FP64 bar is 1e-10 relative L2 per field.  A multi-step trajectory that is
ill-conditioned cannot agree with any other rounding order of the same
arithmetic to better than the oracle agrees with itself when its solver
right-hand sides carry rounding-level noise; such trajectories are held to
max(1e-10, 10 x that self-sensitivity), measured over the same steps.
"""
from __future__ import annotations

from contextlib import contextmanager
from unittest import mock

import numpy as np

TOL64 = 1e-10
MIXED_BAR = 1e-6


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


@contextmanager
def noisy_oracle_solvers(seed=0, eps=1e-15):
    """Within the block every oracle Krylov solve sees its right-hand side
    multiplied by (1 + eps * N(0, 1)) entrywise."""
    import oracle.cgp as oc

    rng = np.random.default_rng(seed)
    pcg, bicg = oc.pcg_jacobi, oc.bicgstab_jacobi

    def noisy(fn):
        def f(A, b, **kw):
            return fn(A, b * (1 + eps * rng.standard_normal(b.shape)), **kw)
        return f

    with mock.patch.object(oc, "pcg_jacobi", noisy(pcg)), \
            mock.patch.object(oc, "bicgstab_jacobi", noisy(bicg)):
        yield


def oracle_trajectory(w, steps, traction=False, log=None):
    """(U, P) of the oracle after each of `steps` steps of workload w from its
    initial fields (forcing and traction data from the workload)."""
    from oracle.cgp import build as build_oracle

    o = build_oracle(w)
    st = o.initial_state(*w.initial_fields(o.fine_xy))
    out = []
    for n in range(steps):
        t = (n + 1) * w.dt
        st = o.step(st, w.dirichlet_values(o.fine_xy[o.dir], t), w.forcing(o.fine_xy, t),
                    T=w.traction(o.fine_xy, t) if traction else None).state
        out.append((st.U.copy(), st.P.copy()))
        if log:
            log(f"[oracle] {w.name} step {n + 1}/{steps}")
    return out


def oracle_sensitivity(w, steps, clean=None, traction=False, log=None):
    """Largest per-step relative L2 change (u or p) of the oracle's trajectory
    when every solver right-hand side carries 1e-15 relative noise."""
    if clean is None:
        clean = oracle_trajectory(w, steps, traction, log)
    with noisy_oracle_solvers():
        pert = oracle_trajectory(w, steps, traction, log)
    return max(max(rel(a[0], b[0]), rel(a[1], b[1])) for a, b in zip(pert, clean))


def sensitivity_bound(sens):
    return max(TOL64, 10.0 * sens)
