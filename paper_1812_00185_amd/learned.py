"""Training data, training loop and time-to-tolerance evaluation of the
learned initial guess for the coarse Poisson solve.

Orchestration only: every numerical step (time steps, coarse solves, network
forward/backward/Adam, guard) is a call into the HIP library.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from .solver import CGP


@dataclass
class Run:
    """Coarse right-hand sides b[t] and solved increments phi[t] of one
    plain run; sample t uses phi[t-1..t-4] (zeros before the start)."""
    b: list = field(default_factory=list)
    phi: list = field(default_factory=list)

    def sample(self, t, zeros):
        hist = [self.phi[t - k] if t - k >= 0 else zeros for k in range(1, 5)]
        return self.b[t], hist, self.phi[t]


def _advance(g: CGP, U_prev, U, P, uD, phi_guess, record=None):
    """One step through the composed entry points; returns the new fields and
    the solved increment (and appends (b, phi) to `record`)."""
    Ut, _ = g.momentum(U_prev, U, P, uD)
    b = g.restrict(Ut)
    phi = phi_guess.clone()
    st = g.pcg_solve(b, phi)
    phif = g.prolong(phi)
    U_new, P_new, _ = g.correct(Ut, phif, P)
    if record is not None:
        record.b.append(b)
        record.phi.append(phi)
    return U_new, P_new, phi, b, Ut, st


def variants(workload, n_runs, seed=0, speed_range=(0.5, 1.5)):
    """Seeded training variants of a workload: lid speeds drawn uniformly
    from speed_range for the cavity, phase shifts (x0, y0) ~ U[0, 1)^2 for
    Taylor-Green (translated exact solutions); other flows repeat as is."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_runs):
        if workload.flow == "cavity":
            out.append(workload.with_(lid_speed=float(rng.uniform(*speed_range))))
        elif workload.flow == "taylor_green":
            out.append(workload.with_(phase=tuple(float(v) for v in rng.uniform(0, 1, 2))))
        else:
            out.append(workload)
    return out


def plain_runs(g: CGP, workloads, steps):
    """One plain run of `steps` steps per workload (same mesh as g) from its
    initial fields, recording (b, phi) of every step."""
    runs = []
    xyd = g.fine_xy[g.dirichlet_nodes]
    for w in workloads:
        Um, U0, P0 = w.initial_fields(g.fine_xy)
        U_prev, U, P = g.to_device(Um), g.to_device(U0), g.to_device(P0)
        phi = g.zeros(g.nc)
        run = Run()
        for n in range(steps):
            uD = g.to_device(w.dirichlet_values(xyd, (n + 1) * w.dt))
            U_new, P, phi, *_ = _advance(g, U_prev, U, P, uD, phi, run)
            U_prev, U = U, U_new
        runs.append(run)
    return runs


def train(g: CGP, runs, epochs=8, lr=1e-3, seed=0, log=None, skip=4):
    """Adam on single-sample steps over shuffled (run, step) pairs with a full
    history (step >= skip; the guard covers the first steps of a run); the
    learning rate decays linearly to lr/10.  Returns (theta, losses)."""
    import torch

    theta = g.net_init(seed)
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    zeros = g.zeros(g.nc)
    pairs = [(r, t) for r in range(len(runs)) for t in range(skip, len(runs[r].b))]
    rng = np.random.default_rng(seed)
    total = epochs * len(pairs)
    step = 0
    losses = []
    loss = torch.empty(1, dtype=torch.float32, device=g.device)
    for ep in range(epochs):
        order = rng.permutation(len(pairs))
        acc = torch.zeros(1, dtype=torch.float32, device=g.device)
        for k in order:
            r, t = pairs[k]
            b, hist, target = runs[r].sample(t, zeros)
            step += 1
            lr_k = lr * (1.0 - 0.9 * step / total)
            g.net_train_step(theta, m, v, step, lr_k, b, hist, target, loss)
            acc += loss
        losses.append(acc.item() / len(pairs))
        if log:
            log(f"[learned] epoch {ep + 1}/{epochs} mean loss {losses[-1]:.4e}")
    return theta, losses


def evaluate(g: CGP, gm: CGP, theta, workload, steps, seed=1, warm=10, extras=()):
    """Time to tolerance of the coarse solve along a fresh run, four ways on
    the same right-hand side and to the same FP64 tolerance: plain FP64 PCG
    from the previous increment (solver g); the guarded quadratic
    extrapolation 3 phi^n - 3 phi^{n-1} + phi^{n-2} with FP64 PCG (a
    network-free point of comparison); the guarded learned guess with FP64
    PCG (g); and the guarded learned guess with mixed-precision refinement
    (solver gm, same mesh).  `extras`: further (name, solver, use_net)
    solvers on the same mesh, each solving the same right-hand side from the
    guarded learned guess (use_net) or from the previous increment, reported
    as iters_<name> and ms_<name>.  The run advances with the plain
    solution.  Returns per-step records and means over the steps after
    `warm`."""
    import torch

    xyd = g.fine_xy[g.dirichlet_nodes]
    Um, U0, P0 = workload.initial_fields(g.fine_xy)
    U_prev, U, P = g.to_device(Um), g.to_device(U0), g.to_device(P0)
    zeros = g.zeros(g.nc)
    phis = []
    rec = []

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, 1e3 * (time.perf_counter() - t0)

    def learned_solve(solver):
        cand = solver.net_guess(theta, b, hist)
        phi, chose = solver.guess_guard(b, cand, hist[0])
        st = solver.pcg_solve(b, phi)
        return phi, chose, st

    def extrap_solve():
        q = g.extrapolate(hist)
        phi, chose = g.guess_guard(b, q, hist[0])
        return g.pcg_solve(b, phi), chose

    for n in range(steps):
        uD = g.to_device(workload.dirichlet_values(xyd, (n + 1) * workload.dt))
        Ut, _ = g.momentum(U_prev, U, P, uD)
        b = g.restrict(Ut)
        hist = [phis[-k] if len(phis) >= k else zeros for k in range(1, 5)]
        phi_a = hist[0].clone()
        st_a, ms_a = timed(lambda: g.pcg_solve(b, phi_a))
        (st_q, chose_q), ms_q = timed(extrap_solve)
        (phi_b, chose, st_b), ms_b = timed(lambda: learned_solve(g))
        (phi_c, _, st_c), ms_c = timed(lambda: learned_solve(gm))
        extra_rec = {}
        for name, solver, use_net in extras:
            if use_net:
                (_, _, st_e), ms_e = timed(lambda: learned_solve(solver))
            else:
                phi_e = hist[0].clone()
                st_e, ms_e = timed(lambda: solver.pcg_solve(b, phi_e))
            extra_rec[f"iters_{name}"] = st_e["iters"]
            extra_rec[f"ms_{name}"] = ms_e
            extra_rec[f"res_{name}"] = st_e["rel_res"]
        na = torch.linalg.norm(phi_a)
        rec.append(dict(**extra_rec, iters_plain=st_a["iters"], iters_extrap=st_q["iters"],
                        ms_extrap=ms_q,
                        iters_learned=st_b["iters"],
                        iters_learned_mixed=st_c["iters"], outer=st_c["outer_iters"],
                        ms_plain=ms_a, ms_learned=ms_b, ms_learned_mixed=ms_c,
                        accepted=int(chose.item() == 0),
                        accepted_extrap=int(chose_q.item() == 0), res_plain=st_a["rel_res"],
                        res_learned=st_b["rel_res"], res_learned_mixed=st_c["rel_res"],
                        diff=float(torch.linalg.norm(phi_b - phi_a) / na),
                        diff_mixed=float(torch.linalg.norm(phi_c - phi_a) / na)))
        phif = g.prolong(phi_a)
        U_new, P, _ = g.correct(Ut, phif, P)
        U_prev, U = U, U_new
        phis.append(phi_a)
    tail = rec[warm:] if len(rec) > warm else rec
    keys = ("iters_plain", "iters_extrap", "iters_learned", "iters_learned_mixed", "ms_plain",
            "ms_extrap", "ms_learned", "ms_learned_mixed", "accepted", "accepted_extrap")
    keys = keys + tuple(f"{p}_{name}" for name, _, _ in extras for p in ("iters", "ms"))
    summary = {k: float(np.mean([r[k] for r in tail])) for k in keys}
    summary["steps"] = len(tail)
    for k in ("res_plain", "res_learned", "res_learned_mixed", "diff", "diff_mixed") + tuple(
            f"res_{name}" for name, _, _ in extras):
        summary["max_" + k] = float(max(r[k] for r in tail))
    return rec, summary
