"""Throughput benchmark of the CGP time step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one full CGP time step (Eqs. 21-26: momentum, restriction, coarse
Poisson solve, prolongation, velocity and pressure correction) of the
2049 x 2049 Taylor-Green workload with 3 coarsening levels (257 x 257 pressure
mesh, rotational form), inputs resident on the GPU.  These forms of the step
run over the same trajectory:
  plain_fp64     FP64 Jacobi-PCG from the previous increment (the paper's step)
  learned_mixed  guarded learned guess + FP32-inner / FP64-refinement PCG
  learned_fp64   guarded learned guess + FP64 PCG
  lumped_p_fp64  plain FP64 with the lumped-mass pressure update (Eq. 27)
  lumped_fp64    plain FP64 with lumped mass in Eqs. 25 and 27 (no mass solves)
  ndchol_fp64    FP64 PCG preconditioned by the nested-dissection Cholesky
                 factor of K_c (one iteration to rounding level)
  ndchol_lumped_fp64  ndchol_fp64 with lumped mass in Eqs. 25 and 27
  s4_fp64        plain_fp64 with the coarse Jacobi-PCG in s-step form (four
                 iterations per launch from one reduction; the same iterates)
  ncgp_fp64      the non-incremental CGP form the paper compares with
                 (no pressure in the momentum equation, P = Phi_f; chi = 0)
  ndchol_mixed   FP64 iterative refinement around FP32 solves with the
                 factor (FP32 storage and accumulation), previous increment
  ndchol_mass32  ndchol_fp64 with the consistent mass solves as FP64
                 refinement around two float-stored Chebyshev solves
  learned_mixed_ndchol  the same from the guarded learned guess
and, for Taylor-Green, each form's error against the exact solution.
The network is first trained on the GPU, with the library's own kernels, on
(b, phi) pairs of plain runs of phase-shifted Taylor-Green flows (other
trajectories than the timed one).  `value` is the throughput in fine
DOF * steps / s (DOF = 3 N_f: u, v, p) of the step with the FP64 coarse
solve preconditioned by the nested-dissection factor and the consistent
mass solves as FP64 refinement around float-stored Chebyshev solves
(ndchol_mass32; every operation in FP64, the mass iterates stored as float;
the problem statement of this workload names no preconditioner;
--main-form picks another form), which matches the FP64 oracle with an
exact coarse solve to 1e-10; the other forms (which agree with it to the
solver tolerance), the coarse-solve time to tolerance of each guess on this
workload and on the 257 x 257 lid-driven cavity with a 129 x 129 pressure
mesh (the learned guess's own workload: trained on lid speeds U[0.5, 1.5],
evaluated on a fresh U = 1 run), the roofline position of the dominant
kernel (HIP events over the timed region), the CPU oracle timed on a bounded
sample (the first --parity-steps steps, configured like the main form), the
parity of the main form (and of the FP64, s-step and mixed forms of the
same oracle configuration) against that oracle prefix at every step and of
every form's first step,
and the other configurations (33 x 33 Taylor-Green, the 257 x 257 cavity at
k = 0..3 in both schemes, plain FP64 and mixed, the channel with the
cylinder, mixed and FP64), each timed and checked against the oracle, are
reported beside it in the same JSON line.
"""
from __future__ import annotations

import argparse
import copy
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fine DOF·steps/s at fixed L2 vs oracle; learned+mixed vs plain PCG time-to-tol"
HBM_PEAK_GBS = 8000.0

# algorithmic bytes per launch of each timed kernel (int32 indices, FP64 values):
# CSR matrix 12 B/nnz + 4 B/row pointer; every vector once.  Arguments: rows n,
# nnz z, right-hand sides nr, coarse triangles t, edges e, vertices v, levels k.
#  mass_spmv:   one Chebyshev step of the fused mass solves after the first.
#               Lattice size 8 (k = 3): over the coarse-edge and vertex nodes
#               (from the node at or below 21 t with an index divisible by 4):
#               per node and rhs b, x_{k-1}, x_k and the new iterate (4
#               values), a Dirichlet flag byte; the values one step inside
#               every coarse triangle along its edges (the 15 ring nodes, one
#               value per rhs); per coarse edge its ends and triangles (16 B);
#               per coarse triangle its area, vertices and edges (32 B); the
#               coarse-vertex rows (2E + V entries of 12 B: FP64 value, lattice
#               column).  Other sizes: over all nodes, with the gathered
#               iterate counted once
#  mass_pair:   lattice size 8: two Chebyshev steps on the interior nodes
#               (21 per coarse triangle): per node and rhs b, x_{k-1}, x_k read
#               and x_{k+1}, x_{k+2} written (5 values), a flag byte; x_k and
#               x_{k+1} at the 7 inner nodes of every coarse edge (2 values per
#               rhs); per coarse triangle its area, vertices and edges (32 B)
#  mass_spmv32, mass_pair32: the same kernels with the iterates and right-
#               hand sides stored as float (the mixed-precision mass solves):
#               4-byte values instead of 8
#  mom_spmv:    BiCGSTAB v = A p^ (2 rhs): p^ read, r^ read, v written (the
#               average includes the launches queued past convergence, which
#               return at once: a bound, not a bandwidth figure)
#  coarse_spmv: one single-reduction PCG iteration: x, p, r, w, s, D^-1 read,
#               x, p, r, w, s written


def _mass_spmv_bytes(n, z, nr, t, e, v, k, vb=8):
    if k != 3:
        return 4 * vb * nr * n + n + 32 * t + 16 * e + 16 * (2 * e + v) + 4 * v
    rng = n - ((21 * t) & ~3)
    return 4 * vb * nr * rng + rng + vb * nr * 15 * t + 16 * e + 32 * t + 12 * (2 * e + v)


def _mass_pair_bytes(n, z, nr, t, e, v, k, vb=8):
    return 21 * t * (5 * vb * nr + 1) + 7 * e * 2 * vb * nr + 32 * t


KERNELS = {
    "mass_spmv": (1, _mass_spmv_bytes),
    "mass_pair": (5, _mass_pair_bytes),
    "mass_spmv32": (1, lambda *a: _mass_spmv_bytes(*a, vb=4)),
    "mass_pair32": (5, lambda *a: _mass_pair_bytes(*a, vb=4)),
    "mom_spmv": (2, lambda n, z, nr, t, e, v, k: 12 * z + 4 * (n + 1) + 3 * 2 * 8 * n),
    "coarse_spmv": (3, lambda n, z, nr, t, e, v, k: 12 * z + 4 * (n + 1) + 11 * 8 * n),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# committed rocprofv3 counter summaries of a timed kernel, per workload, with
# the sources the kernel is compiled from (their hash must match the record's)
TRAFFIC_RECORDS = {
    ("tg2049_k3_fp64", "mass_spmv"): ("k_cheb_lattice3_tg2049_k3_fp64_traffic.md",
                                      ("mass.hip", "lattice.hpp", "cheb2.hpp")),
    ("tg2049_k3_fp64", "mass_pair"): ("k_cheb_pair3_tg2049_k3_fp64_traffic.md",
                                      ("mass.hip", "lattice.hpp", "cheb2.hpp")),
    ("tg2049_k3_fp64", "mass_spmv32"): ("k_cheb_lattice3_f32_tg2049_k3_fp64_traffic.md",
                                        ("mass.hip", "lattice.hpp", "cheb2.hpp")),
    ("tg2049_k3_fp64", "mass_pair32"): ("k_cheb_pair3_f32_tg2049_k3_fp64_traffic.md",
                                        ("mass.hip", "lattice.hpp", "cheb2.hpp")),
    ("sq2049_k0_pcg", "coarse_spmv"): ("k_pcg_iter_sq2049_k0_fp64_traffic.md",
                                       ("kernels.hip",)),
}


def stored_traffic(workload, kernel):
    """Measured HBM bytes per launch (FETCH_SIZE and WRITE_SIZE passes scaled
    by a calibration kernel) from the committed counter summary, or None when
    there is none or the kernels' source has changed since it was taken."""
    rec_entry = TRAFFIC_RECORDS.get((workload, kernel))
    if not rec_entry:
        return None, "no counter summary for this workload and kernel"
    name, sources = rec_entry
    path = os.path.join(ROOT, "profiles", name)
    try:
        text = open(path).read()
        h = hashlib.sha256()
        for f in sources:
            h.update(open(os.path.join(ROOT, "paper_1812_00185_amd", "csrc", f), "rb").read())
        digest = h.hexdigest()
    except OSError as e:
        return None, str(e)
    rec = {}
    for line in text.splitlines():
        if line.startswith("    ") and ": " in line:
            k, v = line.strip().split(": ", 1)
            rec[k] = v
    if rec.get("sources_sha256") != digest:
        return None, "kernels changed since the counters were taken"
    return int(rec["traffic_bytes_per_launch"]), f"profiles/{name}"


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# oracle configuration (mass mode, coarse solver, scheme) matching each form
FORM_MODES = {"ndchol_mixed": ("consistent", "exact", "incremental"),
              "ndchol_mass32": ("consistent", "exact", "incremental"),
              "learned_mixed_ndchol": ("consistent", "exact", "incremental"),
              "lumped_p_fp64": ("lumped_p", "pcg", "incremental"),
              "lumped_fp64": ("lumped", "pcg", "incremental"),
              "ndchol_fp64": ("consistent", "exact", "incremental"),
              "ndchol_lumped_fp64": ("lumped", "exact", "incremental"),
              "ncgp_fp64": ("consistent", "pcg", "nonincremental"),
              "s4_fp64": ("consistent", "pcg", "incremental")}


def cpu_baseline(w, g_fine_xy, first_steps, prefixes, nprefix, main_mode):
    """The oracle (as it stands), single thread, configured like the main
    form (`main_mode`: mass matrices, coarse solver, scheme), over the first
    `nprefix` steps of the same workload from its initial fields: its
    throughput is the CPU baseline, and its states give the parity of the GPU
    forms of that mode that ran the same prefix (every step) and of every
    form's first step (each against the oracle configured like it)."""
    from threadpoolctl import threadpool_limits

    from oracle.cgp import build as build_oracle

    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        ora = build_oracle(w)
        ora.mass_mode, ora.coarse_solver, ora.scheme = main_mode
        t_setup = time.perf_counter() - t0
        st0 = ora.initial_state(*w.initial_fields(ora.fine_xy))
        uD1 = w.dirichlet_values(ora.fine_xy[ora.dir], w.dt)
        states, iters = [], []
        st = st0
        t0 = time.perf_counter()
        for n in range(nprefix):
            r = ora.step(st, w.dirichlet_values(ora.fine_xy[ora.dir], (n + 1) * w.dt))
            st = r.state
            states.append((st.U, st.P))
            iters.append(r.stats["pcg_iters"])
            log(f"[bench] oracle step {n + 1}/{nprefix}")
        t_steps = time.perf_counter() - t0
    assert np.array_equal(ora.fine_xy, g_fine_xy)
    parity = {"pcg_iters_oracle": iters,
              "bar": "1e-10 relative L2 per field (FP64 forms); 1e-6 (mixed)"}
    # every step of the prefix, for the forms that ran it
    for form, traj in prefixes.items():
        per = [(rel(Ug, Uo), rel(Pg, Po)) for (Ug, Pg), (Uo, Po) in zip(traj, states)]
        parity[form + "_prefix"] = {
            "steps": len(per), "u_last": per[-1][0], "p_last": per[-1][1],
            "u_max": max(d[0] for d in per), "p_max": max(d[1] for d in per),
            "oracle": "mass={}, coarse={}, scheme={}".format(*main_mode)}
    # first step of each form against the oracle configured like it (mass
    # matrices of Eqs. 25-27, coarse solver); the operators are shared
    refs = {main_mode: states[0]}
    for form, (U_g, P_g) in first_steps.items():
        mode = FORM_MODES.get(form, ("consistent", "pcg", "incremental"))
        if mode not in refs:
            o2 = copy.copy(ora)
            o2.mass_mode, o2.coarse_solver, o2.scheme = mode
            if o2.scheme == "nonincremental":
                o2.chi = 0
            s2 = o2.step(st0, uD1).state
            refs[mode] = (s2.U, s2.P)
        Uo, Po = refs[mode]
        parity[form] = {"u": rel(U_g, Uo), "p": rel(P_g, Po),
                        "oracle": f"mass={mode[0]}, coarse={mode[1]}, scheme={mode[2]}"}
    dof = 3 * ora.nf
    return {
        "value": dof * nprefix / t_steps, "unit": "DOF*steps/s", "cores": 1, "kind": "oracle",
        "sample": f"the first {nprefix} steps of {w.name} from its initial fields "
                  f"({t_steps:.1f} s; set-up {t_setup:.1f} s untimed), numpy/scipy FP64, "
                  f"1 thread",
        "s_per_step": t_steps / nprefix,
    }, parity


def pcg_calibration(torch, iters, n_side=2049):
    """The coarse PCG iteration kernel at fine scale: the n_side^2 unit square
    with no coarsening, so the Poisson system has all fine nodes (4.2 M rows,
    29.4 M nonzeros at 2049^2) and the iteration streams from HBM instead of
    sitting in cache.  Jacobi-PCG runs `iters` iterations from a zero guess on
    a seeded zero-mean right-hand side (the tolerance is out of reach, so the
    count is fixed); one untimed solve, then one with HIP events around every
    iteration kernel."""
    from paper_1812_00185_amd import CGP
    from workloads import unit_square

    t0 = time.perf_counter()
    g = CGP(unit_square(n_side), 0, 2e-4, 0.005, chi=1, pcg_tol=1e-300, max_iter=iters)
    t_setup = time.perf_counter() - t0
    gen = torch.Generator(device="cuda").manual_seed(0)
    b = torch.randn(g.nc, dtype=torch.float64, device="cuda", generator=gen)
    b -= b.mean()
    x = g.zeros(g.nc)
    g.pcg_solve(b, x)
    x.zero_()
    torch.cuda.synchronize()
    g.timing_enable(KERNELS["coarse_spmv"][0])
    t0 = time.perf_counter()
    st = g.pcg_solve(b, x)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms, nl = g.timing_read()
    g.timing_enable(0)
    nnz = int(g.sizes.nnz_coarse)
    bpl = KERNELS["coarse_spmv"][1](g.nc, nnz, 0, 0, 0, 0, 0)
    avg_s = (kms / 1e3) / max(nl, 1)
    achieved = bpl / avg_s / 1e9
    traffic, src = stored_traffic(f"sq{n_side}_k0_pcg", "coarse_spmv")
    out = {"workload": f"unit square {n_side}x{n_side}, no coarsening, Jacobi-PCG FP64",
           "rows": g.nc, "nnz": nnz, "iterations": st["iters"], "launches": nl,
           "avg_us": avg_s * 1e6, "bytes_per_launch": bpl, "achieved": achieved,
           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
           "traffic": traffic, "traffic_source": src,
           "measured_gbs": (traffic / avg_s / 1e9) if traffic else None,
           "wall_us_per_iteration": 1e6 * wall / max(st["iters"], 1), "set_up_s": t_setup}
    g.close()
    del g, b, x
    torch.cuda.empty_cache()
    return out


def _solver(CGP, w, **over):
    kw = dict(chi=w.chi, restrict=w.restrict, pcg_tol=w.pcg_tol, inner_tol=w.inner_tol,
              mom_tol=w.mom_tol, mass_tol=w.mass_tol, max_iter=w.max_iter, mass=w.mass,
              precond=w.precond, scheme=w.scheme,
              precision="fp64" if w.precision == 0 else "mixed")
    kw.update(over)
    return CGP(w.coarse_mesh(), w.levels, w.dt, w.nu, **kw)


def _leg(torch, CGP, w, steps, warmup, oracle_states, precision):
    """Times `steps` steps after `warmup` of workload w in the given
    precision from its initial fields, and compares the first
    len(oracle_states) steps (run untimed first) with the oracle's."""
    g = _solver(CGP, w, precision=precision)
    Um, U0, P0 = w.initial_fields(g.fine_xy)
    xyd = g.fine_xy[g.dirichlet_nodes]
    total = warmup + steps
    uD = [g.to_device(w.dirichlet_values(xyd, (n + 1) * w.dt)) for n in range(total + 1)]
    out = {"workload": w.name, "precision": precision, "fine_nodes": g.nf,
           "coarse_nodes": g.nc, "levels": w.levels, "chi": w.chi, "pcg_tol": w.pcg_tol}
    if oracle_states:
        sp = g.new_state(Um, U0, P0)
        per = []
        for n, (Uo, Po) in enumerate(oracle_states):
            g.step(sp, uD[n])
            per.append((rel(sp.U.cpu().numpy(), Uo), rel(sp.P.cpu().numpy(), Po)))
        bar = 1e-10 if precision == "fp64" else 1e-6
        out["parity_vs_fp64_oracle"] = {
            "steps": len(per), "u_first": per[0][0], "p_first": per[0][1],
            "u_max": max(d[0] for d in per), "p_max": max(d[1] for d in per),
            "bar": bar, "within_bar": max(max(d) for d in per) <= bar}
        del sp
    el, _, _, st, state = run_form(torch, g, uD, (Um, U0, P0), warmup, steps)
    out.update({"steps": steps, "warmup": warmup, "ms_per_step": 1e3 * el / steps,
                "dof_steps_per_s": 3 * g.nf * steps / el,
                "last_step": {"poisson_iters": st["poisson"]["iters"],
                              "poisson_outer": st["poisson"]["outer_iters"],
                              "momentum_iters": [m["iters"] for m in st["momentum"]]}})
    g.close()
    del g, state, uD
    torch.cuda.empty_cache()
    return out


def config_legs(torch, which, steps, warmup, with_oracle):
    """The other configurations of the problem statement, each in the forms
    it names: 33x33 Taylor-Green (k = 1, FP64 Jacobi-PCG to 1e-10, its whole
    100-step run compared with the oracle); the 257x257 cavity at k = 0..3,
    both schemes, plain FP64 and mixed; the channel with the cylinder
    (k = 2, rotational) mixed and FP64.  Each form is timed over `steps`
    steps after `warmup`; the first step (config 1: every step) is compared
    with the FP64 oracle (bar 1e-10; mixed 1e-6)."""
    from oracle.cgp import build as build_oracle
    from paper_1812_00185_amd import CGP
    from workloads import get_workload

    def oracle_prefix(w, n, noisy=False):
        """The oracle's first n steps; with `noisy` every solver right-hand
        side carries 1e-15 relative noise (its rounding sensitivity)."""
        if not with_oracle:
            return []
        import oracle.cgp as oc

        pcg, bicg = oc.pcg_jacobi, oc.bicgstab_jacobi
        if noisy:
            rng = np.random.default_rng(0)

            def noisy_fn(fn):
                def f(A, b, **kw):
                    return fn(A, b * (1 + 1e-15 * rng.standard_normal(b.shape)), **kw)
                return f
            oc.pcg_jacobi, oc.bicgstab_jacobi = noisy_fn(pcg), noisy_fn(bicg)
        try:
            o = build_oracle(w.with_(precision=0))
            st = o.initial_state(*w.initial_fields(o.fine_xy))
            out = []
            for k in range(n):
                st = o.step(st, w.dirichlet_values(o.fine_xy[o.dir], (k + 1) * w.dt)).state
                out.append((st.U, st.P))
        finally:
            oc.pcg_jacobi, oc.bicgstab_jacobi = pcg, bicg
        return out

    def sensitivity(w, ref):
        """Largest relative change of the oracle's states over the steps of
        ref when its solver right-hand sides carry 1e-15 noise: no other
        rounding order can agree with it more closely."""
        pert = oracle_prefix(w, len(ref), noisy=True)
        return max(max(rel(a[0], b[0]), rel(a[1], b[1])) for a, b in zip(pert, ref))

    def settle(leg, w, ref):
        # FP64 forms: 1e-10, or 10x the oracle's own sensitivity where the
        # trajectory is ill-conditioned (the impulsive channel start)
        par = leg.get("parity_vs_fp64_oracle")
        if par and leg["precision"] == "fp64" and not par["within_bar"]:
            sens = sensitivity(w, ref)
            par["oracle_sensitivity"] = sens
            par["bar"] = max(1e-10, 10 * sens)
            par["within_bar"] = max(par["u_max"], par["p_max"]) <= par["bar"]

    legs = {}
    if "tg33_k1" in which:
        w1 = get_workload("tg33_k1")
        ref1 = oracle_prefix(w1, w1.steps)
        legs["tg33_k1"] = _leg(torch, CGP, w1, w1.steps, 0, ref1, "fp64")
        settle(legs["tg33_k1"], w1, ref1)
        log(f"[bench] config tg33_k1: {json.dumps(legs['tg33_k1'])}")
    for k in (range(4) if "cavity257" in which else ()):
        for chi in (0, 1):
            w = get_workload(f"cavity257_k{k}_chi{chi}_fp64")
            ref = oracle_prefix(w, 1)
            for prec in ("fp64", "mixed"):
                name = f"cavity257_k{k}_chi{chi}_{prec}"
                legs[name] = _leg(torch, CGP, w, steps, warmup, ref, prec)
                settle(legs[name], w, ref)
                log(f"[bench] config {name}: {legs[name]['ms_per_step']:.3f} ms/step")
    w3 = get_workload("channel_k2")
    ref = oracle_prefix(w3, 1) if "channel_k2" in which else []
    for prec in (("mixed", "fp64") if "channel_k2" in which else ()):
        legs[f"channel_k2_{prec}"] = _leg(torch, CGP, w3, steps, warmup, ref, prec)
        settle(legs[f"channel_k2_{prec}"], w3, ref)
        log(f"[bench] config channel_k2_{prec}: "
            f"{legs[f'channel_k2_{prec}']['ms_per_step']:.3f} ms/step")
    return legs


# forms whose consistent mass solves store their iterates as float
MASS32_FORMS = ("ndchol_mass32",)


def main_form_of(args, forms):
    """The form whose throughput is `value`: --main-form if it runs, else
    plain_fp64 if it runs, else the first."""
    if args.main_form in forms:
        return args.main_form
    return "plain_fp64" if "plain_fp64" in forms else forms[0]


def run_form(torch, g, uD, fields, warmup, steps, theta=None, kid=0):
    """W untimed steps, then K timed steps (synchronised on both sides, the
    selected kernel bracketed by HIP events), then one untimed step with
    statistics.  Returns (elapsed s, kernel ms, launches, stats, state)."""
    state = g.new_state(*fields)
    for n in range(warmup):
        g.step(state, uD[n], theta=theta)
    torch.cuda.synchronize()
    if kid:
        g.timing_enable(kid)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for n in range(warmup, warmup + steps):
        g.step(state, uD[n], theta=theta)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kms, nl = g.timing_read() if kid else (0.0, 0)
    g.timing_enable(0)
    st = g.step(state, uD[warmup + steps], theta=theta, stats=True)
    return elapsed, kms, nl, st, state


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="tg2049_k3_fp64")
    ap.add_argument("--learned-workload", default="cavity257_k1_learned")
    ap.add_argument("--learned-runs", type=int, default=4)
    # the learned-guess configuration: 4 runs x 500 steps = 2000 training
    # pairs, then 1000 new steps
    ap.add_argument("--learned-steps", type=int, default=500)
    ap.add_argument("--learned-epochs", type=int, default=3)
    ap.add_argument("--learned-eval", type=int, default=1000)
    ap.add_argument("--timed-kernel", default="mass_spmv", choices=sorted(KERNELS))
    # the timed workload's network: 10 phase-shifted runs x 200 steps = 2000
    # training pairs, as the cavity's
    ap.add_argument("--train-runs", type=int, default=10)
    ap.add_argument("--train-steps", type=int, default=200)
    ap.add_argument("--train-epochs", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--parity-steps", type=int, default=10,
                    help="steps of the trajectory prefix compared with the oracle, every "
                         "step, for the main and the plain form (the oracle run on this "
                         "prefix is also the CPU baseline)")
    ap.add_argument("--config-legs", default="tg33_k1,cavity257,channel_k2",
                    help="the other configurations, each timed and checked against the "
                         "oracle (empty: none)")
    ap.add_argument("--config-steps", type=int, default=30)
    ap.add_argument("--forms",
                    default="plain_fp64,learned_mixed,learned_fp64,lumped_p_fp64,lumped_fp64,"
                            "ndchol_fp64,ndchol_lumped_fp64,ncgp_fp64,s4_fp64,ndchol_mixed,"
                            "learned_mixed_ndchol,ndchol_mass32")
    ap.add_argument("--main-form", default="ndchol_mass32",
                    help="the form whose throughput is `value` (if it runs; else plain_fp64)")
    ap.add_argument("--no-learned", action="store_true",
                    help="the plain FP64 forms only (Jacobi-PCG, standard and s-step): no training, no learned forms or legs")
    ap.add_argument("--pcg-calibration-iters", type=int, default=100,
                    help="iterations of the fine-scale coarse-PCG calibration (0: skip)")
    ap.add_argument("--pcg-calibration-only", action="store_true",
                    help="run only the fine-scale PCG calibration and print it as JSON")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="first run an FP64 scale-by-one kernel over this many MiB (reads "
                         "and writes that many bytes): the reference for HBM counter scaling")
    args = ap.parse_args()
    if args.no_learned:
        args.forms = "plain_fp64,s4_fp64"
        args.learned_workload = ""
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU design is described but not built", file=sys.stderr)
        sys.exit(2)

    import torch

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    from paper_1812_00185_amd import CGP, learned
    from workloads import get_workload

    if args.copy_calibration_mb:
        n = args.copy_calibration_mb * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: 3 x {args.copy_calibration_mb} MiB read + written")
        del src, dst

    if args.pcg_calibration_only:
        print(json.dumps({"calibration": {"pcg_fine_k0": pcg_calibration(
            torch, max(args.pcg_calibration_iters, 1))}}), flush=True)
        return

    w = get_workload(args.workload)
    forms = args.forms.split(",")
    learned_forms = any(f.startswith("learned") for f in forms)
    kw = dict(chi=w.chi, restrict=w.restrict, pcg_tol=w.pcg_tol, inner_tol=w.inner_tol,
              mom_tol=w.mom_tol, mass_tol=w.mass_tol, max_iter=w.max_iter)
    t0 = time.perf_counter()
    g = CGP(w.coarse_mesh(), w.levels, w.dt, w.nu, precision="fp64", **kw)
    gm = CGP(w.coarse_mesh(), w.levels, w.dt, w.nu, precision="mixed", **kw)
    solvers = {"plain_fp64": g, "learned_mixed": gm, "learned_fp64": g}
    # FP64 refinement around FP32 solves with the factor of K_c (the mixed
    # form whose inner solve is not latency bound by its iteration count)
    gmf = None
    if learned_forms or "ndchol_mixed" in forms:
        gmf = CGP(w.coarse_mesh(), w.levels, w.dt, w.nu, precision="mixed", precond="ndchol",
                  **kw)
        solvers["ndchol_mixed"] = gmf
        solvers["learned_mixed_ndchol"] = gmf
    for form, mass, pre in (("lumped_p_fp64", "lumped_p", "jacobi"),
                            ("lumped_fp64", "lumped", "jacobi"),
                            ("ndchol_fp64", "consistent", "ndchol"),
                            ("ndchol_mass32", "mixed", "ndchol"),
                            ("ndchol_lumped_fp64", "lumped", "ndchol"),
                            ("s4_fp64", "consistent", "jacobi_s4")):
        if form in forms:
            solvers[form] = CGP(w.coarse_mesh(), w.levels, w.dt, w.nu, precision="fp64",
                                mass=mass, precond=pre, **kw)
    if "ncgp_fp64" in forms:
        solvers["ncgp_fp64"] = CGP(w.coarse_mesh(), w.levels, w.dt, w.nu, precision="fp64",
                                   scheme="nonincremental", **{**kw, "chi": 0})
    torch.cuda.synchronize()
    log(f"[bench] {w.name}: N_f={g.nf} N_c={g.nc} nnz_f={g.sizes.nnz_fine} "
        f"set-up {time.perf_counter() - t0:.1f} s")

    # --- train the learned guess on other trajectories (phase-shifted flows)
    theta = None
    if learned_forms:
        t0 = time.perf_counter()
        runs = learned.plain_runs(g, learned.variants(w, args.train_runs, seed=0),
                                  args.train_steps)
        torch.cuda.synchronize()
        t_collect = time.perf_counter() - t0
        t0 = time.perf_counter()
        theta, losses = learned.train(g, runs, epochs=args.train_epochs, lr=1e-3, seed=0)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        n_samples = sum(len(r.b) for r in runs)
        del runs
        log(f"[bench] trained on {n_samples} pairs in {t_train:.1f} s (collect "
            f"{t_collect:.1f} s); losses {[round(x, 4) for x in losses]}")
    thetas = {"plain_fp64": None, "learned_mixed": theta, "learned_fp64": theta,
              "lumped_p_fp64": None, "lumped_fp64": None, "ndchol_fp64": None,
              "ndchol_lumped_fp64": None, "ncgp_fp64": None, "s4_fp64": None,
              "ndchol_mixed": None, "learned_mixed_ndchol": theta, "ndchol_mass32": None}

    Um, U0, P0 = w.initial_fields(g.fine_xy)
    xyd = g.fine_xy[g.dirichlet_nodes]
    nsteps = args.warmup + args.steps
    uD = [g.to_device(w.dirichlet_values(xyd, (n + 1) * w.dt)) for n in range(nsteps + 1)]

    # one step of each form from the initial fields for the parity check
    first = {}
    for form in forms:
        s1 = solvers[form].new_state(Um, U0, P0)
        solvers[form].step(s1, uD[0], theta=thetas[form])
        torch.cuda.synchronize()
        first[form] = (s1.U.cpu().numpy(), s1.P.cpu().numpy())
        del s1

    # the mass kernels of a form with float-stored mass iterates
    timed = args.timed_kernel
    mass32 = main_form_of(args, forms) in MASS32_FORMS
    if mass32 and timed in ("mass_spmv", "mass_pair"):
        timed += "32"
    kid = KERNELS[timed][0]
    main_form = main_form_of(args, forms)
    # the main form and the plain step over a prefix of the trajectory, every
    # step kept, for the parity against the oracle over the same prefix
    nprefix = max(1, min(args.parity_steps, nsteps))
    prefixes = {}
    if not args.no_cpu_baseline:
        for form in forms:
            if form != main_form and (form not in ("ndchol_mixed", "s4_fp64", "ndchol_mass32",
                                                   "ndchol_fp64") or
                                      FORM_MODES.get(form) != FORM_MODES.get(main_form)):
                continue
            sp = solvers[form].new_state(Um, U0, P0)
            traj = []
            for n in range(nprefix):
                solvers[form].step(sp, uD[n], theta=thetas[form])
                traj.append((sp.U.cpu().numpy(), sp.P.cpu().numpy()))
            prefixes[form] = traj
            del sp
    results, finals = {}, {}
    for form in forms:
        # the throughput runs carry no per-launch events: those cost host time
        # at every timed launch (the kernel timing runs separately below)
        el, kms, nl, st, state = run_form(torch, solvers[form], uD, (Um, U0, P0),
                                          args.warmup, args.steps, thetas[form], 0)
        results[form] = {"value": 3 * g.nf * args.steps / el,
                         "ms_per_step": 1e3 * el / args.steps, "last_step": st}
        finals[form] = (state.U.cpu().numpy(), state.P.cpu().numpy())
        ex = w.exact(g.fine_xy, (args.warmup + args.steps + 1) * w.dt)
        if ex is not None:
            Ue, Pe = ex
            Pf = finals[form][1]
            results[form]["err_vs_exact"] = {
                "u": rel(finals[form][0], Ue),
                "p": rel(Pf - Pf.mean(), Pe - Pe.mean())}
        log(f"[bench] {form}: {args.steps} steps in {el:.3f} s; last step {st}")
        del state
    ref = finals.get("plain_fp64")
    if ref is not None:
        for form in forms:
            results[form]["vs_plain_fp64_rel_l2"] = {"u": rel(finals[form][0], ref[0]),
                                                     "p": rel(finals[form][1], ref[1])}

    fine_xy = g.fine_xy
    sizes = {"fine_nodes": g.nf, "coarse_nodes": g.nc, "nnz_fine": int(g.sizes.nnz_fine)}
    tc, vc = int(g.sizes.n_coarse_tris), g.nc
    ec = (int(g.sizes.nnz_coarse) - vc) // 2   # the coarse graph holds N + 2E entries

    def kernel_roofline(name, kms, nlaunch):
        """Achieved algorithmic bandwidth of one timed kernel over the timed
        steps (HIP events on the stream it runs on), with the HBM traffic of
        its committed counter record when the sources still match."""
        kid_, kb = KERNELS[name]
        n_rows, nnz = ((g.nc, int(g.sizes.nnz_coarse)) if kid_ == 3
                       else (g.nf, int(g.sizes.nnz_fine)))
        bpl = kb(n_rows, nnz, 3 if w.chi else 2, tc, ec, vc, w.levels)
        avg_s = (kms / 1e3) / max(nlaunch, 1)
        achieved = bpl / avg_s / 1e9 if nlaunch else None
        traffic, traffic_src = stored_traffic(w.name, name)
        return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": traffic,
                "traffic_source": traffic_src, "kernel": name, "form": main_form,
                "launches": nlaunch, "avg_us": avg_s * 1e6, "bytes_per_launch": bpl,
                "ms_per_step": kms / args.steps,
                "measured_gbs": (traffic / avg_s / 1e9) if (traffic and nlaunch) else None}

    # the timed kernel: HIP events around each of its launches, in a run of
    # its own over the same steps
    _, kms1, nl1, _, st1 = run_form(torch, solvers[main_form], uD, (Um, U0, P0), args.warmup,
                                    args.steps, thetas[main_form], kid)
    del st1
    roofs = [kernel_roofline(timed, kms1, nl1)]
    pair = "mass_pair32" if mass32 else "mass_pair"
    if timed in ("mass_spmv", "mass_spmv32") and w.levels == 3:
        # the interior two-step kernel of the same solves, timed in a run of
        # its own over the same steps
        el2, kms2, nl2, _, st2 = run_form(torch, solvers[main_form], uD, (Um, U0, P0),
                                          args.warmup, args.steps, thetas[main_form],
                                          KERNELS[pair][0])
        del st2
        roofs.append(kernel_roofline(pair, kms2, nl2))
    # the contract's object is the kernel with the most time per step
    roofs.sort(key=lambda r: -r["ms_per_step"])
    roofline = dict(roofs[0], others=roofs[1:])

    # coarse-solve time to tolerance along the timed trajectory, every guess
    # solving the same right-hand side to the same FP64 tolerance
    ttt = {}
    if learned_forms:
        extras = [("mixed_factor", gmf, False), ("learned_mixed_factor", gmf, True)]
        if "ndchol_fp64" in solvers:
            extras.insert(0, ("plain_factor", solvers["ndchol_fp64"], False))
        _, tt5 = learned.evaluate(g, gm, theta, w, steps=nsteps, warm=args.warmup,
                                  extras=extras)
        tt5["training"] = {"pairs": n_samples, "epochs": args.train_epochs, "s": t_train,
                           "final_loss": losses[-1]}
        ttt[w.name] = tt5
    del g, gm, gmf, solvers, finals, uD
    torch.cuda.empty_cache()

    # the learned guess on its own workload: cavity, trained on other lid speeds
    if args.learned_workload:
        wl = get_workload(args.learned_workload)
        kl = dict(chi=wl.chi, restrict=wl.restrict, pcg_tol=wl.pcg_tol,
                  inner_tol=wl.inner_tol, mom_tol=wl.mom_tol, mass_tol=wl.mass_tol,
                  max_iter=wl.max_iter)
        gl = CGP(wl.coarse_mesh(), wl.levels, wl.dt, wl.nu, precision="fp64", **kl)
        glm = CGP(wl.coarse_mesh(), wl.levels, wl.dt, wl.nu, precision="mixed", **kl)
        glf = CGP(wl.coarse_mesh(), wl.levels, wl.dt, wl.nu, precision="fp64", precond="ndchol",
                  **kl)
        glmf = CGP(wl.coarse_mesh(), wl.levels, wl.dt, wl.nu, precision="mixed",
                   precond="ndchol", **kl)
        t0 = time.perf_counter()
        runs = learned.plain_runs(gl, learned.variants(wl, args.learned_runs, seed=0),
                                  args.learned_steps)
        t1 = time.perf_counter()
        theta_l, losses_l = learned.train(gl, runs, epochs=args.learned_epochs, lr=1e-3,
                                          seed=0)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        pairs = sum(len(r.b) for r in runs)
        del runs
        _, ttl = learned.evaluate(gl, glm, theta_l, wl.with_(lid_speed=1.0),
                                  steps=args.learned_eval, warm=10,
                                  extras=[("plain_factor", glf, False),
                                          ("mixed_factor", glmf, False),
                                          ("learned_mixed_factor", glmf, True)])
        ttl["training"] = {"pairs": pairs, "epochs": args.learned_epochs,
                           "collect_s": t1 - t0, "s": t2 - t1, "final_loss": losses_l[-1]}
        ttl["config"] = {"fine_nodes": gl.nf, "coarse_nodes": gl.nc, "levels": wl.levels,
                         "pcg_tol": wl.pcg_tol}
        # the same weights with the FP64 Jacobi-PCG in s-step form
        gls = CGP(wl.coarse_mesh(), wl.levels, wl.dt, wl.nu, precision="fp64",
                  precond="jacobi_s4", **kl)
        _, tts = learned.evaluate(gls, glm, theta_l, wl.with_(lid_speed=1.0),
                                  steps=args.learned_eval, warm=10)
        ttl["s_step_fp64"] = {k: tts[k] for k in ("iters_plain", "iters_extrap", "iters_learned",
                                                  "ms_plain", "ms_extrap", "ms_learned",
                                                  "max_res_plain", "max_res_learned", "accepted")}
        ttt[wl.name] = ttl
        log(f"[bench] {wl.name}: {json.dumps(ttl)}")
        del gl, glm, gls, glf, glmf

    calib = None
    if args.pcg_calibration_iters > 0:
        calib = {"pcg_fine_k0": pcg_calibration(torch, args.pcg_calibration_iters)}
        log(f"[bench] PCG calibration: {json.dumps(calib)}")

    legs = None
    if args.config_legs:
        legs = config_legs(torch, set(args.config_legs.split(",")), args.config_steps,
                           args.warmup, not args.no_cpu_baseline)

    cpu, parity = (None, None)
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle sample ...")
        cpu, parity = cpu_baseline(w, fine_xy, first, prefixes, nprefix,
                                   FORM_MODES.get(main_form,
                                                  ("consistent", "pcg", "incremental")))
        del prefixes

    out = {
        "metric": METRIC, "value": results[main_form]["value"], "unit": "DOF*steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": results[main_form]["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32+bf16" if main_form == "learned_mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "form": main_form, **sizes,
                   "levels": w.levels, "dt": w.dt, "nu": w.nu, "chi": w.chi,
                   "restrict": w.restrict, "pcg_tol": w.pcg_tol, "mom_tol": w.mom_tol,
                   "mass_solves": ("FP64 refinement around two float-stored Chebyshev solves "
                                   "(FP64 arithmetic)" if main_form in MASS32_FORMS
                                   else "FP64 Chebyshev")},
        "forms": results, "roofline": roofline, "cpu_baseline": cpu,
        "parity_rel_l2": parity, "time_to_tol": ttt, "calibration": calib,
        "configs": legs,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
