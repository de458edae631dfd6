"""Coarse PCG preconditioned by the nested-dissection Cholesky factor, on the
GPU through the C-ABI, against the oracle's exact coarse solve (the result
that PCG with an exact factor preconditioner reaches): single solves on
pure-Neumann, natural-boundary and unstructured meshes, from zero and from
arbitrary guesses; multi-step trajectories; edge cases (zero right-hand
side, a guess that already converged) and run-to-run reproducibility."""
import numpy as np
import pytest

from oracle.cgp import build as build_oracle
from workloads import get_workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1812_00185_amd import CGP  # noqa: E402

TOL64 = 1e-10


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def make(w):
    w = w.with_(precond="ndchol")
    print(f"\n[case] {w.name} coarse_n={w.coarse_n} k={w.levels} chi={w.chi} ndchol", flush=True)
    g = CGP(w.coarse_mesh(), w.levels, w.dt, w.nu, chi=w.chi, restrict=w.restrict,
            pcg_tol=w.pcg_tol, mom_tol=w.mom_tol, mass_tol=w.mass_tol, max_iter=w.max_iter,
            mass=w.mass, precond="ndchol")
    return w, g, build_oracle(w)


def cavity(n, k, **kw):
    return get_workload("cavity257_k0_chi0_fp64").with_(coarse_n=n, levels=k, **kw)


def channel(k=1, h=0.05, **kw):
    return get_workload("channel_k2").with_(levels=k, channel_h=h, precision=0, **kw)


SOLVE_CASES = [
    ("cavity129_neumann", lambda: cavity(129, 1)),
    ("cavity33_neumann", lambda: cavity(33, 0)),
    ("channel_natural", lambda: channel(1, 0.03)),
    ("disc_neumann", lambda: get_workload("jobelin_disc_chi0")),
]


def compatible_rhs(o, seed):
    b = np.random.default_rng(seed).standard_normal(o.nc)
    b[o.nat_c] = 0.0
    if o.pure_neumann:
        b -= b.mean()
    return b


@pytest.mark.parametrize("name,wf", SOLVE_CASES, ids=[c[0] for c in SOLVE_CASES])
def test_coarse_solve_matches_exact(name, wf):
    w, g, o = make(wf())
    print(f"[case] N_c={g.nc} factor {g.ndchol}", flush=True)
    assert g.ndchol["n_factored"] == o.phi_free.size - (1 if o.pure_neumann else 0)
    for seed, guess in ((1, "zero"), (2, "random")):
        b = compatible_rhs(o, seed)
        x0 = np.zeros(o.nc) if guess == "zero" else np.random.default_rng(seed + 10).standard_normal(o.nc)
        ref, _ = o.poisson(b, x0)
        phi = g.to_device(x0)
        st = g.pcg_solve(g.to_device(b), phi)
        torch.cuda.synchronize()
        d = rel(phi.cpu().numpy(), ref)
        print(f"[result] {name} {guess}: rel diff {d:.3e} stats {st}", flush=True)
        assert st["converged"] and 1 <= st["iters"] <= 2 and st["rel_res"] <= w.pcg_tol
        assert d <= TOL64


def test_zero_rhs_and_converged_guess():
    w, g, o = make(cavity(33, 1))
    phi = g.to_device(np.random.default_rng(0).standard_normal(o.nc))
    st = g.pcg_solve(g.zeros(o.nc), phi)
    assert st["iters"] == 0 and st["converged"]
    assert float(torch.count_nonzero(phi)) == 0
    b = compatible_rhs(o, 4)
    ref, _ = o.poisson(b, np.zeros(o.nc))
    phi = g.to_device(ref)
    st = g.pcg_solve(g.to_device(b), phi)
    assert st["iters"] == 0 and st["converged"]
    assert rel(phi.cpu().numpy(), ref) <= 1e-13


def test_bitwise_reproducible():
    w, g, o = make(cavity(129, 1))
    b = g.to_device(compatible_rhs(o, 9))
    outs = []
    for _ in range(3):
        phi = g.zeros(o.nc)
        g.pcg_solve(b, phi)
        outs.append(phi.cpu().numpy())
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


@pytest.mark.parametrize("name,wf,steps", [
    ("cavity_k1_chi1", lambda: cavity(33, 1, chi=1), 10),
    ("channel_k1_chi1", lambda: channel(1, 0.05, chi=1), 8),
    ("jobelin_chi1", lambda: get_workload("jobelin_disc_chi1"), 6),
])
def test_step_trajectories(name, wf, steps):
    w, g, o = make(wf())
    Um, U0, P0 = w.initial_fields(o.fine_xy)
    so, sg = o.initial_state(Um, U0, P0), g.new_state(Um, U0, P0)
    xyd = o.fine_xy[o.dir]
    worst = 0.0
    for n in range(steps):
        t = (n + 1) * w.dt
        uD, F = w.dirichlet_values(xyd, t), w.forcing(o.fine_xy, t)
        so = o.step(so, uD, F).state
        st = g.step(sg, g.to_device(uD), f=None if F is None else g.to_device(F), stats=True)
        assert st["poisson"]["converged"] and st["poisson"]["iters"] <= 2
        worst = max(worst, rel(sg.U.cpu().numpy(), so.U), rel(sg.P.cpu().numpy(), so.P))
    print(f"[result] {name}: worst relative L2 over {steps} steps {worst:.3e}", flush=True)
    assert worst <= TOL64


# ----------------------------------------------------------------- mixed precision
def make_mixed(w):
    w = w.with_(precond="ndchol", precision=1)
    print(f"\n[case] {w.name} coarse_n={w.coarse_n} k={w.levels} chi={w.chi} ndchol mixed",
          flush=True)
    g = CGP(w.coarse_mesh(), w.levels, w.dt, w.nu, chi=w.chi, restrict=w.restrict,
            pcg_tol=w.pcg_tol, mom_tol=w.mom_tol, mass_tol=w.mass_tol, max_iter=w.max_iter,
            mass=w.mass, precond="ndchol", precision="mixed")
    return w, g, build_oracle(w.with_(precision=0))


@pytest.mark.parametrize("name,wf", SOLVE_CASES, ids=[c[0] for c in SOLVE_CASES])
def test_mixed_refinement_with_fp32_factor(name, wf):
    """FP64 refinement around FP32 factor solves: the FP64 true residual
    (recomputed from the oracle's K_c) meets the tolerance; the solution is
    within kappa x tol of the exact coarse solve (checked against 1e-6); a
    handful of corrections suffice (each removes all but ~kappa eps_32)."""
    w, g, o = make_mixed(wf().with_(pcg_tol=1e-8))
    f = o.phi_free
    for seed, guess in ((1, "zero"), (2, "random")):
        b = compatible_rhs(o, seed)
        x0 = np.zeros(o.nc) if guess == "zero" else np.random.default_rng(seed + 10).standard_normal(o.nc)
        ref, _ = o.poisson(b, x0)
        phi = g.to_device(x0)
        st = g.pcg_solve(g.to_device(b), phi)
        torch.cuda.synchronize()
        x = phi.cpu().numpy()
        true = np.linalg.norm(b[f] - o.Kc_ff @ x[f]) / np.linalg.norm(b[f])
        d = rel(x, ref)
        print(f"[result] {name} {guess}: true rel residual {true:.3e}, vs exact {d:.3e}, "
              f"stats {st}", flush=True)
        assert st["converged"] and 1 <= st["outer_iters"] <= 5
        assert true <= w.pcg_tol and st["rel_res"] <= w.pcg_tol
        assert d <= 1e-6
        assert np.all(x[o.nat_c] == 0.0)


@pytest.mark.parametrize("name,wf,steps", [
    ("cavity_k1_chi1", lambda: cavity(33, 1, chi=1), 10),
    ("channel_k1_chi1", lambda: channel(1, 0.05, chi=1), 8),
])
def test_mixed_step_trajectories(name, wf, steps):
    """Mixed-precision steps with the FP32 factor end to end against the FP64
    oracle (exact coarse solve): within the mixed path's bar, 1e-6."""
    w, g, o = make_mixed(wf().with_(pcg_tol=1e-8))
    Um, U0, P0 = w.initial_fields(o.fine_xy)
    so, sg = o.initial_state(Um, U0, P0), g.new_state(Um, U0, P0)
    xyd = o.fine_xy[o.dir]
    worst = 0.0
    for n in range(steps):
        t = (n + 1) * w.dt
        uD = w.dirichlet_values(xyd, t)
        so = o.step(so, uD).state
        st = g.step(sg, g.to_device(uD), stats=True)
        assert st["poisson"]["converged"] and st["poisson"]["rel_res"] <= w.pcg_tol
        worst = max(worst, rel(sg.U.cpu().numpy(), so.U), rel(sg.P.cpu().numpy(), so.P))
    print(f"[result] {name}: mixed (FP32 factor) vs FP64 oracle, worst over {steps} steps "
          f"{worst:.3e}", flush=True)
    assert worst <= 1e-6
