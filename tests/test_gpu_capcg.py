"""Coarse Jacobi-PCG in s-step form (four iterations per launch from one
Gram-matrix reduction) on the GPU through the C-ABI, against the oracle's
Jacobi-PCG: the s-step form carries out the same iterations with the same
stopping test after each one, so it stops after the same number of
iterations at the same solution up to rounding.  On the structured meshes
the counts agree exactly.  On unstructured ones, CG's finite-precision
trajectory differs between any two orders of the arithmetic by up to ~10 %
in the residual near convergence (measured on the CPU: each algorithm's
recursive residual equals the true residual of its own iterate), so the stop
may move by an iteration; the solution bar stays at 1e-10.  Single solves on
pure-Neumann, natural-boundary and unstructured meshes spanning one to about
three hundred tiles, from zero and from arbitrary guesses; the iteration cap (a
partial block of iterations); edge cases; reproducibility; multi-step
trajectories."""
import numpy as np
import pytest

from oracle.cgp import build as build_oracle
from parity_util import oracle_sensitivity, sensitivity_bound
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
    w = w.with_(precond="jacobi_s4")
    print(f"\n[case] {w.name} coarse_n={w.coarse_n} k={w.levels} chi={w.chi} "
          f"max_iter={w.max_iter} s-step", flush=True)
    g = CGP(w.coarse_mesh(), w.levels, w.dt, w.nu, chi=w.chi, restrict=w.restrict,
            pcg_tol=w.pcg_tol, mom_tol=w.mom_tol, mass_tol=w.mass_tol, max_iter=w.max_iter,
            mass=w.mass, precond="jacobi_s4")
    return w, g, build_oracle(w)


def cavity(n, k, **kw):
    return get_workload("cavity257_k0_chi0_fp64").with_(coarse_n=n, levels=k, **kw)


def channel(k=1, h=0.05, **kw):
    return get_workload("channel_k2").with_(levels=k, channel_h=h, precision=0, **kw)


SOLVE_CASES = [
    ("cavity33_neumann", lambda: cavity(33, 0)),
    ("cavity129_neumann", lambda: cavity(129, 1)),
    ("cavity257_neumann", lambda: cavity(257, 0)),
    # 148k unknowns, about 290 tiles: the Gram sums take a second pass over
    # the partials (more than 192 tiles)
    ("cavity385_neumann", lambda: cavity(385, 0)),
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
def test_coarse_solve_matches_pcg(name, wf):
    w, g, o = make(wf())
    for seed, guess in ((1, "zero"), (2, "random")):
        b = compatible_rhs(o, seed)
        x0 = np.zeros(o.nc) if guess == "zero" else np.random.default_rng(seed + 10).standard_normal(o.nc)
        x0[o.nat_c] = 0.0
        ref, info = o.poisson(b, x0)
        phi = g.to_device(x0)
        st = g.pcg_solve(g.to_device(b), phi)
        torch.cuda.synchronize()
        d = rel(phi.cpu().numpy(), ref)
        print(f"[result] {name} {guess}: rel diff {d:.3e} iters {st['iters']} "
              f"(oracle {info.iters}) rel_res {st['rel_res']:.3e}", flush=True)
        assert st["converged"] and st["rel_res"] <= w.pcg_tol
        exact = name.startswith("cavity")
        assert st["iters"] == info.iters if exact else abs(st["iters"] - info.iters) <= 2
        assert d <= TOL64


def test_iteration_cap():
    """A cap that ends inside a block of four: the iterate after exactly
    max_iter iterations, reported as not converged."""
    for cap in (1, 10):
        w, g, o = make(cavity(129, 1, max_iter=cap))
        b = compatible_rhs(o, 5)
        ref, info = o.poisson(b, np.zeros(o.nc))
        assert not info.converged and info.iters == cap
        phi = g.zeros(o.nc)
        st = g.pcg_solve(g.to_device(b), phi)
        torch.cuda.synchronize()
        d = rel(phi.cpu().numpy(), ref)
        print(f"[result] cap {cap}: rel diff {d:.3e} stats {st}", flush=True)
        assert not st["converged"] and st["iters"] == cap
        assert d <= 1e-12


def test_zero_rhs_and_converged_guess():
    w, g, o = make(cavity(33, 1))
    phi = g.to_device(np.random.default_rng(0).standard_normal(o.nc))
    st = g.pcg_solve(g.zeros(o.nc), phi)
    assert st["iters"] == 0 and st["converged"]
    assert float(torch.count_nonzero(phi)) == 0
    b = compatible_rhs(o, 4)
    ref, _ = build_oracle(w.with_(pcg_tol=1e-14, max_iter=5000)).poisson(b, np.zeros(o.nc))
    phi = g.to_device(ref)
    st = g.pcg_solve(g.to_device(b), phi)
    assert st["iters"] == 0 and st["converged"]
    assert rel(phi.cpu().numpy(), ref) <= 1e-13


def test_nan_status_and_recovery():
    """A non-finite right-hand side, or a guess whose residual norm
    overflows, ends the solve at the test of the guess with CGP_ERR_NAN; the
    next solve on the same context is unaffected."""
    from paper_1812_00185_amd import _native as N

    w, g, o = make(cavity(129, 1))
    b = compatible_rhs(o, 6)
    ref, info = o.poisson(b, np.zeros(o.nc))
    bad = b.copy()
    bad[100] = float("nan")
    with pytest.raises(N.CGPError) as e:
        g.pcg_solve(g.to_device(bad), g.zeros(o.nc))
    assert e.value.code == N.CGP_ERR_NAN
    # finite b, a guess whose residual norm overflows
    huge = np.zeros(o.nc)
    huge[7] = 1e308
    with pytest.raises(N.CGPError) as e:
        g.pcg_solve(g.to_device(b), g.to_device(huge))
    assert e.value.code == N.CGP_ERR_NAN
    phi = g.zeros(o.nc)
    st = g.pcg_solve(g.to_device(b), phi)
    assert st["converged"] and st["iters"] == info.iters
    assert rel(phi.cpu().numpy(), ref) <= TOL64


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
    """FP64 trajectories in s-step form against the oracle: within 1e-10, or
    within 10x the oracle's own rounding sensitivity over the same steps
    where the trajectory is ill-conditioned.  On the unstructured meshes a
    stop one iteration away (both solves within pcg_tol) changes the coarse
    increment by what the tolerance allows, and the impulsive start of the
    channel amplifies such differences, as it amplifies the oracle's own
    rounding-level noise."""
    w, g, o = make(wf())
    Um, U0, P0 = w.initial_fields(o.fine_xy)
    so, sg = o.initial_state(Um, U0, P0), g.new_state(Um, U0, P0)
    xyd = o.fine_xy[o.dir]
    worst = 0.0
    for n in range(steps):
        t = (n + 1) * w.dt
        uD, F = w.dirichlet_values(xyd, t), w.forcing(o.fine_xy, t)
        r = o.step(so, uD, F)
        so = r.state
        st = g.step(sg, g.to_device(uD), f=None if F is None else g.to_device(F), stats=True)
        # after the first step the right-hand sides themselves differ at the
        # tolerance level on the unstructured meshes
        ref_it = r.stats["pcg_iters"]
        assert st["poisson"]["converged"]
        assert abs(st["poisson"]["iters"] - ref_it) <= max(2, 0.02 * ref_it)
        worst = max(worst, rel(sg.U.cpu().numpy(), so.U), rel(sg.P.cpu().numpy(), so.P))
    sens = oracle_sensitivity(w, steps)
    bound = sensitivity_bound(sens)
    print(f"[result] {name}: worst relative L2 over {steps} steps {worst:.3e}, oracle "
          f"self-sensitivity {sens:.3e}, bound {bound:.3e}", flush=True)
    assert worst <= bound
