"""What the trained network gains: train the learned guess on the GPU with
the library's own forward/backward/Adam kernels on (b, phi) pairs of plain
runs, then solve a fresh run's coarse problems to the same tolerance from
the plain previous-step guess, from the guarded quadratic extrapolation of
the history (network-free, formed by the library) and from the guarded
network guess.

Lid-driven cavity, 65 x 65 fine nodes, one coarsening level (33 x 33
coarse), lid speeds U[0.5, 1.5] for training, U = 1 for evaluation.
"""
import numpy as np
import pytest

from workloads import get_workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1812_00185_amd import CGP, learned  # noqa: E402


def test_trained_network_reduces_coarse_iterations():
    w = get_workload("cavity257_k1_learned").with_(coarse_n=33, levels=1)
    print(f"\n[case] learned guess cavity coarse 33^2 k=1 tol={w.pcg_tol}", flush=True)
    g = CGP(w.coarse_mesh(), w.levels, w.dt, w.nu, chi=w.chi, precision="fp64",
            pcg_tol=w.pcg_tol)
    gm = CGP(w.coarse_mesh(), w.levels, w.dt, w.nu, chi=w.chi, precision="mixed",
             pcg_tol=w.pcg_tol)
    runs = learned.plain_runs(g, learned.variants(w, 3, seed=0), steps=120)
    theta, losses = learned.train(g, runs, epochs=4, lr=1e-3, seed=0)
    print(f"[result] training loss per epoch {[f'{x:.3e}' for x in losses]}", flush=True)
    assert np.isfinite(losses).all() and losses[-1] < losses[0]
    rec, summ = learned.evaluate(g, gm, theta, w.with_(lid_speed=1.0), steps=120, warm=10)
    print("[result] " + ", ".join(f"{k} {v:.4g}" for k, v in summ.items()), flush=True)
    # every variant reaches the FP64 tolerance on the same right-hand side
    assert summ["max_res_plain"] <= w.pcg_tol
    assert summ["max_res_learned"] <= w.pcg_tol
    assert summ["max_res_learned_mixed"] <= w.pcg_tol
    # same discrete solution up to the solver tolerance
    assert summ["max_diff"] <= 1e-5 and summ["max_diff_mixed"] <= 1e-5
    # the gain over the method without the network: against the previous
    # increment, and against the network-free quadratic extrapolation of the
    # history that the network refines (both guarded, same tolerance)
    assert summ["iters_learned"] <= 0.8 * summ["iters_plain"]
    assert summ["iters_learned"] < summ["iters_extrap"]
    assert summ["accepted"] >= 0.9
    # the same weights, guard and coarse solves with the FP64 Jacobi-PCG in
    # s-step form: the same tolerance, the same iterations (structured mesh)
    gs = CGP(w.coarse_mesh(), w.levels, w.dt, w.nu, chi=w.chi, precision="fp64",
             pcg_tol=w.pcg_tol, precond="jacobi_s4")
    _, s4 = learned.evaluate(gs, gm, theta, w.with_(lid_speed=1.0), steps=120, warm=10)
    print("[result] s-step: " + ", ".join(f"{k} {v:.4g}" for k, v in s4.items()), flush=True)
    assert s4["max_res_plain"] <= w.pcg_tol and s4["max_res_learned"] <= w.pcg_tol
    assert s4["iters_learned"] <= 0.8 * s4["iters_plain"]
    assert abs(s4["iters_plain"] - summ["iters_plain"]) <= 0.02 * summ["iters_plain"]
    assert abs(s4["iters_learned"] - summ["iters_learned"]) <= 0.02 * summ["iters_learned"] + 1
