"""cgp_pcg_solve_noalloc through the C-ABI: the coarse FP64 Jacobi-PCG with
its Krylov vectors in the library's per-GPU scratch array instead of the
context's workspace, for callers that cannot allocate.  Two calls in a row on
two contexts, the second smaller (and with natural-boundary rows, so the
first call's scratch contents lie under and beyond the second's), each
against cgp_pcg_solve on the same context (FP64 bar 1e-10, same iteration
count) and against the oracle's Jacobi-PCG; then the rejections of an
oversized system and of an unsupported solver form."""
import numpy as np
import pytest

from oracle.cgp import build as build_oracle
from parity_util import TOL64, rel
from workloads import get_workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1812_00185_amd import CGP  # noqa: E402
from paper_1812_00185_amd import _native as N  # noqa: E402


def make(w, **kw):
    print(f"\n[case] {w.name} coarse_n={w.coarse_n} k={w.levels} {kw}", flush=True)
    return CGP(w.coarse_mesh(), w.levels, w.dt, w.nu, chi=w.chi, pcg_tol=w.pcg_tol,
               max_iter=w.max_iter, **kw)


def compatible_rhs(o, seed):
    b = np.random.default_rng(seed).standard_normal(o.nc)
    b[o.nat_c] = 0.0
    if o.pure_neumann:
        b -= b.mean()
    return b


def check_against_workspace_solve(w, seed):
    g = make(w)
    o = build_oracle(w)
    b = compatible_rhs(o, seed)
    guess = 1e-2 * np.random.default_rng(seed + 1).standard_normal(o.nc)
    guess[o.nat_c] = 0.0
    ref, info = o.poisson(b, guess)
    bd = g.to_device(b)
    x_ws = g.to_device(guess)
    st_ws = g.pcg_solve(bd, x_ws)
    x_na = g.to_device(guess)
    st_na = g.pcg_solve_noalloc(bd, x_na)
    torch.cuda.synchronize()
    a, c = x_na.cpu().numpy(), x_ws.cpu().numpy()
    d = rel(a, c)
    print(f"[result] N_c={o.nc}: no-alloc vs workspace {d:.3e} (bitwise "
          f"{np.array_equal(a, c)}), iterations {st_na['iters']} / {st_ws['iters']} "
          f"(oracle {info.iters}), vs oracle {rel(a, ref):.3e}", flush=True)
    assert st_na["converged"] and st_ws["converged"]
    assert st_na["iters"] == st_ws["iters"]
    assert d <= TOL64
    assert rel(a, ref) <= TOL64
    return o.nc


def test_noalloc_solve_matches_workspace_solve_twice():
    cav = get_workload("cavity257_k0_chi0_fp64").with_(coarse_n=129, levels=1, pcg_tol=1e-10)
    chan = get_workload("channel_k2").with_(levels=1, channel_h=0.05, precision=0,
                                            pcg_tol=1e-10)
    n1 = check_against_workspace_solve(cav, 31)
    n2 = check_against_workspace_solve(chan, 32)
    assert n2 < n1


def test_noalloc_rejects_oversized_and_unsupported_forms():
    big = get_workload("cavity257_k0_chi0_fp64").with_(coarse_n=363, levels=0)
    g = make(big)
    assert g.nc > 131072
    b = g.zeros(g.nc)
    with pytest.raises(N.CGPError) as e:
        g.pcg_solve_noalloc(b, g.zeros(g.nc))
    assert e.value.code == N.CGP_ERR_WORKSPACE
    del g, b
    small = get_workload("cavity257_k0_chi0_fp64").with_(coarse_n=17, levels=1)
    for kw in (dict(precond="jacobi_s4"), dict(precision="mixed")):
        g = make(small, **kw)
        with pytest.raises(N.CGPError) as e:
            g.pcg_solve_noalloc(g.zeros(g.nc), g.zeros(g.nc))
        assert e.value.code == N.CGP_ERR_INVALID
