"""The learned initial guess on the GPU against the FP64 oracle network.

BF16 MFMA inputs with FP32 accumulation: forward and gradient agree with the
FP64 network within a few BF16 ulps (2^-8) relative; the guard picks the
candidate with the smaller FP64 residual exactly; a guided step still
converges to the solver tolerance.
"""
import numpy as np
import pytest

from oracle import mpnn
from oracle.cgp import build as build_oracle
from workloads import get_workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1812_00185_amd import CGP  # noqa: E402


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def setup(n=17, k=1, seed=0, natural=False):
    w = get_workload("cavity257_k0_chi0_fp64").with_(coarse_n=n, levels=k)
    print(f"\n[case] net coarse_n={n} k={k} seed={seed}", flush=True)
    g = CGP(w.coarse_mesh(), w.levels, w.dt, w.nu, chi=0)
    o = build_oracle(w)
    graph = mpnn.Graph(o.C.xy, o.C.K)
    rng = np.random.default_rng(seed)
    theta = g.net_init(seed).cpu().numpy()
    theta = theta + 0.05 * rng.standard_normal(theta.shape).astype(np.float32)
    th = mpnn.unpack(theta.astype(np.float64))
    th["w"][...] = 0.3 * rng.standard_normal(32)
    theta = np.concatenate([v.ravel() for v in (th[nm] for nm, _ in mpnn.layout())]).astype(np.float32)
    b = rng.standard_normal(o.nc)
    hist = [rng.standard_normal(o.nc) * (0.5 ** j) for j in range(4)]
    return g, o, graph, theta, b, hist


def test_forward_matches_fp64_network():
    g, o, graph, theta, b, hist = setup()
    out = g.net_guess(g.to_device(theta).float(), g.to_device(b), [g.to_device(h) for h in hist])
    torch.cuda.synchronize()
    X, q, s = mpnn.features(graph, b, np.array(hist))
    y_o, _ = mpnn.forward(theta.astype(np.float64), graph, X)
    y_g = (out.cpu().numpy() - q) / s
    err = rel(y_g, y_o)
    print(f"[result] forward relative error {err:.3e} (|y| {np.linalg.norm(y_o):.3e})", flush=True)
    assert err <= 3e-2


def test_gradient_matches_fp64_network():
    g, o, graph, theta, b, hist = setup(seed=1)
    rng = np.random.default_rng(5)
    target = hist[0] + 0.1 * rng.standard_normal(o.nc)
    grad, loss = g.net_grad(g.to_device(theta).float(), g.to_device(b),
                            [g.to_device(h) for h in hist], g.to_device(target))
    torch.cuda.synchronize()
    X, q, s = mpnn.features(graph, b, np.array(hist))
    t = mpnn.target(q, s, target)
    L_o, G_o = mpnn.loss_grad(theta.astype(np.float64), graph, X, t)
    G_g = grad.cpu().numpy().astype(np.float64)
    print(f"[result] loss gpu {loss.item():.6e} oracle {L_o:.6e}; "
          f"gradient relative error {rel(G_g, G_o):.3e}", flush=True)
    assert abs(loss.item() - L_o) <= 2e-2 * L_o
    assert rel(G_g, G_o) <= 5e-2
    P_g, P_o = mpnn.unpack(G_g), mpnn.unpack(G_o)
    for name in ("We", "A0", "B2", "C1", "U1", "v0", "w"):
        assert rel(P_g[name], P_o[name]) <= 8e-2, name


def test_adam_step_and_training_reduces_loss():
    g, o, graph, theta, b, hist = setup(seed=2)
    rng = np.random.default_rng(7)
    target = hist[0] + 0.05 * b
    th = g.to_device(theta).float()
    m = torch.zeros_like(th)
    v = torch.zeros_like(th)
    bd, hd, td = g.to_device(b), [g.to_device(h) for h in hist], g.to_device(target)
    grad, loss0 = g.net_grad(th, bd, hd, td)
    t0 = th.clone()
    g.net_train_step(th, m, v, 1, 1e-3, bd, hd, td)
    torch.cuda.synchronize()
    step = (t0 - th).cpu().numpy()
    gr = grad.cpu().numpy()
    big = np.abs(gr) > 1e-4
    np.testing.assert_allclose(step[big], 1e-3 * np.sign(gr[big]), rtol=1e-3)
    losses = []
    for k in range(2, 200):
        losses.append(g.net_train_step(th, m, v, k, 3e-3, bd, hd, td).item())
    print(f"[result] loss {loss0.item():.4e} -> {losses[-1]:.4e}", flush=True)
    assert losses[-1] < 0.2 * loss0.item()


def test_guard_picks_smaller_residual():
    g, o, graph, theta, b, hist = setup(seed=3)
    f = o.phi_free
    bb = b - b.mean()
    exact = np.zeros(o.nc)
    exact[f], _ = __import__("oracle.krylov", fromlist=["pcg_jacobi"]).pcg_jacobi(
        o.Kc_ff, bb[f], tol=1e-12)
    rng = np.random.default_rng(1)
    good = exact + 1e-3 * rng.standard_normal(o.nc)
    bad = exact + 1e-1 * rng.standard_normal(o.nc)
    for cand, prev, want in ((good, bad, 0), (bad, good, 1)):
        out, chose = g.guess_guard(g.to_device(bb), g.to_device(cand), g.to_device(prev))
        torch.cuda.synchronize()
        assert chose.item() == want
        np.testing.assert_array_equal(out.cpu().numpy(), cand if want == 0 else prev)


def test_learned_step_converges_and_matches_plain_step():
    w = get_workload("cavity257_k0_chi0_fp64").with_(coarse_n=17, levels=1, pcg_tol=1e-10)
    g = CGP(w.coarse_mesh(), w.levels, w.dt, w.nu, chi=0, pcg_tol=w.pcg_tol)
    o = build_oracle(w)
    theta = g.net_init(0)
    Um, U0, P0 = w.initial_fields(o.fine_xy)
    sa, sb = g.new_state(Um, U0, P0), g.new_state(Um, U0, P0)
    xyd = o.fine_xy[o.dir]
    used = 0
    for n in range(6):
        uD = g.to_device(w.dirichlet_values(xyd, (n + 1) * w.dt))
        st_a = g.step(sa, uD, stats=True)
        st_b = g.step(sb, uD, stats=True, theta=theta)
        assert st_a["poisson"]["converged"] and st_b["poisson"]["converged"]
        used += st_b["guess_net"]
        # same discrete problem solved to 1e-10 from two guesses
        assert rel(sb.U.cpu().numpy(), sa.U.cpu().numpy()) <= 1e-7
        assert rel(sb.P.cpu().numpy(), sa.P.cpu().numpy()) <= 1e-6
    print(f"[result] learned guess accepted in {used} of 6 steps", flush=True)
