"""Pins of the synthetic input data: the Taylor-Green fields (shifted or not)
solve the incompressible Navier-Stokes equations (Eqs. 1-2 with zero
forcing), checked by central differences; boundary data of the cavity and
the channel."""
import numpy as np
import pytest

from workloads import flows, get_workload
from workloads.meshes import CHANNEL_H


@pytest.mark.parametrize("phase", [(0.0, 0.0), (0.31, 0.77)])
def test_taylor_green_solves_navier_stokes(phase):
    w = get_workload("tg2049_k3_fp64").with_(phase=phase)
    nu = w.nu
    rng = np.random.default_rng(0)
    pts = rng.uniform(0, 1, size=(50, 2))
    t, h = 0.37, 1e-4

    def fields(xy, tt):
        (u, v), p = w.exact(xy, tt)
        return u, v, p

    def d(f, k, tt=t):
        e = np.zeros(2)
        e[k] = h
        a, b = fields(pts + e, tt), fields(pts - e, tt)
        return [(ai - bi) / (2 * h) for ai, bi in zip(a, b)]

    def lap(tt=t):
        c = fields(pts, tt)
        out = [np.zeros(len(pts)) for _ in range(3)]
        for k in range(2):
            e = np.zeros(2)
            e[k] = h
            a, b = fields(pts + e, tt), fields(pts - e, tt)
            for i in range(3):
                out[i] += (a[i] - 2 * c[i] + b[i]) / (h * h)
        return out

    u, v, p = fields(pts, t)
    ux, vx, px = d(fields, 0)
    uy, vy, py = d(fields, 1)
    fp, fm = fields(pts, t + h), fields(pts, t - h)
    ut, vt = (fp[0] - fm[0]) / (2 * h), (fp[1] - fm[1]) / (2 * h)
    lu, lv, _ = lap()
    np.testing.assert_allclose(ux + vy, 0.0, atol=1e-7)
    np.testing.assert_allclose(ut + u * ux + v * uy + px - nu * lu, 0.0, atol=1e-5)
    np.testing.assert_allclose(vt + u * vx + v * vy + py - nu * lv, 0.0, atol=1e-5)


def test_phase_shift_translates_the_fields():
    w0 = get_workload("tg33_k1")
    w1 = w0.with_(phase=(0.25, 0.5))
    xy = np.random.default_rng(1).uniform(0, 1, size=(20, 2))
    (U1, P1), (U0, P0) = w1.exact(xy + [0.25, 0.5], 0.1), w0.exact(xy, 0.1)
    np.testing.assert_allclose(U1, U0, atol=1e-14)
    np.testing.assert_allclose(P1, P0, atol=1e-14)
    np.testing.assert_allclose(w1.dirichlet_values(xy + [0.25, 0.5], 0.1), U0, atol=1e-14)


def test_boundary_data():
    x = np.array([0.0, 0.5, 1.0, 0.5])
    y = np.array([1.0, 1.0, 1.0, 0.0])
    u, v = flows.cavity_lid(x, y, 1.5)
    np.testing.assert_array_equal(u, [0.0, 1.5, 0.0, 0.0])
    np.testing.assert_array_equal(v, 0.0)
    yy = np.linspace(0, CHANNEL_H, 1001)
    u, v = flows.channel_inflow(np.zeros(1001), yy, 0.3)
    assert u[500] == pytest.approx(0.3, rel=1e-12) and u[0] == 0
    assert u[-1] == pytest.approx(0, abs=1e-15)
    # mean inflow 2/3 U_m (Simpson's rule is exact for the parabola)
    mean = (yy[1] - yy[0]) / 3 * (u[0] + u[-1] + 4 * u[1:-1:2].sum() + 2 * u[2:-1:2].sum())
    assert mean / CHANNEL_H == pytest.approx(0.2, rel=1e-12)


def test_jobelin_disc_forcing_balances_navier_stokes():
    """The hand-derived forcing of the Jobelin vortex: u_t + (u . grad) u +
    grad p - nu lap u - f = 0 and div u = 0 by central differences."""
    w = get_workload("jobelin_disc_chi0")
    nu, t, h = w.nu, 0.43, 1e-4
    ang = np.random.default_rng(3).uniform(0, 2 * np.pi, 40)
    rad = 0.45 * np.sqrt(np.random.default_rng(4).uniform(0, 1, 40))
    pts = np.stack([rad * np.cos(ang), rad * np.sin(ang)], axis=1)

    def F(xy, tt):
        (u, v), p = w.exact(xy, tt)
        return u, v, p

    ex, ey = np.array([h, 0.0]), np.array([0.0, h])
    c = F(pts, t)
    px, mx, py, my = F(pts + ex, t), F(pts - ex, t), F(pts + ey, t), F(pts - ey, t)
    tp, tm = F(pts, t + h), F(pts, t - h)
    d = lambda a, b: [(ai - bi) / (2 * h) for ai, bi in zip(a, b)]  # noqa: E731
    ux, vx, pxx = d(px, mx)
    uy, vy, pyy = d(py, my)
    ut, vt, _ = d(tp, tm)
    lap = [(px[i] + mx[i] + py[i] + my[i] - 4 * c[i]) / h ** 2 for i in range(2)]
    fx, fy = w.forcing(pts, t)
    u, v = c[0], c[1]
    np.testing.assert_allclose(ux + vy, 0.0, atol=1e-7)
    np.testing.assert_allclose(ut + u * ux + v * uy + pxx - nu * lap[0] - fx, 0.0, atol=1e-5)
    np.testing.assert_allclose(vt + u * vx + v * vy + pyy - nu * lap[1] - fy, 0.0, atol=1e-5)


def test_jobelin_open_forcing_and_traction():
    """The open-boundary Jobelin vortex (Sect. 3.2): the hand-derived forcing
    balances the Navier-Stokes equations and the traction equals
    -p n + nu (grad u) n on x = 0 (n = (-1, 0)), both by central differences;
    the traction is zero away from the natural side."""
    w = get_workload("jobelin_open_k0")
    nu, t, h = w.nu, 0.37, 1e-4
    pts = np.random.default_rng(5).uniform(0.05, 0.95, (40, 2))

    def F(xy, tt):
        (u, v), p = w.exact(xy, tt)
        return u, v, p

    ex, ey = np.array([h, 0.0]), np.array([0.0, h])
    c = F(pts, t)
    px, mx, py, my = F(pts + ex, t), F(pts - ex, t), F(pts + ey, t), F(pts - ey, t)
    tp, tm = F(pts, t + h), F(pts, t - h)
    d = lambda a, b: [(ai - bi) / (2 * h) for ai, bi in zip(a, b)]  # noqa: E731
    ux, vx, pxx = d(px, mx)
    uy, vy, pyy = d(py, my)
    ut, vt, _ = d(tp, tm)
    lap = [(px[i] + mx[i] + py[i] + my[i] - 4 * c[i]) / h ** 2 for i in range(2)]
    fx, fy = w.forcing(pts, t)
    u, v = c[0], c[1]
    np.testing.assert_allclose(ux + vy, 0.0, atol=1e-7)
    np.testing.assert_allclose(ut + u * ux + v * uy + pxx - nu * lap[0] - fx, 0.0, atol=1e-5)
    np.testing.assert_allclose(vt + u * vx + v * vy + pyy - nu * lap[1] - fy, 0.0, atol=1e-5)
    # traction on x = 0 from one-sided differences into the domain
    side = np.stack([np.zeros(15), np.linspace(0, 1, 15)], axis=1)
    inner = side + ex
    inner2 = side + 2 * ex
    a0, a1, a2 = F(side, t), F(inner, t), F(inner2, t)
    dudx = [(-3 * a0[i] + 4 * a1[i] - a2[i]) / (2 * h) for i in range(2)]
    T = w.traction(side, t)
    np.testing.assert_allclose(T[0], a0[2] - nu * dudx[0], atol=1e-6)   # -p(-1) + nu u_x(-1)
    np.testing.assert_allclose(T[1], -nu * dudx[1], atol=1e-6)
    assert np.all(w.traction(pts, t) == 0.0)
    # the literal homogeneous condition of Eq. 34 does not hold for this flow
    assert np.abs(T[0]).max() > 0.5
    m = w.coarse_mesh()
    assert set(np.unique(m["btag"])) == {1, 2}
    nat = m["bedge"][m["btag"] == 2]
    assert np.all(m["xy"][nat.ravel(), 0] == 0.0)
