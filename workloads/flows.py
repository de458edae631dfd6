"""Closed-form flow data for the synthetic workloads (input data only).

Initial fields and Dirichlet boundary values, evaluated at whatever node
coordinates the caller supplies.  Nothing here discretises or solves anything.
"""
from __future__ import annotations

import numpy as np

from .meshes import CHANNEL_H


def taylor_green(x, y, t, nu):
    """Taylor-Green vortex (Sect. 3.1, Eqs. 28-30) with 1/Re replaced by nu.

    An exact Navier-Stokes solution with zero forcing on [0,1]^2:
      u = -cos(2 pi x) sin(2 pi y) exp(-8 pi^2 nu t)
      v =  sin(2 pi x) cos(2 pi y) exp(-8 pi^2 nu t)
      p = -(cos(4 pi x) + cos(4 pi y)) / 4 * exp(-16 pi^2 nu t)
    """
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    e = np.exp(-8.0 * np.pi ** 2 * nu * t)
    u = -np.cos(2 * np.pi * x) * np.sin(2 * np.pi * y) * e
    v = np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y) * e
    p = -0.25 * (np.cos(4 * np.pi * x) + np.cos(4 * np.pi * y)) * e * e
    return u, v, p


def cavity_lid(x, y, speed=1.0):
    """Lid-driven cavity wall velocity: (speed, 0) on the lid y = 1 strictly
    between the two top corners, zero on every other wall node (the corners
    belong to the side walls)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    lid = (y == 1.0) & (x > 0.0) & (x < 1.0)
    return np.where(lid, speed, 0.0), np.zeros_like(x)


def channel_inflow(x, y, u_max=0.3):
    """Parabolic inflow 4 U_m y (H - y) / H^2 at x = 0; zero on walls and the
    cylinder (every other Dirichlet node)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    H = CHANNEL_H
    inflow = x == 0.0
    u = np.where(inflow, 4.0 * u_max * y * (H - y) / (H * H), 0.0)
    return u, np.zeros_like(x)


def jobelin_disc(x, y, t):
    """The Jobelin vortex of the paper's circle test (Sect. 3, Dirichlet
    boundary conditions on x^2 + y^2 < 1/4):
      u = sin(x + t) sin(y + t),  v = cos(x + t) cos(y + t),  p = cos(x - y + t),
    divergence free."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    a, b = x + t, y + t
    return np.sin(a) * np.sin(b), np.cos(a) * np.cos(b), np.cos(x - y + t)


def jobelin_disc_forcing(x, y, t, nu):
    """f = u_t + (u . grad) u + grad p - nu lap u for jobelin_disc (derived by
    hand: u_t = sin(a + b), v_t = -sin(a + b), (u . grad) u = sin a cos a,
    (u . grad) v = -sin b cos b, lap u = -2 u, lap v = -2 v with a = x + t,
    b = y + t)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    a, b = x + t, y + t
    s = np.sin(x - y + t)
    fx = np.sin(a + b) + np.sin(a) * np.cos(a) - s + 2.0 * nu * np.sin(a) * np.sin(b)
    fy = -np.sin(a + b) - np.sin(b) * np.cos(b) + s + 2.0 * nu * np.cos(a) * np.cos(b)
    return fx, fy


def jobelin_open(x, y, t):
    """The Jobelin vortex of the paper's open-boundary test (Sect. 3.2,
    Eqs. 31-33) on [0, 1]^2:
      u = sin(x) sin(y + t),  v = cos(x) cos(y + t),  p = cos(x) sin(y + t),
    divergence free."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    b = y + t
    return np.sin(x) * np.sin(b), np.cos(x) * np.cos(b), np.cos(x) * np.sin(b)


def jobelin_open_forcing(x, y, t, nu):
    """f = u_t + (u . grad) u + grad p - nu lap u for jobelin_open (derived by
    hand with b = y + t: u_t = sin x cos b, v_t = -cos x sin b,
    (u . grad) u = sin x cos x, (u . grad) v = -sin b cos b,
    grad p = (-sin x sin b, cos x cos b), lap u = -2 u, lap v = -2 v)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    b = y + t
    fx = (np.sin(x) * np.cos(b) + np.sin(x) * np.cos(x) - np.sin(x) * np.sin(b)
          + 2.0 * nu * np.sin(x) * np.sin(b))
    fy = (-np.cos(x) * np.sin(b) - np.sin(b) * np.cos(b) + np.cos(x) * np.cos(b)
          + 2.0 * nu * np.cos(x) * np.cos(b))
    return fx, fy


_SIDE_NORMALS = {"left": (-1.0, 0.0), "right": (1.0, 0.0), "bottom": (0.0, -1.0),
                 "top": (0.0, 1.0)}


def _on_side(x, y, side):
    return {"left": x == 0.0, "right": x == 1.0, "bottom": y == 0.0, "top": y == 1.0}[side]


def jobelin_open_traction(xy, t, nu, sides):
    """[2, N] traction -p n + nu (grad u) n of jobelin_open at the nodes of
    the given unit-square sides (outward normal n), zero elsewhere.  The
    velocity gradient by hand: u_x = cos x sin b, u_y = sin x cos b,
    v_x = -sin x cos b, v_y = -cos x sin b (b = y + t)."""
    x = np.asarray(xy[:, 0], np.float64)
    y = np.asarray(xy[:, 1], np.float64)
    b = y + t
    p = np.cos(x) * np.sin(b)
    ux, uy = np.cos(x) * np.sin(b), np.sin(x) * np.cos(b)
    vx, vy = -np.sin(x) * np.cos(b), -np.cos(x) * np.sin(b)
    T = np.zeros((2, x.size))
    for side in sides:
        nx, ny = _SIDE_NORMALS[side]
        m = _on_side(x, y, side)
        T[0, m] = (-p * nx + nu * (ux * nx + uy * ny))[m]
        T[1, m] = (-p * ny + nu * (vx * nx + vy * ny))[m]
    return T
