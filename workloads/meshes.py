"""Seeded synthetic coarse meshes (input data only).

These generators produce the *coarse* (pressure) triangle meshes that both the
HIP library and the CPU oracle take as input.  They hold none of the method's
arithmetic: no refinement, no finite-element assembly, no solver.  Each mesh is
a dict with

  xy    float64 [n_nodes, 2]  node coordinates
  tri   int32   [n_tris, 3]   counter-clockwise vertex triples
  bedge int32   [n_bedges, 2] boundary edges
  btag  int32   [n_bedges]    DIRICHLET (velocity prescribed) or NATURAL
                              (traction-free outflow, phi = 0)
"""
from __future__ import annotations

import numpy as np

DIRICHLET = 1
NATURAL = 2


def unit_square(n: int, tags=None) -> dict:
    """Structured right-triangle mesh of [0,1]^2 with n x n nodes.

    Node (i, j) sits at (i/(n-1), j/(n-1)) with index j*n + i.  Every square
    cell is split by its diagonal from (i+1, j) to (i, j+1); this orientation is
    reproduced exactly by uniform 4:1 refinement, so refined meshes are the
    structured meshes with 2n-1 nodes per side.

    tags: mapping side -> tag for sides 'bottom', 'right', 'top', 'left'
          (default: all DIRICHLET).
    """
    if n < 2:
        raise ValueError("unit_square needs n >= 2")
    tags = dict(tags or {})
    side_tag = {s: tags.get(s, DIRICHLET) for s in ("bottom", "right", "top", "left")}
    s = np.linspace(0.0, 1.0, n)
    X, Y = np.meshgrid(s, s, indexing="xy")          # X[j, i] = s[i]
    xy = np.stack([X.ravel(), Y.ravel()], axis=1)
    i, j = np.meshgrid(np.arange(n - 1), np.arange(n - 1), indexing="xy")
    i = i.ravel()
    j = j.ravel()
    n00 = j * n + i
    n10 = j * n + i + 1
    n01 = (j + 1) * n + i
    n11 = (j + 1) * n + i + 1
    lower = np.stack([n00, n10, n01], axis=1)
    upper = np.stack([n10, n11, n01], axis=1)
    tri = np.empty((2 * len(n00), 3), dtype=np.int64)
    tri[0::2] = lower
    tri[1::2] = upper
    k = np.arange(n - 1)
    bottom = np.stack([k, k + 1], axis=1)
    right = np.stack([k * n + (n - 1), (k + 1) * n + (n - 1)], axis=1)
    top = np.stack([(n - 1) * n + k + 1, (n - 1) * n + k], axis=1)
    left = np.stack([(k + 1) * n, k * n], axis=1)
    bedge = np.concatenate([bottom, right, top, left])
    btag = np.concatenate([np.full(n - 1, side_tag[s])
                           for s in ("bottom", "right", "top", "left")])
    return dict(xy=xy.astype(np.float64), tri=tri.astype(np.int32),
                bedge=bedge.astype(np.int32), btag=btag.astype(np.int32))


CHANNEL_L = 2.2
CHANNEL_H = 0.41
CYL_C = (0.2, 0.2)
CYL_R = 0.05


def channel_cylinder(h: float = 0.0082, seed: int = 0) -> dict:
    """Seeded Delaunay mesh of the channel [0, 2.2] x [0, 0.41] minus the disc
    of radius 0.05 centred at (0.2, 0.2).

    Boundary points are equally spaced (spacing ~h) on the four walls and the
    circle; interior points form a hexagonal lattice of spacing h with a seeded
    jitter of +-0.15h, kept at least 0.5h away from every boundary.  A ring of
    ghost points outside the rectangle makes every wall point a triangulation
    vertex; triangles whose centroid is outside the channel or inside the disc
    are dropped.  Tags: inflow (x=0), walls and cylinder DIRICHLET, outflow
    (x=2.2) NATURAL.
    """
    from scipy.spatial import Delaunay

    rng = np.random.default_rng(seed)
    L, H = CHANNEL_L, CHANNEL_H
    cx, cy = CYL_C
    r = CYL_R

    nx = int(round(L / h))
    ny = int(round(H / h))
    xs = np.linspace(0.0, L, nx + 1)
    ys = np.linspace(0.0, H, ny + 1)
    # rectangle boundary, counter-clockwise, corners once
    bottom = np.stack([xs, np.zeros_like(xs)], 1)
    right = np.stack([np.full(ny - 1, L), ys[1:-1]], 1)
    top = np.stack([xs[::-1], np.full_like(xs, H)], 1)
    left = np.stack([np.zeros(ny - 1), ys[1:-1][::-1]], 1)
    rect = np.concatenate([bottom, right, top, left])
    ncirc = int(round(2 * np.pi * r / h))
    th = np.linspace(0.0, 2 * np.pi, ncirc, endpoint=False)
    circ = np.stack([cx + r * np.cos(th), cy + r * np.sin(th)], 1)

    # interior hexagonal lattice with jitter
    dy = h * np.sqrt(3) / 2
    rows = np.arange(0.0, H + dy, dy)
    pts = []
    for k, yv in enumerate(rows):
        off = 0.5 * h if (k % 2) else 0.0
        xv = np.arange(off, L + h, h)
        pts.append(np.stack([xv, np.full_like(xv, yv)], 1))
    lat = np.concatenate(pts)
    lat = lat + rng.uniform(-0.15 * h, 0.15 * h, size=lat.shape)
    keep = ((lat[:, 0] > 0.5 * h) & (lat[:, 0] < L - 0.5 * h)
            & (lat[:, 1] > 0.5 * h) & (lat[:, 1] < H - 0.5 * h)
            & (np.hypot(lat[:, 0] - cx, lat[:, 1] - cy) > r + 0.5 * h))
    lat = lat[keep]

    # ghost ring outside the rectangle (removed after triangulation)
    gx = np.arange(-h, L + 2 * h, h)
    gy = np.arange(0.0, H + h, h)
    ghost = np.concatenate([
        np.stack([gx, np.full_like(gx, -h)], 1),
        np.stack([gx, np.full_like(gx, H + h)], 1),
        np.stack([np.full_like(gy, -h), gy], 1),
        np.stack([np.full_like(gy, L + h), gy], 1),
    ])

    nb = len(rect) + len(circ)
    allp = np.concatenate([rect, circ, lat, ghost])
    dt = Delaunay(allp)
    tri = dt.simplices.astype(np.int64)
    nreal = nb + len(lat)
    cen = allp[tri].mean(axis=1)
    inside = ((cen[:, 0] > 0) & (cen[:, 0] < L) & (cen[:, 1] > 0) & (cen[:, 1] < H)
              & (np.hypot(cen[:, 0] - cx, cen[:, 1] - cy) > r)
              & np.all(tri < nreal, axis=1))
    tri = tri[inside]
    xy = allp[:nreal]
    # counter-clockwise orientation
    a, b, c = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]
    det = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (c[:, 0] - a[:, 0]) * (b[:, 1] - a[:, 1])
    flip = det < 0
    tri[flip] = tri[flip][:, [0, 2, 1]]

    # boundary edges: rectangle walls (ccw around the domain), circle (cw as
    # seen from the cylinder centre, i.e. the domain lies to the left)
    nr = len(rect)
    redges = np.stack([np.arange(nr), (np.arange(nr) + 1) % nr], 1)
    cedges = np.stack([nr + (np.arange(ncirc) + 1) % ncirc, nr + np.arange(ncirc)], 1)
    bedge = np.concatenate([redges, cedges])
    mid = 0.5 * (xy[bedge[:, 0]] + xy[bedge[:, 1]])
    btag = np.full(len(bedge), DIRICHLET, dtype=np.int64)
    btag[np.isclose(mid[:, 0], L) & (np.arange(len(bedge)) < nr)] = NATURAL

    # compact: drop unreferenced nodes (none expected) and verify edges exist
    used = np.zeros(len(xy), bool)
    used[tri.ravel()] = True
    if not used.all():
        remap = -np.ones(len(xy), np.int64)
        remap[used] = np.arange(used.sum())
        xy = xy[used]
        tri = remap[tri]
        bedge = remap[bedge]
        if (bedge < 0).any():
            raise RuntimeError("boundary point lost by the triangulation")
    edges = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    key = set(map(tuple, np.sort(edges, 1).tolist()))
    missing = [e for e in np.sort(bedge, 1).tolist() if tuple(e) not in key]
    if missing:
        raise RuntimeError(f"{len(missing)} boundary segments missing from the triangulation")
    return dict(xy=xy.astype(np.float64), tri=tri.astype(np.int32),
                bedge=bedge.astype(np.int32), btag=btag.astype(np.int32))


def disc(n_boundary: int = 96, n_interior: int = 1105, radius: float = 0.5,
         seed: int = 0) -> dict:
    """Seeded Delaunay mesh of the disc x^2 + y^2 < radius^2: n_boundary equally
    spaced circle points plus n_interior interior points drawn uniformly
    (rejection sampling, kept 0.3 spacings inside the circle).  All boundary
    edges are tagged DIRICHLET.  Because the point set is in convex position
    on the circle, the triangulation has 2 (n_boundary + n_interior) -
    n_boundary - 2 triangles."""
    from scipy.spatial import Delaunay

    rng = np.random.default_rng(seed)
    th = 2 * np.pi * np.arange(n_boundary) / n_boundary
    bnd = radius * np.stack([np.cos(th), np.sin(th)], 1)
    spacing = 2 * np.pi * radius / n_boundary
    rmax = radius - 0.3 * spacing
    pts = []
    while sum(len(p) for p in pts) < n_interior:
        cand = rng.uniform(-rmax, rmax, size=(2 * n_interior, 2))
        pts.append(cand[np.hypot(cand[:, 0], cand[:, 1]) < rmax])
    inner = np.concatenate(pts)[:n_interior]
    xy = np.concatenate([bnd, inner])
    tri = Delaunay(xy).simplices.astype(np.int64)
    a, b, c = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]
    det = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (c[:, 0] - a[:, 0]) * (b[:, 1] - a[:, 1])
    flip = det < 0
    tri[flip] = tri[flip][:, [0, 2, 1]]
    k = np.arange(n_boundary)
    bedge = np.stack([k, (k + 1) % n_boundary], 1)
    return dict(xy=xy.astype(np.float64), tri=tri.astype(np.int32),
                bedge=bedge.astype(np.int32),
                btag=np.full(n_boundary, DIRICHLET, dtype=np.int32))
