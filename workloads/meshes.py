"""Triangle meshes used by the test problems.

Two families:
* ``periodic_square``: an n x n lattice of squares on [0, L]^2, each square cut along its
  (i, j) -> (i+1, j+1) diagonal, giving 2 n^2 right triangles.  Nodes on x = L / y = L duplicate
  those on x = 0 / y = 0; the solver pairs the boundary edges by translation.
* ``jittered_square``: the (n+1)^2 lattice of [0, 1]^2 with interior nodes moved by independent
  uniform offsets in [-j h, j h] (boundary nodes move along the boundary only, corners stay),
  then Delaunay-triangulated (2 n^2 triangles).

All triangles are returned counter-clockwise as int32 [T, 3] with float64 node coordinates [N, 2].
"""
from __future__ import annotations

import numpy as np


def _orient_ccw(xy: np.ndarray, tri: np.ndarray) -> np.ndarray:
    a, b, c = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]
    cross = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])
    tri = tri.copy()
    neg = cross < 0
    tri[neg, 1], tri[neg, 2] = tri[neg, 2].copy(), tri[neg, 1].copy()
    return tri


def periodic_square(n: int, length: float = 2.0):
    """Structured right-triangle mesh of [0, length]^2 with periodic pairing.

    Returns (node_xy [N,2] f64, tri [2n^2,3] i32, periodic_L (length, length)).
    """
    h = length / n
    ii, jj = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="ij")
    xy = np.stack([ii.ravel() * h, jj.ravel() * h], axis=1).astype(np.float64)
    # exact end coordinates so that translated nodes coincide bit for bit
    xy[ii.ravel() == n, 0] = length
    xy[jj.ravel() == n, 1] = length

    def nid(i, j):
        return i * (n + 1) + j

    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    i, j = i.ravel(), j.ravel()
    a, b, c, d = nid(i, j), nid(i + 1, j), nid(i + 1, j + 1), nid(i, j + 1)
    t1 = np.stack([a, b, c], axis=1)
    t2 = np.stack([a, c, d], axis=1)
    tri = np.empty((2 * n * n, 3), dtype=np.int64)
    tri[0::2] = t1
    tri[1::2] = t2
    return xy, tri.astype(np.int32), (float(length), float(length))


def jittered_square(n: int, seed: int, jitter: float = 0.3):
    """Jittered-lattice Delaunay mesh of the unit square with 2 n^2 triangles."""
    from scipy.spatial import Delaunay

    h = 1.0 / n
    rng = np.random.default_rng(seed)
    ii, jj = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="ij")
    ii, jj = ii.ravel(), jj.ravel()
    x = ii * h
    y = jj * h
    dx = rng.uniform(-jitter * h, jitter * h, size=x.shape)
    dy = rng.uniform(-jitter * h, jitter * h, size=x.shape)
    on_x = (ii == 0) | (ii == n)
    on_y = (jj == 0) | (jj == n)
    dx[on_x] = 0.0  # nodes on x = 0 / x = 1 slide along y only
    dy[on_y] = 0.0
    x = x + dx
    y = y + dy
    x[ii == n] = 1.0
    y[jj == n] = 1.0
    x[ii == 0] = 0.0
    y[jj == 0] = 0.0
    xy = np.stack([x, y], axis=1).astype(np.float64)
    dl = Delaunay(xy)
    tri = _orient_ccw(xy, dl.simplices.astype(np.int64))
    if tri.shape[0] != 2 * n * n:
        raise RuntimeError(f"Delaunay gave {tri.shape[0]} triangles, expected {2 * n * n}")
    used = np.zeros(xy.shape[0], dtype=bool)
    used[tri.ravel()] = True
    if not used.all():
        raise RuntimeError("Delaunay dropped nodes")
    order = _morton_order(xy[tri].mean(axis=1))
    return xy, tri[order].astype(np.int32)


def jittered_rect(nx: int, ny: int, lx: float, ly: float, seed: int, jitter: float = 0.3):
    """Jittered-lattice Delaunay mesh of [0, lx] x [0, ly] with 2 nx ny triangles: the
    (nx+1) x (ny+1) lattice with interior nodes moved by uniform offsets within jitter times the
    local spacing (boundary nodes along the boundary only), Morton-ordered."""
    from scipy.spatial import Delaunay

    hx, hy = lx / nx, ly / ny
    rng = np.random.default_rng(seed)
    ii, jj = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), indexing="ij")
    ii, jj = ii.ravel(), jj.ravel()
    x = ii * hx + rng.uniform(-jitter * hx, jitter * hx, size=ii.shape)
    y = jj * hy + rng.uniform(-jitter * hy, jitter * hy, size=ii.shape)
    x[(ii == 0) | (ii == nx)] = (ii[(ii == 0) | (ii == nx)] * hx)
    y[(jj == 0) | (jj == ny)] = (jj[(jj == 0) | (jj == ny)] * hy)
    x[ii == nx] = lx
    y[jj == ny] = ly
    xy = np.stack([x, y], axis=1).astype(np.float64)
    tri = _orient_ccw(xy, Delaunay(xy).simplices.astype(np.int64))
    if tri.shape[0] != 2 * nx * ny:
        raise RuntimeError(f"Delaunay gave {tri.shape[0]} triangles, expected {2 * nx * ny}")
    order = _morton_order(xy[tri].mean(axis=1))
    return xy, tri[order].astype(np.int32)


def _morton_order(c: np.ndarray) -> np.ndarray:
    """Permutation sorting points along a Z-order curve (spatial locality of cell numbering)."""
    lo = c.min(axis=0)
    span = np.maximum(c.max(axis=0) - lo, 1e-300)
    q = np.clip(((c - lo) / span * 65535.0).astype(np.int64), 0, 65535)

    def spread(v):
        v = (v | (v << 8)) & 0x00FF00FF
        v = (v | (v << 4)) & 0x0F0F0F0F
        v = (v | (v << 2)) & 0x33333333
        v = (v | (v << 1)) & 0x55555555
        return v

    key = spread(q[:, 0]) | (spread(q[:, 1]) << 1)
    return np.argsort(key, kind="stable")
