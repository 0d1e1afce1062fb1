"""Initial data for the two-layer shallow water test problems.

The state is given as cell averages ``W0[6, T]`` and cell-averaged gradients ``gradW0[6, 2, T]``
in the component order of the conservative system: (h2, h2 U2, h2 V2, h1, h1 U1, h1 V1), layer 1
being the lower, denser layer.  Smooth data are averaged with a collapsed (Duffy) Gauss-Legendre
rule over each triangle and the gradients come from the divergence theorem with Gauss-Legendre
points on the edges.  Rest states over a bottom given at the nodes use that bottom's piecewise
linear interpolant, so that h1 + B is exactly the prescribed level cell by cell.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional

import numpy as np

from .meshes import jittered_rect, jittered_square, periodic_square

COMPONENTS = ("h2", "h2U2", "h2V2", "h1", "h1U1", "h1V1")


@dataclasses.dataclass
class Scenario:
    name: str
    node_xy: np.ndarray          # [N, 2] f64
    tri: np.ndarray              # [T, 3] i32, counter-clockwise
    node_B: np.ndarray           # [N] f64 bottom at nodes (piecewise linear)
    boundary: str                # "periodic", "wall" or "free"
    periodic_L: Optional[tuple]  # (Lx, Ly) for periodic meshes
    G: float
    chi: float
    cfl: float
    t_end: float
    W0: np.ndarray               # [6, T]
    gradW0: np.ndarray           # [6, 2, T]
    exact: Optional[Callable] = None  # exact(t) -> W cell averages [6, T] when known
    h_dry: float = 0.0           # wet/dry threshold of the scheme (0: every layer wet everywhere)

    @property
    def n_tri(self) -> int:
        return int(self.tri.shape[0])


# ---------------------------------------------------------------------------------------------
# quadrature of analytic data (input preparation only)

def _gl01(q: int):
    x, w = np.polynomial.legendre.leggauss(q)
    return 0.5 * (x + 1.0), 0.5 * w


def _tri_rule(q: int):
    """Collapsed Gauss-Legendre rule on the reference triangle {(s, t): s, t >= 0, s + t <= 1}.

    Returns barycentric-free reference points (s, t) and weights summing to 1 (an average)."""
    g, w = _gl01(q)
    s = np.repeat(g, q)
    r = np.tile(g, q)
    t = r * (1.0 - s)
    wt = np.repeat(w, q) * np.tile(w, q) * (1.0 - s)
    return s, t, wt / wt.sum()


def _geometry(xy, tri):
    a, b, c = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]
    area = 0.5 * ((b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0]))
    return a, b, c, area


def cell_average(xy, tri, fn, q: int = 8):
    """Average of fn(x, y) (vectorised, returns [k, ...]) over each triangle -> [k, T]."""
    a, b, c, _ = _geometry(xy, tri)
    s, t, w = _tri_rule(q)
    acc = None
    for sk, tk, wk in zip(s, t, w):
        x = a[:, 0] + sk * (b[:, 0] - a[:, 0]) + tk * (c[:, 0] - a[:, 0])
        y = a[:, 1] + sk * (b[:, 1] - a[:, 1]) + tk * (c[:, 1] - a[:, 1])
        v = np.asarray(fn(x, y)) * wk
        acc = v if acc is None else acc + v
    return acc


def cell_gradient(xy, tri, fn, q: int = 8):
    """Cell-averaged gradient (1/|T|) * boundary integral of fn * n over each triangle -> [k, 2, T]."""
    a, b, c, area = _geometry(xy, tri)
    g, w = _gl01(q)
    acc = None
    for p, r in ((a, b), (b, c), (c, a)):
        ex, ey = r[:, 0] - p[:, 0], r[:, 1] - p[:, 1]
        # outward normal times edge length for a counter-clockwise triangle
        nlx, nly = ey, -ex
        for gk, wk in zip(g, w):
            x = p[:, 0] + gk * ex
            y = p[:, 1] + gk * ey
            v = np.asarray(fn(x, y)) * wk
            term = np.stack([v * nlx, v * nly], axis=-2)
            acc = term if acc is None else acc + term
    return acc / area


def _p1_bottom(xy, tri, node_B):
    """Mean and gradient of the piecewise-linear bottom on each triangle."""
    a, b, c, area = _geometry(xy, tri)
    Ba, Bb, Bc = node_B[tri[:, 0]], node_B[tri[:, 1]], node_B[tri[:, 2]]
    mean = (Ba + Bb + Bc) / 3.0
    # gradient of the plane through the three vertices
    gx = (Ba * (b[:, 1] - c[:, 1]) + Bb * (c[:, 1] - a[:, 1]) + Bc * (a[:, 1] - b[:, 1])) / (2 * area)
    gy = (Ba * (c[:, 0] - b[:, 0]) + Bb * (a[:, 0] - c[:, 0]) + Bc * (b[:, 0] - a[:, 0])) / (2 * area)
    return mean, gx, gy


def _pack_smooth(xy, tri, prim):
    """prim(x, y) -> (h2, U2, V2, h1, U1, V1) arrays; returns conservative averages and gradients."""

    def cons(x, y):
        h2, U2, V2, h1, U1, V1 = prim(x, y)
        return np.stack([h2, h2 * U2, h2 * V2, h1, h1 * U1, h1 * V1])

    return cell_average(xy, tri, cons), cell_gradient(xy, tri, cons)


# ---------------------------------------------------------------------------------------------
# the problems

def smooth_periodic(n: int = 20, chi: float = 0.98, cfl: float = 0.3, t_end: float = 0.1,
                    G: float = 9.81) -> Scenario:
    """Periodic [0,2]^2, flat bottom, h1 = 1 + 0.2 sin(pi(x+y)), h2 = 1 - 0.1 sin(pi(x+y)),
    U = V = 0.5 in both layers (the small single-instance FP64 problem)."""
    xy, tri, L = periodic_square(n, 2.0)

    def prim(x, y):
        s = np.sin(np.pi * (x + y))
        one = np.ones_like(x)
        return (1.0 - 0.1 * s, 0.5 * one, 0.5 * one, 1.0 + 0.2 * s, 0.5 * one, 0.5 * one)

    W0, gW0 = _pack_smooth(xy, tri, prim)
    return Scenario(f"smooth_periodic_n{n}", xy, tri, np.zeros(xy.shape[0]), "periodic", L, G, chi,
                    cfl, t_end, W0, gW0)


def accuracy_e1(n: int, cfl: float = 0.5, t_end: float = 0.1, G: float = 9.81) -> Scenario:
    """Translating two-layer Gaussian with chi = 1 on [0,2]^2 (mesh leg h = 2/n), exact solution
    known: h1 = 0.9 + 0.02 exp(-50 |x - (1+t, 1+t)|^2), h2 = 1 - h1, U = V = 1."""
    xy, tri, L = periodic_square(n, 2.0)

    def prim_at(t):
        def prim(x, y):
            h1 = 0.9 + 0.02 * np.exp(-50.0 * ((x - 1.0 - t) ** 2 + (y - 1.0 - t) ** 2))
            one = np.ones_like(x)
            return (1.0 - h1, one, one, h1, one, one)
        return prim

    W0, gW0 = _pack_smooth(xy, tri, prim_at(0.0))

    def exact(t):
        return _pack_smooth(xy, tri, prim_at(t))[0]

    return Scenario(f"accuracy_e1_n{n}", xy, tri, np.zeros(xy.shape[0]), "periodic", L, G, 1.0,
                    cfl, t_end, W0, gW0, exact)


def accuracy_e1_free(n: int, cfl: float = 0.5, t_end: float = 0.1, G: float = 9.81) -> Scenario:
    """The translating Gaussian of accuracy_e1 with the free boundary the paper states for it:
    the same right-triangle lattice of [0,2]^2 without the periodic pairing (mass flows out at
    x, y = 2 and in at x, y = 0)."""
    sc = accuracy_e1(n, cfl=cfl, t_end=t_end, G=G)
    return dataclasses.replace(sc, name=f"accuracy_e1_free_n{n}", boundary="free", periodic_L=None)


def uniform_stream(n: int, seed: int = 20230621, U=(0.7, -0.4), chi: float = 0.95, cfl: float = 0.3,
                   t_end: float = 1e9, G: float = 9.81) -> Scenario:
    """A uniform two-layer stream (h1 = 0.6, h2 = 0.4, both layers moving with U) over a flat
    bottom on a jittered mesh of [0,1]^2 with free boundaries: an exact steady solution that a
    transmissive boundary must keep."""
    xy, tri = jittered_square(n, seed)
    T = tri.shape[0]
    W0 = np.zeros((6, T))
    W0[0], W0[1], W0[2] = 0.4, 0.4 * U[0], 0.4 * U[1]
    W0[3], W0[4], W0[5] = 0.6, 0.6 * U[0], 0.6 * U[1]
    return Scenario(f"uniform_stream_n{n}", xy, tri, np.zeros(xy.shape[0]), "free", None, G, chi, cfl, t_end,
                    W0, np.zeros((6, 2, T)))


def free_outflow(n: int, seed: int = 20230622, chi: float = 0.95, cfl: float = 0.3, t_end: float = 1e9,
                 G: float = 9.81) -> Scenario:
    """A smooth two-layer hump moving out of a free-boundary box: jittered mesh of [0,1]^2, bump
    bottom 0.1 exp(-30 |x - (0.5, 0.5)|^2), lower level 1 + 0.05 exp(-80 |x - (0.7, 0.5)|^2), upper
    layer 0.5, both layers flowing with U = (0.8, 0.3)."""
    xy, tri = jittered_square(n, seed)
    node_B = _bump(xy, amp=0.1, k=30.0)
    Bm, Bx, By = _p1_bottom(xy, tri, node_B)

    def prim(x, y):
        eta = 1.0 + 0.05 * np.exp(-80.0 * ((x - 0.7) ** 2 + (y - 0.5) ** 2))
        one = np.ones_like(x)
        return (0.5 * one, 0.8 * one, 0.3 * one, eta, 0.8 * one, 0.3 * one)

    W0, gW0 = _pack_smooth(xy, tri, prim)
    # the lower layer's thickness is the level minus the piecewise-linear bottom; its momentum
    # follows the thickness
    W0[3] -= Bm
    gW0[3, 0] -= Bx
    gW0[3, 1] -= By
    W0[4], W0[5] = 0.8 * W0[3], 0.3 * W0[3]
    gW0[4], gW0[5] = 0.8 * gW0[3], 0.3 * gW0[3]
    return Scenario(f"free_outflow_n{n}", xy, tri, node_B, "free", None, G, chi, cfl, t_end, W0, gW0)


def smooth_jittered(n: int, seed: int = 20230623, chi: float = 0.95, cfl: float = 0.3, t_end: float = 1e9,
                    G: float = 9.81) -> Scenario:
    """Both layers varying smoothly on a jittered wall mesh of [0,1]^2 over the bump bottom
    0.1 exp(-30 |x - (0.5, 0.5)|^2): lower level 1 + 0.05 sin(2 pi x) cos(2 pi y), upper thickness
    0.5 + 0.04 cos(2 pi x + 0.4) sin(2 pi y), velocities (0.2 + 0.1 sin(2 pi y), -0.1 cos(2 pi x))
    below and (0.1 cos(2 pi (x + y)), 0.15) above."""
    xy, tri = jittered_square(n, seed)
    node_B = _bump(xy, amp=0.1, k=30.0)
    Bm, Bx, By = _p1_bottom(xy, tri, node_B)
    tp = 2.0 * np.pi

    def prim(x, y):
        eta = 1.0 + 0.05 * np.sin(tp * x) * np.cos(tp * y)
        h2 = 0.5 + 0.04 * np.cos(tp * x + 0.4) * np.sin(tp * y)
        one = np.ones_like(x)
        return (h2, 0.1 * np.cos(tp * (x + y)), 0.15 * one, eta, 0.2 + 0.1 * np.sin(tp * y), -0.1 * np.cos(tp * x))

    def cons(x, y):
        h2, U2, V2, eta, U1, V1 = prim(x, y)
        return np.stack([h2, h2 * U2, h2 * V2, eta, eta * U1, eta * V1])

    W0 = cell_average(xy, tri, cons)
    gW0 = cell_gradient(xy, tri, cons)
    # the lower layer's thickness is the level minus the piecewise-linear bottom; its momentum is
    # that thickness times the level's mean velocity, and the momentum gradient drops the bottom's
    # share U grad B (smooth synthetic data, not an exact solution)
    U1 = W0[4] / W0[3]
    V1 = W0[5] / W0[3]
    W0[3] -= Bm
    gW0[3, 0] -= Bx
    gW0[3, 1] -= By
    W0[4], W0[5] = U1 * W0[3], V1 * W0[3]
    gW0[4, 0] -= U1 * Bx
    gW0[4, 1] -= U1 * By
    gW0[5, 0] -= V1 * Bx
    gW0[5, 1] -= V1 * By
    return Scenario(f"smooth_jittered_n{n}", xy, tri, node_B, "wall", None, G, chi, cfl, t_end, W0, gW0)


def _bump(xy, amp=0.5, cx=0.5, cy=0.5, k=50.0):
    return amp * np.exp(-k * ((xy[:, 0] - cx) ** 2 + (xy[:, 1] - cy) ** 2))


def lake_at_rest(n: int, seed: int = 20230604, chi: float = 0.98, eta1: float = 0.8,
                 h2: float = 0.2, perturb: float = 0.0, disk=(0.3, 0.3, 0.1), cfl: float = 0.3,
                 t_end: float = 1e9, G: float = 9.81, bump_amp: float = 0.5) -> Scenario:
    """Jittered Delaunay mesh of [0,1]^2 with walls, bottom B = bump_amp exp(-50 r^2) about the
    centre, lower-layer level h1 + B = eta1, upper layer h2, at rest.  With ``perturb`` != 0 the
    interface inside the disk |x - (cx, cy)| < r (cell centroids) is raised by ``perturb`` and the
    upper layer thinned by the same amount (free surface unchanged)."""
    xy, tri = jittered_square(n, seed)
    node_B = _bump(xy, amp=bump_amp)
    return _level_state(f"lake_at_rest_n{n}", xy, tri, node_B, chi, cfl, t_end, G,
                        lambda cx, cy: (np.full_like(cx, eta1), np.full_like(cx, h2)),
                        perturb, disk)


def well_balance_bump(n: int = 40, seed: int = 20230613, chi: float = 1.0, cfl: float = 0.5,
                      t_end: float = 100.0, G: float = 9.81) -> Scenario:
    """The well-balance test of Sec. 4: [0, 2]^2 with walls, jittered Delaunay mesh of cell size
    2/n (n = 40: 0.05), bottom B = 0.5 exp(-50 |x - (1, 1)|^2), h1 = 0.8 - B, h2 = 0.2, at rest,
    density ratio 1, CFL 0.5, run to t = 100."""
    xy, tri = jittered_rect(n, n, 2.0, 2.0, seed)
    node_B = _bump(xy, amp=0.5, cx=1.0, cy=1.0)
    return _level_state(f"well_balance_bump_n{n}", xy, tri, node_B, chi, cfl, t_end, G,
                        lambda cx, cy: (np.full_like(cx, 0.8), np.full_like(cx, 0.2)), 0.0, None)


def dam_break(n: int, seed: int = 20230605, chi: float = 0.95, x_dam: float = 0.5,
              left=(1.0, 0.5), right=(0.5, 1.0), sin_amp: float = 0.1, bump_amp: float = 0.0,
              cfl: float = 0.3, t_end: float = 1e9, G: float = 9.81) -> Scenario:
    """Two-layer dam break on a jittered mesh of [0,1]^2 with walls: lower-layer level h1 + B and
    upper thickness h2 jump from ``left`` to ``right`` across x = x_dam (by cell centroid), bottom
    B = sin_amp sin(2 pi x) sin(2 pi y) + bump_amp exp(-50 |x - (0.75, 0.5)|^2), fluid at rest."""
    xy, tri = jittered_square(n, seed)
    node_B = sin_amp * np.sin(2 * np.pi * xy[:, 0]) * np.sin(2 * np.pi * xy[:, 1])
    if bump_amp:
        node_B = node_B + _bump(xy, amp=bump_amp, cx=0.75, cy=0.5)

    def levels(cx, cy):
        lft = cx < x_dam
        return np.where(lft, left[0], right[0]), np.where(lft, left[1], right[1])

    return _level_state(f"dam_break_n{n}", xy, tri, node_B, chi, cfl, t_end, G, levels, 0.0, None)


def _level_state(name, xy, tri, node_B, chi, cfl, t_end, G, levels, perturb, disk, h_dry=0.0):
    T = tri.shape[0]
    Bm, Bx, By = _p1_bottom(xy, tri, node_B)
    c = xy[tri].mean(axis=1)
    eta1, h2 = levels(c[:, 0], c[:, 1])
    eta1 = np.asarray(eta1, dtype=np.float64).copy()
    h2 = np.asarray(h2, dtype=np.float64).copy()
    if perturb:
        cx, cy, r = disk
        inside = (c[:, 0] - cx) ** 2 + (c[:, 1] - cy) ** 2 < r * r
        eta1[inside] += perturb
        h2[inside] -= perturb
    W0 = np.zeros((6, T))
    gW0 = np.zeros((6, 2, T))
    W0[0] = h2
    W0[3] = eta1 - Bm
    gW0[3, 0] = -Bx
    gW0[3, 1] = -By
    if h_dry > 0:
        if (W0[3] < 0).any() or (W0[0] < 0).any():
            raise ValueError("negative layer thickness in initial data")
    elif (W0[3] <= 0).any() or (W0[0] <= 0).any():
        raise ValueError("non-positive layer thickness in initial data")
    return Scenario(name, xy, tri, node_B, "wall", None, G, chi, cfl, t_end, W0, gW0, h_dry=h_dry)


# ---------------------------------------------------------------------------------------------
# vanishing layers (wet/dry)

def dam_break_dry(n: int = 100, seed: int = 20230607, chi: float = 1.0, h_dry: float = 1e-6, cfl: float = 0.3,
                  t_end: float = 0.08, G: float = 9.81) -> Scenario:
    """The paper's two-layer dam break (Sec. 4, dam-break problems at density ratios 1 and 0.2):
    [0, 1] x [0, 0.5], flat bottom, walls, at rest; lower layer 0.357 everywhere, upper layer 1 for
    x < 0.5 and dry (0) beyond; jittered Delaunay mesh of cell size 1/n."""
    xy, tri = jittered_rect(n, max(n // 2, 2), 1.0, 0.5, seed)

    def levels(cx, cy):
        return np.full_like(cx, 0.357), np.where(cx < 0.5, 1.0, 0.0)

    return _level_state(f"dam_break_dry_n{n}", xy, tri, np.zeros(xy.shape[0]), chi, cfl, t_end, G, levels,
                        0.0, None, h_dry=h_dry)


def _ritter(x, t, h0, x0, G):
    """Ritter's dam break onto a dry bed: thickness and velocity of the single-layer equations."""
    c0 = math.sqrt(G * h0)
    xi = (np.asarray(x, dtype=np.float64) - x0) / t
    h = np.where(xi <= -c0, h0, np.where(xi >= 2 * c0, 0.0, (2 * c0 - xi) ** 2 / (9 * G)))
    u = np.where(xi <= -c0, 0.0, np.where(xi >= 2 * c0, 0.0, 2.0 / 3.0 * (c0 + xi)))
    return h, u


def ritter_channel(n: int = 200, layer: str = "lower", seed: int = 20230608, h0: float = 1.0, x0: float = 1.0,
                   h_dry: float = 1e-6, chi: float = 0.98, cfl: float = 0.3, t_end: float = 0.1,
                   G: float = 9.81) -> Scenario:
    """A single-layer dam break onto a dry bed in the two-layer system: one layer (``layer``) is h0
    for x < x0 and dry beyond, the other layer is dry everywhere, flat bottom, walls, channel
    [0, 2] x [0, 0.2] (jittered mesh, cell size 2/n).  With the other layer absent the equations
    are the single-layer ones, whose solution is Ritter's: exact(t) gives its cell averages."""
    xy, tri = jittered_rect(n, max(n // 10, 2), 2.0, 0.2, seed)
    T = tri.shape[0]
    c = xy[tri].mean(axis=1)
    o = 3 if layer == "lower" else 0
    W0 = np.zeros((6, T))
    W0[o] = np.where(c[:, 0] < x0, h0, 0.0)

    def exact(t):
        W = np.zeros((6, T))
        if t <= 0:
            W[o] = W0[o]
            return W
        W[o] = cell_average(xy, tri, lambda x, y: _ritter(x, t, h0, x0, G)[0], q=12)
        W[o + 1] = cell_average(xy, tri, lambda x, y: np.prod(_ritter(x, t, h0, x0, G), axis=0), q=12)
        return W

    return Scenario(f"ritter_{layer}_n{n}", xy, tri, np.zeros(xy.shape[0]), "wall", None, G, chi, cfl, t_end,
                    W0, np.zeros((6, 2, T)), exact=exact, h_dry=h_dry)


def dry_bump_dam_break(n: int = 100, seed: int = 20230610, chi: float = 0.98, h_dry: float = 1e-6,
                       cfl: float = 0.3, t_end: float = 0.5, G: float = 9.81) -> Scenario:
    """A lower layer running over dry land: the bottom of the headline workload (Gaussian bump 0.5
    high at the centre of [0,1]^2, jittered mesh, walls), the lower layer's level 0.45 for x < 0.3
    and 0.3 beyond, so that the bump's top stands dry, the upper layer 0.2 thick everywhere, at
    rest; the lower layer thickness max(level - B, 0) by cell."""
    xy, tri = jittered_square(n, seed)
    node_B = _bump(xy)
    Bm, _, _ = _p1_bottom(xy, tri, node_B)
    c = xy[tri].mean(axis=1)
    T = tri.shape[0]
    W0 = np.zeros((6, T))
    W0[0] = 0.2
    W0[3] = np.maximum(np.where(c[:, 0] < 0.3, 0.45, 0.3) - Bm, 0.0)
    return Scenario(f"dry_bump_dam_break_n{n}", xy, tri, node_B, "wall", None, G, chi, cfl, t_end, W0,
                    np.zeros((6, 2, T)), h_dry=h_dry)


def dam_break_breach(kind: str = "dry", n: int = 80, seed: int = 20230609, chi: float = 0.98, h_dry: float = 1e-6,
                     cfl: float = 0.3, t_end: float = 7.2, G: float = 9.81) -> Scenario:
    """A stand-in for the paper's 2-D dam break in an irregular domain (Sec. 4): a dam of width 10
    whose left side is at x = 95, with a breach of length 75 starting at y = 95, in a flat-bottom
    basin [0, 260] x [0, 200] (the far wall is beyond the reach of a dry-bed front, speed at most
    2 sqrt(G 10), by t = 7.2); jittered mesh of cell size 200/n with the dam's triangles removed,
    walls.  Lower / upper thicknesses (9, 1) for x < 95 and, beyond, (5, 0) for the wet bed or
    (1e-3, 1e-3) for the dry one."""
    xy, tri = jittered_rect(int(round(1.3 * n)), n, 260.0, 200.0, seed)
    c = xy[tri].mean(axis=1)
    dam = (c[:, 0] > 95.0) & (c[:, 0] < 105.0) & ~((c[:, 1] > 95.0) & (c[:, 1] < 170.0))
    tri = tri[~dam]
    used = np.unique(tri)
    remap = np.full(xy.shape[0], -1, dtype=np.int64)
    remap[used] = np.arange(used.size)
    xy = xy[used]
    tri = remap[tri].astype(np.int32)
    right = (5.0, 0.0) if kind == "wet" else (1e-3, 1e-3)

    def levels(cx, cy):
        left = cx < 95.0
        return np.where(left, 9.0, right[0]), np.where(left, 1.0, right[1])

    return _level_state(f"dam_break_breach_{kind}_n{n}", xy, tri, np.zeros(xy.shape[0]), chi, cfl, t_end, G,
                        levels, 0.0, None, h_dry=h_dry)


def riemann_exchange(n: int = 100, chi: float = 0.98, cfl: float = 0.3, t_end: float = 0.1,
                     G: float = 10.0) -> Scenario:
    """Two-layer exchange flow with a small interface jump (Sec. 4, first Riemann problem): lower /
    upper thicknesses (0.5, 0.5) for x < 0.3 and (0.55, 0.45) beyond, both layers moving with
    U = 2.5, flat bottom, G = 10.  On the periodic right-triangle lattice of [0, 1]^2 (the wrap at
    x = 0 adds a second jump), so the data are invariant under the lattice's y translations."""
    xy, tri, L = periodic_square(n, 1.0)
    c = xy[tri].mean(axis=1)
    left = c[:, 0] < 0.3
    T = tri.shape[0]
    W0 = np.zeros((6, T))
    W0[3] = np.where(left, 0.5, 0.55)      # lower layer h1
    W0[0] = np.where(left, 0.5, 0.45)      # upper layer h2
    W0[4] = 2.5 * W0[3]
    W0[1] = 2.5 * W0[0]
    return Scenario(f"riemann_exchange_n{n}", xy, tri, np.zeros(xy.shape[0]), "periodic", L, G, chi,
                    cfl, t_end, W0, np.zeros((6, 2, T)))


def riemann_interface(nx: int = 400, ny: int = 40, seed: int = 20230611, chi: float = 0.98,
                      cfl: float = 0.3, t_end: float = 1.0, G: float = 9.81) -> Scenario:
    """Two-layer Riemann problem with a large interface jump (Sec. 4, second Riemann problem):
    thicknesses (0.2, 1.8) for x < 5 and (1.8, 0.2) beyond, at rest, flat bottom, on a jittered
    Delaunay mesh of [0, 10] x [0, 1] (cell size 1/40) with walls."""
    xy, tri = jittered_rect(nx, ny, 10.0, 1.0, seed)

    def levels(cx, cy):
        left = cx < 5.0
        return np.where(left, 0.2, 1.8), np.where(left, 1.8, 0.2)

    return _level_state(f"riemann_interface_{nx}x{ny}", xy, tri, np.zeros(xy.shape[0]), chi, cfl, t_end, G,
                        levels, 0.0, None)


def circular_interface(n: int = 100, seed: int = 20230612, chi: float = 0.98, cfl: float = 0.3,
                       t_end: float = 4.0, G: float = 9.81) -> Scenario:
    """Circular interface propagation (Sec. 4): thicknesses (1.8, 0.2) inside the circle of radius 2
    about (5, 5) and (0.2, 1.8) outside, at rest, flat bottom, on a jittered Delaunay mesh of
    [0, 10]^2 (cell size 10/n) with walls."""
    xy, tri = jittered_rect(n, n, 10.0, 10.0, seed)

    def levels(cx, cy):
        inside = (cx - 5.0) ** 2 + (cy - 5.0) ** 2 < 4.0
        return np.where(inside, 1.8, 0.2), np.where(inside, 0.2, 1.8)

    return _level_state(f"circular_interface_n{n}", xy, tri, np.zeros(xy.shape[0]), chi, cfl, t_end, G,
                        levels, 0.0, None)


def _ensemble_member(args):
    s, n, seed, chi, amp, cfl, G = args
    sc = lake_at_rest(n, seed=seed, chi=chi, perturb=amp, cfl=cfl, G=G)
    sc.name = f"ensemble_{s}_n{n}"
    return sc


def ensemble(n_scen: int = 256, seed: int = 20230606, t_min: int = 5000, t_max: int = 200000,
             cfl: float = 0.3, G: float = 9.81, workers: Optional[int] = None):
    """Independent bump + rest + disk-perturbation scenarios with log-uniform sizes, log-uniform
    perturbation amplitudes in [1e-4, 1e-2] and density ratios uniform in [0.90, 0.99].  The
    parameters are drawn in order from one seeded generator; the meshes are built by a pool of
    processes (at most 16)."""
    import os
    from concurrent.futures import ProcessPoolExecutor

    rng = np.random.default_rng(seed)
    jobs = []
    for s in range(n_scen):
        T = math.exp(rng.uniform(math.log(t_min), math.log(t_max)))
        n = max(4, int(round(math.sqrt(T / 2.0))))
        amp = math.exp(rng.uniform(math.log(1e-4), math.log(1e-2)))
        chi = float(rng.uniform(0.90, 0.99))
        jobs.append((s, n, seed + 1 + s, chi, amp, cfl, G))
    workers = workers if workers is not None else min(16, os.cpu_count() or 1)
    if workers <= 1 or n_scen < 4:
        return [_ensemble_member(j) for j in jobs]
    with ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(_ensemble_member, jobs, chunksize=4))
