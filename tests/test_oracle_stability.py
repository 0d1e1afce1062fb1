"""Stability pins of the oracle (CPU).

* The reading that drops flat sub-stencils from the nonlinear reconstruction (Sec. 3.4): on the
  520,200-triangle jittered mesh one cell's sub-stencil {0, i, j} has centroid offsets at a sine of
  0.011.  A small interface jump passing that cell (a patch of the mesh cut around it, walls at
  the cut) stays bounded for 150 steps; with that plane kept as a candidate the same run is NaN
  after about 30 steps (its huge slope enters the WENO-AO combination through the
  -(omega_0 / d_0) d_m P_m term once the weights turn nonlinear).
* The one-step map of the linear scheme at rest on the periodic right-triangle lattice (the mesh
  family of the accuracy tests) is not expansive: power iteration of its finite-difference
  linearisation grows by at most 1 + 1e-6 per step.
"""
import numpy as np
import pytest

import oracle as o
import workloads as w
from workloads.scenarios import _level_state


def _cut(sc, centre, radius):
    xy, tri = sc.node_xy, sc.tri
    cen = xy[tri].mean(axis=1)
    keep = np.hypot(cen[:, 0] - centre[0], cen[:, 1] - centre[1]) < radius
    t = tri[keep]
    used = np.unique(t.ravel())
    remap = -np.ones(xy.shape[0], dtype=np.int64)
    remap[used] = np.arange(used.size)
    return xy[used], remap[t].astype(np.int32), sc.node_B[used]


def _plane_sines(mesh, c):
    """Sines of the angles between the centroid offsets of the three plane sub-stencils of cell c."""
    _, cx, cy = mesh.geometry()
    cells, maps = mesh.stencil(c)
    off = []
    for l in range(1, 4):
        R, t = maps[l, :4].reshape(2, 2), maps[l, 4:]
        off.append(R @ np.array([cx[cells[l]], cy[cells[l]]]) + t - np.array([cx[c], cy[c]]))
    out = []
    for s in range(3):
        a, b = off[s], off[(s + 1) % 3]
        out.append(abs(a[0] * b[1] - a[1] * b[0]) / (np.linalg.norm(a) * np.linalg.norm(b)))
    return out


def test_interface_jump_past_a_flat_substencil_stays_bounded():
    sc = w.lake_at_rest(510, seed=20230604)
    cen = sc.node_xy[sc.tri].mean(axis=1)
    c0 = int(np.argmin(np.hypot(cen[:, 0] - 0.53482, cen[:, 1] - 0.19665)))
    centre = cen[c0]
    xy, tri, nB = _cut(sc, centre, 0.02)
    # interface raised by 1e-3 inside a disk of radius 0.006 whose edge passes through the cell
    psc = _level_state("patch", xy, tri, nB, 0.98, 0.3, 1e9, 9.81,
                       lambda x, y: (np.full_like(x, 0.8), np.full_like(x, 0.2)), 1e-3,
                       (centre[0] - 0.006, centre[1], 0.006))
    mesh = o.Mesh.from_scenario(psc)
    pc = np.hypot(*(psc.node_xy[psc.tri].mean(axis=1) - centre).T).argmin()
    assert min(_plane_sines(mesh, int(pc))) < 0.02      # the flat sub-stencil is in the patch
    p = o.params_of(psc)
    W, gW = psc.W0.copy(), psc.gradW0.copy()
    m0 = o.mass(mesh, W)
    peak = []
    for k in range(150):
        W, gW = o.step(mesh, p, o.dt(mesh, p, W), W, gW)
        assert np.isfinite(W).all() and np.isfinite(gW).all(), k
        peak.append(np.abs(W[[1, 2, 4, 5]]).max())
    assert max(peak) < 5 * peak[24], (peak[24], max(peak))
    assert np.abs(o.mass(mesh, W) - m0).max() < 1e-13 * m0.max()


def test_linear_one_step_map_on_the_lattice_is_not_expansive():
    sc = w.smooth_periodic(16)
    T = sc.n_tri
    W0 = np.zeros((6, T))
    W0[0], W0[3] = 0.2, 0.8                              # rest, flat bottom
    gW0 = np.zeros((6, 2, T))
    mesh = o.Mesh.from_scenario(sc)
    p = o.params(G=sc.G, chi=sc.chi, cfl=0.3, linear=True)
    dt = o.dt(mesh, p, W0)
    eps = 1e-7

    def apply(v):
        dW, dg = v[:6 * T].reshape(6, T), v[6 * T:].reshape(6, 2, T)
        Wp, gp = o.step(mesh, p, dt, W0 + eps * dW, gW0 + eps * dg)
        Wm, gm = o.step(mesh, p, dt, W0 - eps * dW, gW0 - eps * dg)
        return np.concatenate([((Wp - Wm) / (2 * eps)).ravel(), ((gp - gm) / (2 * eps)).ravel()])

    v = np.random.default_rng(5).standard_normal(18 * T)
    v /= np.linalg.norm(v)
    growth = []
    for _ in range(150):
        u = apply(v)
        growth.append(np.linalg.norm(u))
        v = u / growth[-1]
    rate = np.exp(np.mean(np.log(growth[-50:])))
    print(f"lattice one-step growth {rate:.8f}")
    assert rate < 1 + 1e-6, rate
