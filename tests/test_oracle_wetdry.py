"""Pins of the oracle's wet/dry reading (h_dry > 0; the paper's dam breaks over a dry bed, Sec. 4,
for which it gives no treatment) against what the mathematics fixes: the kinetic upwind mass flux
out of a wet side into a vacuum, Ritter's exact dam break onto a dry bed, the absence of any force
from an absent layer, the lake at rest with one layer absent, and positivity with exact mass
conservation on the paper's dam breaks."""
import dataclasses
import math

import numpy as np
import pytest
from scipy.special import erfc

import oracle as o
import workloads as w

G = 9.81


def _kfvs_mass_flux(h, U):
    """h <u>_{u>0} over the Maxwellian with mean U and variance G h / 2."""
    lam = 1.0 / (G * h)
    return h * (U * 0.5 * erfc(-math.sqrt(lam) * U) + math.exp(-lam * U * U) / (2 * math.sqrt(math.pi * lam)))


@pytest.mark.parametrize("h,U,V", [(1.0, 0.0, 0.0), (0.3, 1.2, -0.4), (2.0, -0.8, 0.3)])
def test_vacuum_side_passes_the_kinetic_upwind_flux(h, U, V):
    """Next to a vacuum the first-order evolution's mass flux is the upwind half-moment of the wet
    side's Maxwellian whatever the collision time (the interface equilibrium holds exactly the
    particles that side sends), it carries the side's tangential velocity, and it has no time
    derivative; with the vacuum on the left the same flux runs the other way."""
    s = np.zeros(11)
    s[:3] = (h, U, V)
    vac = np.zeros(11)
    dt = 1e-3
    F0, Ft, Wb, Wbt = o.gks_point_wd(s, vac, G, dt, 1e-6, order1=True)
    ref = _kfvs_mass_flux(h, U)
    assert abs(F0[0] - ref) <= 1e-13 * max(1.0, abs(ref)), (F0[0], ref)
    assert abs(F0[2] - V * F0[0]) <= 1e-13 * max(1.0, abs(F0[0]))
    assert np.all(Ft == 0.0) and np.all(Wbt == 0.0)
    # mirror: vacuum on the left, the side moving the other way
    s2 = s.copy()
    s2[1] = -U
    F0m, _, _, _ = o.gks_point_wd(vac, s2, G, dt, 1e-6, order1=True)
    assert abs(F0m[0] + ref) <= 1e-13 * max(1.0, abs(ref))
    # both sides dry, or an interface holding less than h_dry: nothing passes
    for pair, h_dry in (((vac, vac), 1e-6), ((s, vac), 10 * h)):
        out = o.gks_point_wd(pair[0], pair[1], G, dt, h_dry, order1=True)
        assert all(np.all(a == 0.0) for a in out)


def test_cell_velocity_is_desingularised_only_in_thin_layers():
    """m / h at and above the thin-layer thickness 1000 h_dry (continuous there), the
    desingularised form below it, which vanishes with h; no division by a zero thickness."""
    h_dry = 1e-6
    for h in (1e-3, 0.01, 1.0):
        assert o.cell_velocity(h, 0.7 * h, h_dry) == pytest.approx(0.7, rel=1e-15)
    hs = 1000 * h_dry
    below = o.cell_velocity(hs * (1 - 1e-12), 0.7 * hs, h_dry)
    assert below == pytest.approx(0.7, rel=1e-9)
    assert abs(o.cell_velocity(1e-9, 1e-9, h_dry)) < 1e-8
    assert o.cell_velocity(0.0, 0.0, h_dry) == 0.0


def _run(sc, t_end=None, max_steps=20000, p=None):
    mesh = o.Mesh.from_scenario(sc)
    p = p or o.params_of(sc)
    W, gW = sc.W0.copy(), sc.gradW0.copy()
    t_end = sc.t_end if t_end is None else t_end
    t, n, hmin = 0.0, 0, 0.0
    while t < t_end - 1e-14 and n < max_steps:
        d = min(o.dt(mesh, p, W), t_end - t)
        W, gW = o.step(mesh, p, d, W, gW)
        t += d
        n += 1
        hmin = min(hmin, W[[0, 3]].min())
    return mesh, W, gW, t, n, hmin


_RITTER = {}


def _ritter(n, layer="lower"):
    if (n, layer) not in _RITTER:
        sc = w.ritter_channel(n, layer=layer)
        _RITTER[(n, layer)] = (sc,) + _run(sc)
    return _RITTER[(n, layer)]


def test_ritter_dam_break_onto_a_dry_bed():
    """Ritter's exact solution of the single-layer dam break onto a dry bed (the other layer absent
    everywhere): relative L1 errors of the thickness under 1 % and 0.5 % at cell sizes 1/50 and
    1/100 (measured 0.58 % and 0.31 %, first order, as the front band and the solution's kink at
    the front allow), the discharge within 5 % and 3 %, no negative thickness, the mass to round-off
    and the absent layer exactly zero."""
    errs = []
    for n, eh, em in ((100, 0.01, 0.05), (200, 0.005, 0.03)):
        sc, mesh, W, gW, t, steps, hmin = _ritter(n)
        assert t == pytest.approx(sc.t_end)
        ex = sc.exact(t)
        a, _, _ = mesh.geometry()
        e = (a * np.abs(W[3] - ex[3])).sum() / (a * ex[3]).sum()
        e_m = (a * np.abs(W[4] - ex[4])).sum() / (a * np.abs(ex[4])).sum()
        print(f"Ritter n={n}: {steps} steps, rel L1 h {e:.3e} hu {e_m:.3e}, min h {hmin:.1e}")
        assert e < eh and e_m < em, (n, e, e_m)
        assert hmin >= 0.0
        assert abs((a * W[3]).sum() - (a * sc.W0[3]).sum()) <= 1e-14 * (a * sc.W0[3]).sum()
        assert np.all(W[0:3] == 0.0)
        errs.append(e)
    assert errs[0] / errs[1] > 1.5


def test_absent_layer_exerts_no_force():
    """With the upper layer absent everywhere the lower layer evolves as in the single-layer
    equations: the density ratio has no effect (bit for bit), and the same dam break carried by
    the upper layer over an absent lower one (flat bottom) gives the same thickness."""
    base = w.ritter_channel(60, layer="lower")
    runs = [_run(dataclasses.replace(base, chi=chi), t_end=0.03)[1] for chi in (0.98, 0.5)]
    assert np.array_equal(runs[0], runs[1])
    up = w.ritter_channel(60, layer="upper")
    Wu = _run(up, t_end=0.03)[1]
    assert np.abs(Wu[0] - runs[0][3]).max() < 1e-12
    assert np.abs(Wu[1:3] - runs[0][4:6]).max() < 1e-12


def test_wet_dry_threshold_is_inert_on_wet_smooth_flows():
    """Without thin layers or steep thickness fronts the wet/dry reading changes nothing, bit for
    bit."""
    sc = w.smooth_jittered(10)
    ref = _run(sc, t_end=1e9, max_steps=3, p=o.params_of(sc, h_dry=0.0))
    got = _run(sc, t_end=1e9, max_steps=3, p=o.params_of(sc, h_dry=1e-6))
    assert np.array_equal(ref[1], got[1]) and np.array_equal(ref[2], got[2])


def test_lake_at_rest_with_an_absent_upper_layer():
    """A lake at rest over the bump with the upper layer absent everywhere stays at rest to
    round-off: the lower layer keeps its balance and nothing flows in the absent layer."""
    sc = w.lake_at_rest(10, chi=0.98)
    W0 = sc.W0.copy()
    W0[0] = 0.0
    gW0 = sc.gradW0.copy()
    gW0[0] = 0.0
    sc = dataclasses.replace(sc, W0=W0, gradW0=gW0, h_dry=1e-6)
    _, W, gW, _, _, hmin = _run(sc, t_end=1e9, max_steps=60)
    assert np.all(W[0:3] == 0.0)
    assert np.abs(W[4:6]).max() < 1e-13
    assert np.abs(W[3] - W0[3]).max() < 1e-13


@pytest.mark.parametrize("chi", [1.0, 0.2])
def test_paper_dam_break_over_a_dry_upper_bed(chi):
    """The paper's two-layer dam break (Sec. 4) with the upper layer dry beyond x = 0.5, to
    t = 0.08: no negative thickness, both layers' mass to round-off and the upper layer's front
    past x = 0.6."""
    sc = w.dam_break_dry(40, chi=chi)
    mesh, W, gW, t, n, hmin = _run(sc)
    assert t == pytest.approx(0.08) and np.isfinite(W).all()
    a, cx, _ = mesh.geometry()
    assert hmin >= 0.0
    for q in (0, 3):
        m0 = (a * sc.W0[q]).sum()
        assert abs((a * W[q]).sum() - m0) <= 1e-14 * m0
    assert (W[0][cx > 0.6] > 1e-3).any()


@pytest.mark.parametrize("kind", ["wet", "dry"])
def test_breached_dam_runs_to_the_papers_time(kind):
    """The 2-D dam break through a breach (Sec. 4, synthetic domain) on a coarse mesh: both beds
    reach t = 7.2 with no negative thickness, the mass of both layers to round-off, and speeds below
    the dry-bed front speed bound 2 sqrt(G 10) (plus the largest wave speed sqrt(G 10))."""
    sc = w.dam_break_breach(kind, n=40)
    mesh, W, gW, t, n, hmin = _run(sc)
    assert t == pytest.approx(7.2) and np.isfinite(W).all()
    a, _, _ = mesh.geometry()
    assert hmin >= 0.0
    for q in (0, 3):
        m0 = (a * sc.W0[q]).sum()
        assert abs((a * W[q]).sum() - m0) <= 1e-13 * m0
    bound = 3 * math.sqrt(G * 10.0)
    for q in (0, 3):
        U = np.array([o.cell_velocity(W[q, c], W[q + 1, c], sc.h_dry) for c in range(W.shape[1])])
        assert np.abs(U).max() < bound


def _dry_strip_lattice(n=40):
    """A strip of upper layer (0.25 < x < 0.5) over a uniform lower layer on the periodic
    right-triangle lattice of [0, 1]^2, dry elsewhere: data that depend on x only."""
    xy, tri, L = w.periodic_square(n, 1.0)
    c = xy[tri].mean(axis=1)
    T = tri.shape[0]
    W0 = np.zeros((6, T))
    W0[3] = 0.357
    W0[0] = np.where((c[:, 0] > 0.25) & (c[:, 0] < 0.5), 1.0, 0.0)
    sc = w.Scenario("dry_strip", xy, tri, np.zeros(xy.shape[0]), "periodic", L, G, 0.98, 0.3, 0.02, W0,
                    np.zeros((6, 2, T)), h_dry=1e-6)
    return sc, c, 1.0 / n


def _y_shift_partner(c, h):
    """Index of the cell one lattice spacing further in y (periodic) for every cell."""
    key = {(round(x / h * 6), round(y / h * 6) % round(6 / h)): i for i, (x, y) in enumerate(c)}
    return np.array([key[(round(x / h * 6), round((y + h) / h * 6) % round(6 / h))] for x, y in c])


def test_dry_strip_keeps_the_lattice_translation_invariance():
    """Wet/dry reading on data that depend on x only: the solution keeps the periodic lattice's
    invariance under translation by one cell in y (the vacuum sides, the front band and the dry
    interfaces treat translated cells alike), and it stays symmetric about the strip's centre line
    x = 0.375 in the thickness (the lattice's point reflection maps the strip onto itself)."""
    sc, c, h = _dry_strip_lattice()
    _, W, gW, t, n, hmin = _run(sc)
    assert t == pytest.approx(0.02) and hmin >= 0.0
    partner = _y_shift_partner(c, h)
    assert np.abs(W - W[:, partner]).max() < 1e-13
    assert np.abs(gW - gW[:, :, partner]).max() < 1e-11
    assert (W[0][(c[:, 0] > 0.5) & (c[:, 0] < 0.6)] > 1e-3).any()   # the strip spreads right
    assert (W[0][(c[:, 0] > 0.15) & (c[:, 0] < 0.25)] > 1e-3).any()  # and left
    # point reflection through (0.375, 0.5): thicknesses equal, x-momenta opposite
    k = round(6 / h)
    key = {(round(x / h * 6) % k, round(y / h * 6) % k): i for i, (x, y) in enumerate(c)}
    mirror = np.array([key[(round((0.75 - x) / h * 6) % k, round((1.0 - y) / h * 6) % k)] for x, y in c])
    for q in (0, 3):
        assert np.abs(W[q] - W[q][mirror]).max() < 1e-13
        assert np.abs(W[q + 1] + W[q + 1][mirror]).max() < 1e-13


def test_lower_layer_running_over_dry_land():
    """A lower layer dam-breaking over the Gaussian bump whose top stands dry (the case that needs
    the partially flooded cells in the front band: without them a thin sheet on the bump's flank
    is evolved at high order and its flux time derivative drains it below zero within 200 steps):
    to t = 0.3 no negative thickness and both layers' mass to round-off."""
    sc = w.dry_bump_dam_break(60)
    mesh, W, gW, t, n, hmin = _run(sc, t_end=0.3)
    assert t == pytest.approx(0.3) and np.isfinite(W).all()
    assert hmin >= 0.0
    a, _, _ = mesh.geometry()
    assert (sc.W0[3] == 0.0).sum() > 10  # dry land at the start
    for q in (0, 3):
        m0 = (a * sc.W0[q]).sum()
        assert abs((a * W[q]).sum() - m0) <= 1e-13 * m0
