"""Wet/dry layers (h_dry > 0; the paper's dam breaks over a dry bed, Sec. 4) on the GPU against the
oracle in the same reading: steps at the FP64 bound on every wet/dry case, whole runs to the
paper's end times, Ritter's exact dam break onto a dry bed, the mixed path at its own bound,
batches equal to single runs (eager and graph), and bad parameter combinations rejected."""
import dataclasses

import numpy as np
import pytest

import oracle as o
import workloads as w
from tests._parity import TOL_FP64, scales

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gks():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2306_04467_amd as g

    g.load()
    return g


def _absent_upper():
    sc = w.lake_at_rest(16, chi=0.98, perturb=1e-2, seed=81)
    W0, gW0 = sc.W0.copy(), sc.gradW0.copy()
    W0[0] = 0.0
    gW0[0] = 0.0
    return dataclasses.replace(sc, W0=W0, gradW0=gW0, h_dry=1e-6)


CASES = {
    "ritter_lower": lambda: w.ritter_channel(60, layer="lower"),
    "ritter_upper": lambda: w.ritter_channel(60, layer="upper"),
    "dam_dry_chi1": lambda: w.dam_break_dry(30, chi=1.0),
    "dam_dry_chi02": lambda: w.dam_break_dry(30, chi=0.2),
    "breach_dry": lambda: w.dam_break_breach("dry", n=24),
    "breach_wet": lambda: w.dam_break_breach("wet", n=24),
    "absent_upper": _absent_upper,
    "dry_bump": lambda: w.dry_bump_dam_break(24),
}


def _errs(W, gW, Wr, gWr, G=9.81):
    """The parity measures of the other GPU tests, with each layer's scale floored by the other
    layer's (an absent layer has none of its own)."""
    sc = scales(Wr, G)
    sc[[0, 3]] = max(sc[0], sc[3])
    sc[[1, 2, 4, 5]] = max(sc[1], sc[4])
    e = max(np.abs(W[v] - Wr[v]).max() / sc[v] for v in range(6))
    g = max(np.abs(gW[v] - gWr[v]).max() / max(sc[v], np.abs(gWr[v]).max()) for v in range(6))
    return e, g


def _rel_l1(W, Wr, a):
    err = []
    for q in (0, 3):
        m = (a * np.abs(Wr[q])).sum()
        if m == 0:
            continue
        err.append((a * np.abs(W[q] - Wr[q])).sum() / m)
        scale = (a * np.abs(Wr[q + 1:q + 3])).sum() + 1e-300
        err.append((a * np.abs(W[q + 1:q + 3] - Wr[q + 1:q + 3])).sum() / scale)
    return max(err)


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("nsteps", [1, 3, 10])
def test_wet_dry_steps_match_oracle(gks, case, nsteps):
    sc = CASES[case]()
    print(f"[wd] {case} T={sc.n_tri} {nsteps} steps", flush=True)
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc)
    om = o.Mesh.from_scenario(sc)
    p = o.params_of(sc)
    Wr, gWr = sc.W0, sc.gradW0
    ddt = 0.0
    for _ in range(nsteps):
        dt = st.step(1, want_dt=True)
        ddt = max(ddt, abs(dt - o.dt(om, p, Wr)) / dt)
        Wr, gWr = o.step(om, p, dt, Wr, gWr)
    W, gW, _ = st.read()
    e, g = _errs(W, gW, Wr, gWr)
    print(f"   state {e:.2e} grad {g:.2e} dt {ddt:.1e} min h {W[[0, 3]].min():.1e}", flush=True)
    # the largest speed may sit in a front cell a millionth of the depth thick, whose velocity
    # carries the state's absolute rounding (1e-16 of the depth) relative to its own thickness
    assert ddt < 1e-8
    assert e < nsteps * TOL_FP64 and g < nsteps * TOL_FP64 * 10
    assert W[[0, 3]].min() > -1e-6


@pytest.mark.parametrize("case", ["dam_dry_chi1", "dam_dry_chi02", "breach_dry", "dry_bump"])
def test_wet_dry_run_to_end_time_matches_oracle(gks, case):
    """Whole runs to the end times (t = 0.08 for the paper's two-layer dam break, 7.2 for the
    breached dam, 0.5 for the lower layer running over the dry-topped bump): the device keeps every
    thickness above -h_dry (the non-finite / negative flag is never raised), both layers' mass to
    round-off, and the final state within 1e-9 (relative L1) of the oracle's run."""
    sc = CASES[case]()
    print(f"[wd] {case} to t={sc.t_end}", flush=True)
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc, t_end=sc.t_end)
    om = o.Mesh.from_scenario(sc)
    p = o.params_of(sc)
    a, _, _ = om.geometry()
    Wr, gWr, t_ref, n_ref = o.run(om, p, sc.W0, sc.gradW0, sc.t_end)
    n = 0
    while True:
        st.step(100)
        n += 100
        t, _ = st.time()
        if t >= sc.t_end or n > 50 * n_ref:
            break
    W, gW, t = st.read()
    assert t == pytest.approx(sc.t_end)
    mass = st.mass()
    for k, q in enumerate((0, 3)):
        m0 = (a * sc.W0[q]).sum()
        assert abs((a * W[q]).sum() - m0) <= 1e-13 * m0
    e = _rel_l1(W, Wr, a)
    print(f"   {n_ref} oracle steps, rel-L1 vs oracle {e:.2e}, min h {W[[0, 3]].min():.1e}, mass {mass}", flush=True)
    assert e < 1e-9
    assert W[[0, 3]].min() >= -1e-12


def test_ritter_dam_break_on_the_gpu(gks):
    """Ritter's exact dam break onto a dry bed at cell size 1/100 on the GPU: the same error bound
    as the oracle's pin (relative L1 of the thickness under 0.5 %), no negative thickness, mass to
    round-off, the absent layer exactly zero."""
    sc = w.ritter_channel(200, layer="lower")
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc, t_end=sc.t_end)
    st.step(2000)
    W, gW, t = st.read()
    assert t == pytest.approx(sc.t_end)
    om = o.Mesh.from_scenario(sc)
    a, _, _ = om.geometry()
    ex = sc.exact(t)
    e = (a * np.abs(W[3] - ex[3])).sum() / (a * ex[3]).sum()
    print(f"[wd] Ritter on the GPU: rel L1 {e:.3e} min h {W[3].min():.1e}", flush=True)
    assert e < 0.005 and W[3].min() >= 0.0
    assert abs((a * W[3]).sum() - (a * sc.W0[3]).sum()) <= 1e-13 * (a * sc.W0[3]).sum()
    assert np.all(W[0:3] == 0.0)


@pytest.mark.parametrize("case", ["ritter_lower", "dam_dry_chi02", "breach_wet"])
def test_wet_dry_mixed_precision(gks, case):
    """The mixed path with wet/dry layers: three steps within 1e-5 (relative L1) of the oracle's
    FP64 steps."""
    sc = CASES[case]()
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc, precision="fp32")
    om = o.Mesh.from_scenario(sc)
    p = o.params_of(sc)
    a, _, _ = om.geometry()
    Wr, gWr = sc.W0, sc.gradW0
    for _ in range(3):
        dt = o.dt(om, p, Wr)
        st.stage(0, dt)
        st.stage(1)
        Wr, gWr = o.step(om, p, dt, Wr, gWr)
    W, _, _ = st.read()
    e = _rel_l1(W, Wr, a)
    print(f"[wd] {case} fp32 3 steps: rel-L1 {e:.2e}", flush=True)
    assert e <= 1e-5


def test_wet_dry_batch_equals_single_runs(gks):
    """A batch of wet/dry scenarios equals its single runs bit for bit, stepped eagerly and
    replayed from a captured graph (each replay checked against the eager steps)."""
    scs = [w.ritter_channel(40, layer="lower"), w.dam_break_dry(20, chi=0.2), w.dam_break_breach("dry", n=16)]
    meshes = [gks.Mesh.from_scenario(s) for s in scs]
    bm = gks.Mesh.batch(meshes)
    bst = gks.State.from_scenarios(bm, scs)
    gst = gks.State.from_scenarios(bm, scs)
    for _ in range(3):
        bst.step(4)
        gst.batch_step(4)
        Wb, gWb, _ = bst.read()
        Wg, gWg, _ = gst.read()
        assert np.array_equal(Wg, Wb) and np.array_equal(gWg, gWb)
    off = 0
    for s, mm in zip(scs, meshes):
        st = gks.State.from_scenario(mm, s)
        st.step(12)
        W, gW, _ = st.read()
        assert np.array_equal(W, Wb[:, off:off + s.n_tri])
        assert np.array_equal(gW, gWb[:, :, off:off + s.n_tri])
        off += s.n_tri


def test_wet_dry_parameters_checked(gks):
    sc = w.dam_break_dry(10)
    m = gks.Mesh.from_scenario(sc)
    for h_dry in (-1e-6, float("nan"), float("inf")):
        with pytest.raises(gks.GksError) as ei:
            gks.State.from_scenario(m, sc, h_dry=h_dry)
        assert ei.value.code == gks.GKS_EINVAL
    with pytest.raises(gks.GksError) as ei:
        gks.State.from_scenario(m, sc, src_order=4)  # wet/dry needs the second-order coupling
    assert ei.value.code == gks.GKS_EINVAL
    with pytest.raises(gks.GksError) as ei:
        gks.State.from_scenario(m, sc, h_dry=0.0)  # a zero thickness needs wet/dry layers
    assert ei.value.code == gks.GKS_ENONFINITE
    st = gks.State.from_scenario(m, sc)
    with pytest.raises(gks.GksError) as ei:
        st.indicator(np.zeros(7105, dtype=np.float32), 0.0)
    assert ei.value.code == gks.GKS_EINVAL
    scs = [w.ritter_channel(20), w.ritter_channel(20, h_dry=1e-5)]
    bm = gks.Mesh.batch([gks.Mesh.from_scenario(s) for s in scs])
    with pytest.raises(gks.GksError) as ei:
        gks.State.from_scenarios(bm, scs)
    assert ei.value.code == gks.GKS_EINVAL


@pytest.mark.parametrize("case", ["dam_dry_fine", "breach_dry_full"])
def test_wet_dry_full_size_step_parity(gks, case):
    """The timed wet/dry workloads at full size: the paper's dam break at its fine cell size 1/400
    (160,000 triangles) and the breached dam over a dry bed (406,000 triangles); one S2O4 step with
    the CFL step, then a second, every cell against the oracle."""
    sc = w.dam_break_dry(400, chi=1.0) if case == "dam_dry_fine" else w.dam_break_breach("dry", n=400)
    print(f"[wd] full size {case} T={sc.n_tri}", flush=True)
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc)
    om = o.Mesh.from_scenario(sc)
    p = o.params_of(sc)
    Wr, gWr = sc.W0, sc.gradW0
    for k in range(2):
        dt = st.step(1, want_dt=True)
        dref = o.dt(om, p, Wr)
        assert abs(dt - dref) <= 1e-8 * dref
        Wr, gWr = o.step(om, p, dt, Wr, gWr)
    W, gW, _ = st.read()
    e, g = _errs(W, gW, Wr, gWr)
    print(f"   state {e:.2e} grad {g:.2e} min h {W[[0, 3]].min():.1e}", flush=True)
    assert e < 2 * TOL_FP64 and g < 20 * TOL_FP64
    assert W[[0, 3]].min() >= 0.0


@pytest.mark.parametrize("grad_mode,alpha_mode", [("discontinuous", "reading"), ("continuous", "paper"),
                                                  ("discontinuous", "paper")])
@pytest.mark.parametrize("case", ["dam_dry_chi02", "breach_wet"])
def test_wet_dry_with_the_other_options(gks, case, grad_mode, alpha_mode):
    """Wet/dry layers together with the discontinuous gradient values and the paper's alpha
    constants (the flux instances that combine them): three steps against the oracle in the same
    modes at the FP64 bound."""
    sc = CASES[case]()
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc, grad_mode=grad_mode, alpha_mode=alpha_mode)
    om = o.Mesh.from_scenario(sc)
    p = o.params_of(sc, grad_mode=grad_mode, alpha_mode=alpha_mode)
    Wr, gWr = sc.W0, sc.gradW0
    for _ in range(3):
        dt = st.step(1, want_dt=True)
        Wr, gWr = o.step(om, p, dt, Wr, gWr)
    W, gW, _ = st.read()
    e, g = _errs(W, gW, Wr, gWr)
    print(f"[wd] {case} {grad_mode} {alpha_mode}: state {e:.2e} grad {g:.2e}", flush=True)
    assert e < 3 * TOL_FP64 and g < 30 * TOL_FP64


def test_dry_strip_on_the_periodic_lattice(gks):
    """A strip of upper layer over a uniform lower one on the periodic lattice, dry elsewhere, to
    t = 0.02: the GPU run equals the oracle's at the FP64 bound and keeps the lattice's invariance
    under translation by one cell in y."""
    from tests.test_oracle_wetdry import _dry_strip_lattice, _y_shift_partner

    sc, c, h = _dry_strip_lattice()
    st = gks.State.from_scenario(gks.Mesh.from_scenario(sc), sc, t_end=sc.t_end)
    om = o.Mesh.from_scenario(sc)
    p = o.params_of(sc)
    Wr, gWr = sc.W0, sc.gradW0
    n = 0
    while st.time()[0] < sc.t_end:
        dt = st.step(1, want_dt=True)
        Wr, gWr = o.step(om, p, dt, Wr, gWr)
        n += 1
    W, gW, _ = st.read()
    e, g = _errs(W, gW, Wr, gWr)
    partner = _y_shift_partner(c, h)
    print(f"[wd] dry strip {n} steps: state {e:.2e} grad {g:.2e}", flush=True)
    assert e < n * TOL_FP64 and g < n * TOL_FP64 * 10
    assert np.abs(W - W[:, partner]).max() < 1e-13
