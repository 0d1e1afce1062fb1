"""Parity of the HIP path (through the C ABI) with the FP64 oracle, on the GPU.

Each case runs the same seeded input through gks_stage / gks_step and through the oracle and
compares cell averages and cell-averaged gradients component by component (tests/_parity.py),
at 1e-12 of the component's scale per step.
"""
import numpy as np
import pytest

import oracle as o
import workloads as w
from tests._parity import TOL_FP64, grad_err, state_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gks():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2306_04467_amd as g

    g.load()
    return g


def _pair(gks, sc, linear=False):
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc, linear=linear)
    om = o.Mesh.from_scenario(sc)
    return m, st, om, o.params_of(sc, linear=linear)


CASES = {
    "periodic_n8": lambda: w.smooth_periodic(8),
    "periodic_n20": lambda: w.smooth_periodic(20),
    "wall_bump_perturbed_n12": lambda: w.lake_at_rest(12, perturb=1e-2, seed=3),
    "dam_break_n14": lambda: w.dam_break(14, bump_amp=0.2),
}


@pytest.mark.parametrize("case", list(CASES))
def test_stage0_parity(gks, case):
    sc = CASES[case]()
    m, st, om, p = _pair(gks, sc)
    dt = o.dt(om, p, sc.W0)
    print(f"[parity] {case}: T={sc.n_tri} stage 0", flush=True)
    st.stage(0, dt)
    W, gW, t = st.read()
    Wr, gWr = o.step(om, p, dt, sc.W0, sc.gradW0, nstages=1)
    e, g = state_err(W, Wr), grad_err(gW, gWr, Wr)
    print(f"   stage-0 state err {e.max():.2e} grad err {g.max():.2e}", flush=True)
    assert e.max() < TOL_FP64, e
    assert g.max() < TOL_FP64, g
    assert abs(t - 0.5 * dt) <= 1e-15 * dt


@pytest.mark.parametrize("case", list(CASES))
def test_multistep_parity(gks, case):
    sc = CASES[case]()
    m, st, om, p = _pair(gks, sc)
    W, gW = sc.W0.copy(), sc.gradW0.copy()
    print(f"[parity] {case}: T={sc.n_tri} 5 steps", flush=True)
    for n in range(5):
        dt = o.dt(om, p, W)
        st.stage(0, dt)
        st.stage(1)
        W, gW = o.step(om, p, dt, W, gW)
        Wg, gWg, _ = st.read()
        e, g = state_err(Wg, W), grad_err(gWg, gW, W)
        assert e.max() < TOL_FP64 * (n + 1), (n, e)
        assert g.max() < TOL_FP64 * (n + 1), (n, g)


def test_linear_reconstruction_parity(gks):
    sc = w.dam_break(12, bump_amp=0.2)
    m, st, om, p = _pair(gks, sc, linear=True)
    dt = o.dt(om, p, sc.W0)
    st.stage(0, dt)
    st.stage(1)
    W, gW, _ = st.read()
    Wr, gWr = o.step(om, p, dt, sc.W0, sc.gradW0)
    assert state_err(W, Wr).max() < TOL_FP64
    assert grad_err(gW, gWr, Wr).max() < TOL_FP64


def test_device_time_step_matches_oracle(gks):
    sc = w.lake_at_rest(12, perturb=1e-2, seed=5)
    m, st, om, p = _pair(gks, sc)
    dt = st.step(1, want_dt=True)
    dref = o.dt(om, p, sc.W0)
    assert abs(dt - dref) <= 4e-16 * dref
    W, gW, t = st.read()
    Wr, gWr = o.step(om, p, dref, sc.W0, sc.gradW0)
    assert state_err(W, Wr).max() < TOL_FP64


def test_time_clipped_to_t_end(gks):
    sc = w.smooth_periodic(8)
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc, t_end=0.0123)
    st.step(40)
    _, _, t = st.read()
    assert abs(t - 0.0123) < 1e-15


def test_lake_at_rest_on_gpu(gks):
    sc = w.lake_at_rest(16, chi=0.98)
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc)
    st.step(200)
    W, gW, _ = st.read()
    assert np.abs(W[[1, 2, 4, 5]]).max() < 1e-13
    assert np.abs(W[[0, 3]] - sc.W0[[0, 3]]).max() < 1e-13
    assert np.abs(gW - sc.gradW0).max() < 1e-11


def test_layer_mass_on_gpu(gks):
    sc = w.dam_break(16, bump_amp=0.2)
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc)
    m0 = st.mass()
    om = o.Mesh.from_scenario(sc)
    np.testing.assert_allclose(m0, o.mass(om, sc.W0), rtol=1e-14)
    st.step(30)
    m1 = st.mass()
    assert np.all(np.abs(m1 - m0) <= 30 * 1e-14 * m0), (m1 - m0) / m0


def test_bitwise_deterministic(gks):
    sc = w.dam_break(16, bump_amp=0.2)
    out = []
    for _ in range(2):
        m = gks.Mesh.from_scenario(sc)
        st = gks.State.from_scenario(m, sc)
        st.step(10)
        out.append(st.read())
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_rejects_bad_input(gks):
    sc = w.smooth_periodic(6)
    m = gks.Mesh.from_scenario(sc)
    W = sc.W0.copy()
    W[3, 5] = -1.0
    with pytest.raises(gks.GksError) as ei:
        gks.State(m, W, sc.gradW0)
    assert ei.value.code == 5
    W[3, 5] = np.nan
    with pytest.raises(gks.GksError):
        gks.State(m, W, sc.gradW0)
    st = gks.State.from_scenario(m, sc)
    with pytest.raises(gks.GksError):
        st.stage(0, -1.0)


def test_full_size_step_parity(gks):
    """The benchmarked workload at full size (520,200 triangles): one S2O4 step with the device's
    CFL step, every cell compared with the oracle's step."""
    sc = w.lake_at_rest(510, seed=20230604, perturb=1e-3, disk=(0.3, 0.3, 0.1))
    print(f"[parity] full size T={sc.n_tri}", flush=True)
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc)
    dt = st.step(1, want_dt=True)
    W, gW, _ = st.read()
    om = o.Mesh.from_scenario(sc)
    p = o.params_of(sc)
    dref = o.dt(om, p, sc.W0)
    assert abs(dt - dref) <= 4e-16 * dref
    Wr, gWr = o.step(om, p, dref, sc.W0, sc.gradW0)
    e, g = state_err(W, Wr), grad_err(gW, gWr, Wr)
    print(f"   state err {e.max():.2e} grad err {g.max():.2e}", flush=True)
    assert e.max() < TOL_FP64 and g.max() < TOL_FP64, (e, g)


_DAM_BREAK_REF = {}


def _dam_break_reference():
    """The 1M-triangle dam break and the oracle's first step on it (computed once per session)."""
    if not _DAM_BREAK_REF:
        sc = w.dam_break(707, seed=20230605)
        om = o.Mesh.from_scenario(sc)
        p = o.params_of(sc)
        dref = o.dt(om, p, sc.W0)
        Wr, gWr = o.step(om, p, dref, sc.W0, sc.gradW0)
        a, _, _ = om.geometry()
        _DAM_BREAK_REF.update(sc=sc, dt=dref, W=Wr, gW=gWr, area=a)
    return _DAM_BREAK_REF


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_full_size_dam_break_step_parity(gks, precision):
    """The 999,698-triangle two-layer dam break over a sinusoidal bottom (density ratio 0.95) at
    full size: one S2O4 step with the CFL step, every cell against the oracle's step.  Here the
    nonlinear weights, the force model's plane gradients and the collision time's jump term are
    all active.  FP64 to the per-step bound; the mixed path to its relative L1 bound."""
    print(f"[parity] dam break {precision}, 999,698 triangles (oracle step computed once)", flush=True)
    ref = _dam_break_reference()
    sc, dref, Wr, gWr = ref["sc"], ref["dt"], ref["W"], ref["gW"]
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc, precision=precision)
    st.stage(0, dref)
    st.stage(1)
    W, gW, _ = st.read()
    if precision == "fp64":
        e, g = state_err(W, Wr), grad_err(gW, gWr, Wr)
        print(f"   state err {e.max():.2e} grad err {g.max():.2e}", flush=True)
        assert e.max() < TOL_FP64 and g.max() < TOL_FP64, (e, g)
    else:
        a = ref["area"]
        err = []
        for q in (0, 3):
            h = Wr[q]
            err.append((a * np.abs(W[q] - h)).sum() / (a * np.abs(h)).sum())
            den = (a * h * np.sqrt(sc.G * h)).sum()
            for v in (q + 1, q + 2):
                err.append((a * np.abs(W[v] - Wr[v])).sum() / den)
        print(f"   rel-L1 {max(err):.2e}", flush=True)
        assert max(err) <= 1e-5, err
