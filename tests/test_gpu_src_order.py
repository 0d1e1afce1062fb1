"""The higher-order layer coupling (src_order 4; Sec. 3.2, Eq. SWE-source-discretization and its
closing remark) on the GPU against the oracle in the same mode: the interior correction cell by
cell, whole steps at the FP64 bound in both precisions' own bounds, the lake at rest kept, batches
equal to single runs, and bad values of the switch rejected."""
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


def _case(name):
    if name == "lake":
        return w.lake_at_rest(24, perturb=1e-2, seed=51)
    if name == "dam":
        return w.dam_break(20, seed=52)
    if name == "e1":
        return w.accuracy_e1(16)
    if name == "jittered":
        return w.smooth_jittered(16)
    return w.smooth_periodic(12)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-4)])
@pytest.mark.parametrize("case", ["jittered", "smooth", "e1"])
def test_interior_correction_matches_oracle(gks, case, precision, tol):
    """The correction k_recon writes (GKS_BUF_SRC) against om_coupling_correction, on the initial
    state: every component, relative to the largest of its kind (values, then rates).  The cases
    have both thicknesses varying (a lake at rest has none: its correction is round-off).  In the
    mixed path the correction is a small difference of FP32 reconstructions, about 1e-3 of the
    coupling term it is added to, so 1e-4 of its own size is 1e-7 of that term: FP32 rounding."""
    sc = _case(case)
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc, precision=precision, src_order=4)
    st.stage(0)
    got = st.buffer("src").astype(np.float64)
    om = o.Mesh.from_scenario(sc)
    ref = np.stack([o.coupling_correction(om, c, sc.W0, sc.gradW0, G=sc.G) for c in range(sc.n_tri)], axis=1)
    for rows in ((0, 1, 2, 3), (4, 5, 6, 7)):
        scale = np.abs(ref[list(rows)]).max()
        err = np.abs(got[list(rows)] - ref[list(rows)]).max() / scale
        print(f"[src4] {case} {precision} rows {rows}: scale {scale:.2e} err {err:.2e}", flush=True)
        assert scale > 0 and err < tol, (rows, err)


@pytest.mark.parametrize("case", ["lake", "dam", "smooth", "jittered"])
@pytest.mark.parametrize("nsteps", [1, 3])
def test_higher_order_coupling_matches_oracle(gks, case, nsteps):
    sc = _case(case)
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc, src_order=4)
    om = o.Mesh.from_scenario(sc)
    p = o.params_of(sc, src_order=4)
    Wr, gWr = sc.W0, sc.gradW0
    for _ in range(nsteps):
        dt = st.step(1, want_dt=True)
        Wr, gWr = o.step(om, p, dt, Wr, gWr)
    W, gW, _ = st.read()
    e, g = state_err(W, Wr).max(), grad_err(gW, gWr, Wr).max()
    print(f"[src4] {case} {nsteps} steps: state {e:.2e} grad {g:.2e}", flush=True)
    assert e < nsteps * TOL_FP64 and g < nsteps * TOL_FP64 * 10
    # the two forms differ on these flows
    ref = gks.State.from_scenario(m, sc)
    ref.step(nsteps)
    assert not np.array_equal(ref.read()[0], W)


@pytest.mark.parametrize("case", ["dam", "jittered"])
def test_higher_order_coupling_mixed_precision_close_to_oracle(gks, case):
    sc = _case(case)
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc, precision="fp32", src_order=4)
    om = o.Mesh.from_scenario(sc)
    p = o.params_of(sc, src_order=4)
    Wr, gWr = sc.W0, sc.gradW0
    for _ in range(3):
        dt = st.step(1, want_dt=True)
        Wr, gWr = o.step(om, p, dt, Wr, gWr)
    W, _, _ = st.read()
    e = state_err(W, Wr).max()
    print(f"[src4] {case} fp32 3 steps: state {e:.2e}", flush=True)
    assert e < 1e-5


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_higher_order_coupling_keeps_the_lake_at_rest(gks, precision):
    sc = w.lake_at_rest(32, seed=53)
    st = gks.State.from_scenario(gks.Mesh.from_scenario(sc), sc, precision=precision, src_order=4)
    st.step(200)
    W, _, _ = st.read()
    bound = 1e-12 if precision == "fp64" else 1e-9
    dev = max(np.abs(W[[1, 2, 4, 5]]).max(), np.abs(W[[0, 3]] - sc.W0[[0, 3]]).max())
    print(f"[src4] lake at rest {precision} 200 steps: {dev:.2e}", flush=True)
    assert dev < bound


def test_higher_order_coupling_batch_equals_single_runs(gks):
    """A batch with the higher-order coupling equals its single runs bit for bit, stepped eagerly
    and replayed from a graph."""
    scs = [w.lake_at_rest(10, perturb=1e-2, seed=60 + k) for k in range(3)]
    meshes = [gks.Mesh.from_scenario(s) for s in scs]
    bm = gks.Mesh.batch(meshes)
    bst = gks.State.from_scenarios(bm, scs, src_order=4)
    bst.step(4)
    Wb, _, _ = bst.read()
    gst = gks.State.from_scenarios(bm, scs, src_order=4)
    gst.batch_step(4)  # the same steps replayed from a captured HIP graph
    assert np.array_equal(gst.read()[0], Wb)
    off = 0
    for s, mm in zip(scs, meshes):
        st = gks.State.from_scenario(mm, s, src_order=4)
        st.step(4)
        W, _, _ = st.read()
        assert np.array_equal(W, Wb[:, off:off + s.n_tri])
        off += s.n_tri


def test_bad_src_order_is_rejected(gks):
    sc = w.lake_at_rest(6, seed=54)
    m = gks.Mesh.from_scenario(sc)
    with pytest.raises(gks.GksError) as ei:
        gks.State.from_scenario(m, sc, src_order=3)
    assert ei.value.code == gks.GKS_EINVAL
    st = gks.State.from_scenario(m, sc)
    st.stage(0)
    with pytest.raises(gks.GksError):
        st.buffer("src")  # only a state with the higher-order coupling has the correction


def test_full_size_dam_break_step_parity_higher_order_coupling(gks):
    """The 999,698-triangle two-layer dam break at full size with the higher-order coupling: one
    S2O4 step with the CFL step, every cell against the oracle's step in the same mode (in the
    second stage the front's new gradients make the interior correction non-zero)."""
    sc = w.dam_break(707, seed=20230605)
    print(f"[src4] full size dam break T={sc.n_tri}", flush=True)
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc, src_order=4)
    dt = st.step(1, want_dt=True)
    W, gW, _ = st.read()
    om = o.Mesh.from_scenario(sc)
    p = o.params_of(sc, src_order=4)
    dref = o.dt(om, p, sc.W0)
    assert abs(dt - dref) <= 4e-16 * dref
    Wr, gWr = o.step(om, p, dref, sc.W0, sc.gradW0)
    e, g = state_err(W, Wr), grad_err(gW, gWr, Wr)
    print(f"   state err {e.max():.2e} grad err {g.max():.2e}", flush=True)
    assert e.max() < TOL_FP64 and g.max() < TOL_FP64, (e, g)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_higher_order_coupling_with_the_fused_indicator(gks, precision):
    """The reconstruction variants that fuse the learned indicator also form the interior correction:
    a network whose logit is a constant 1 (all weights zero, output bias 1) skips every cell at
    threshold 0 and none at threshold 2, so three steps must equal, bit for bit, the linear
    reconstruction and the full one, each with the higher-order coupling."""
    sc = _case("jittered")
    m = gks.Mesh.from_scenario(sc)
    from paper_2306_04467_amd.gks import MLP_PARAMS

    P = np.zeros(MLP_PARAMS, dtype=np.float32)
    P[-1] = 1.0
    out = {}
    for name, kw, thr in (("skip_all", {}, 0.0), ("linear", {"linear": True}, None),
                          ("skip_none", {}, 2.0), ("full", {}, None)):
        st = gks.State.from_scenario(m, sc, precision=precision, src_order=4, **kw)
        if thr is not None:
            st.indicator(P, thr)
        st.step(3)
        out[name] = st.read()[0]
    assert np.array_equal(out["skip_all"], out["linear"])
    assert np.array_equal(out["skip_none"], out["full"])
    assert not np.array_equal(out["linear"], out["full"])
