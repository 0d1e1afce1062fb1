"""The discontinuous interface values of the gradient update (grad_mode 1; Sec. 3.3, the values
W^l != W^r at the inner sides of an edge) on the GPU against the oracle in the same mode: whole
steps at the FP64 bound, the mixed path at its own bound, the lake at rest kept, batches equal to
single runs (eager and graph), the full-size headline mesh, and bad values of the switch rejected."""
import numpy as np
import pytest

import oracle as o
import workloads as w
from tests._parity import TOL_FP64, grad_err, state_err

pytestmark = pytest.mark.gpu

GM = "discontinuous"


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
        return w.lake_at_rest(24, perturb=1e-2, seed=71)
    if name == "dam":
        return w.dam_break(20, seed=72)
    if name == "jittered":
        return w.smooth_jittered(16)
    if name == "free":
        return w.free_outflow(14)
    return w.smooth_periodic(12)


def _rel_l1(W, Wr, G, a):
    err = []
    for q in (0, 3):
        h = Wr[q]
        err.append((a * np.abs(W[q] - h)).sum() / (a * np.abs(h)).sum())
        den = (a * h * np.sqrt(G * h)).sum()
        for v in (q + 1, q + 2):
            err.append((a * np.abs(W[v] - Wr[v])).sum() / den)
    return max(err)


@pytest.mark.parametrize("case", ["lake", "dam", "smooth", "jittered", "free"])
@pytest.mark.parametrize("nsteps", [1, 3])
def test_discontinuous_gradient_update_matches_oracle(gks, case, nsteps):
    sc = _case(case)
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc, grad_mode=GM)
    om = o.Mesh.from_scenario(sc)
    p = o.params_of(sc, grad_mode=GM)
    Wr, gWr = sc.W0, sc.gradW0
    for _ in range(nsteps):
        dt = st.step(1, want_dt=True)
        Wr, gWr = o.step(om, p, dt, Wr, gWr)
    W, gW, _ = st.read()
    e, g = state_err(W, Wr).max(), grad_err(gW, gWr, Wr).max()
    print(f"[grad] {case} {nsteps} steps: state {e:.2e} grad {g:.2e}", flush=True)
    assert e < nsteps * TOL_FP64 and g < nsteps * TOL_FP64 * 10
    # the two readings give different gradients on these flows
    ref = gks.State.from_scenario(m, sc)
    ref.step(nsteps)
    assert not np.array_equal(ref.read()[1], gW)


@pytest.mark.parametrize("case", ["dam", "jittered"])
def test_discontinuous_gradient_update_mixed_precision(gks, case):
    """The mixed path in this mode: three steps within the mixed path's relative L1 bound of the
    oracle's FP64 steps."""
    sc = _case(case)
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc, precision="fp32", grad_mode=GM)
    om = o.Mesh.from_scenario(sc)
    p = o.params_of(sc, grad_mode=GM)
    a, _, _ = om.geometry()
    Wr, gWr = sc.W0, sc.gradW0
    for _ in range(3):
        dt = o.dt(om, p, Wr)
        st.stage(0, dt)
        st.stage(1)
        Wr, gWr = o.step(om, p, dt, Wr, gWr)
    W, _, _ = st.read()
    e = _rel_l1(W, Wr, sc.G, a)
    print(f"[grad] {case} fp32 3 steps: rel-L1 {e:.2e}", flush=True)
    assert e <= 1e-5


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_discontinuous_gradient_update_keeps_the_lake_at_rest(gks, precision):
    sc = w.lake_at_rest(32, seed=73)
    st = gks.State.from_scenario(gks.Mesh.from_scenario(sc), sc, precision=precision, grad_mode=GM)
    st.step(200)
    W, gW, _ = st.read()
    bound = 1e-12 if precision == "fp64" else 1e-9
    dev = max(np.abs(W[[1, 2, 4, 5]]).max(), np.abs(W[[0, 3]] - sc.W0[[0, 3]]).max())
    print(f"[grad] lake at rest {precision} 200 steps: {dev:.2e}", flush=True)
    assert dev < bound


def test_discontinuous_gradient_update_batch_equals_single_runs(gks):
    """A batch in this mode equals its single runs bit for bit, stepped eagerly and replayed from a
    captured graph (each replay checked against the eager steps)."""
    scs = [w.dam_break(8 + k, seed=74 + k) for k in range(3)]
    meshes = [gks.Mesh.from_scenario(s) for s in scs]
    bm = gks.Mesh.batch(meshes)
    bst = gks.State.from_scenarios(bm, scs, grad_mode=GM)
    gst = gks.State.from_scenarios(bm, scs, grad_mode=GM)
    for _ in range(3):
        bst.step(2)
        gst.batch_step(2)
        Wb, gWb, _ = bst.read()
        Wg, gWg, _ = gst.read()
        assert np.array_equal(Wg, Wb) and np.array_equal(gWg, gWb)
    off = 0
    for s, mm in zip(scs, meshes):
        st = gks.State.from_scenario(mm, s, grad_mode=GM)
        st.step(6)
        W, gW, _ = st.read()
        assert np.array_equal(W, Wb[:, off:off + s.n_tri])
        assert np.array_equal(gW, gWb[:, :, off:off + s.n_tri])
        off += s.n_tri


def test_bad_grad_mode_is_rejected(gks):
    sc = w.lake_at_rest(6, seed=75)
    m = gks.Mesh.from_scenario(sc)
    p = gks.make_params(G=sc.G, chi=sc.chi, cfl=sc.cfl)
    p.grad_mode = 2
    with pytest.raises(gks.GksError) as ei:
        gks.State(m, sc.W0, sc.gradW0, params=p)
    assert ei.value.code == gks.GKS_EINVAL
    # the scenarios of a batch share the reading
    scs = [w.lake_at_rest(5, seed=76), w.lake_at_rest(6, seed=77)]
    bm = gks.Mesh.batch([gks.Mesh.from_scenario(s) for s in scs])
    ps = [gks.make_params(G=s.G, chi=s.chi, cfl=s.cfl, grad_mode=gm) for s, gm in zip(scs, ("continuous", GM))]
    W0 = np.concatenate([s.W0 for s in scs], axis=1)
    gW0 = np.concatenate([s.gradW0 for s in scs], axis=2)
    with pytest.raises(gks.GksError) as ei:
        gks.State(bm, W0, gW0, params=ps)
    assert ei.value.code == gks.GKS_EINVAL


def test_full_size_headline_step_parity_discontinuous(gks):
    """The 520,200-triangle jittered-mesh lake with its disk perturbation at full size in this mode:
    one S2O4 step with the CFL step, every cell against the oracle's step.  The state is held to
    the FP64 bound; the gradients, Green-Gauss sums (Eq. slope-1) of terms as large as
    h |boundary| / |cell|, to ten times it: on this mesh's smallest cell (perimeter over area 1.04e4)
    one rounding of such a term is already 1.2e-12 of the thickness-gradient scale."""
    sc = w.build_config("C2")
    print(f"[grad] full size T={sc.n_tri}", flush=True)
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc, grad_mode=GM)
    dt = st.step(1, want_dt=True)
    W, gW, _ = st.read()
    om = o.Mesh.from_scenario(sc)
    p = o.params_of(sc, grad_mode=GM)
    dref = o.dt(om, p, sc.W0)
    assert abs(dt - dref) <= 4e-16 * dref
    Wr, gWr = o.step(om, p, dref, sc.W0, sc.gradW0)
    e, g = state_err(W, Wr), grad_err(gW, gWr, Wr)
    print(f"   state err {e.max():.2e} grad err {g.max():.2e}", flush=True)
    assert e.max() < TOL_FP64 and g.max() < 10 * TOL_FP64, (e, g)


@pytest.mark.parametrize("kw", [{"src_order": 4}, {"alpha_mode": "paper"}, {"src_order": 4, "alpha_mode": "paper"}])
@pytest.mark.parametrize("case", ["dam", "jittered"])
def test_discontinuous_gradient_values_with_the_other_options(gks, case, kw):
    """The discontinuous gradient values together with the higher-order coupling and the paper's
    alpha constants (the kernel instances that combine them): three steps against the oracle in
    the same modes at the FP64 bound."""
    sc = _case(case)
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc, grad_mode=GM, **kw)
    om = o.Mesh.from_scenario(sc)
    p = o.params_of(sc, grad_mode=GM, **kw)
    Wr, gWr = sc.W0, sc.gradW0
    for _ in range(3):
        dt = st.step(1, want_dt=True)
        Wr, gWr = o.step(om, p, dt, Wr, gWr)
    W, gW, _ = st.read()
    e, g = state_err(W, Wr).max(), grad_err(gW, gWr, Wr).max()
    print(f"[grad] {case} {kw}: state {e:.2e} grad {g:.2e}", flush=True)
    assert e < 3 * TOL_FP64 and g < 30 * TOL_FP64
