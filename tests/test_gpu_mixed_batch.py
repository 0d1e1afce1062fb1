"""GPU tests of the mixed-precision path and of batched ensembles (through the C ABI).

Mixed precision (FP32 bulk, FP64 hydrostatic balance and thicknesses): error against the FP64
oracle measured as the relative L1 error of the benchmark metric (area-weighted; momenta against
h sqrt(G h)), lake at rest and per-layer mass.  Batches: a batch of independent meshes advanced in
one set of launches must reproduce each scenario's own run bit for bit in FP64, and the
graph-replayed steps must equal the eagerly launched ones.
"""
import numpy as np
import pytest

import oracle as o
import workloads as w
from tests._parity import TOL_FP64, grad_err, state_err

pytestmark = pytest.mark.gpu

TOL_FP32_REL_L1 = 1e-5  # relative L1 error of the mixed path against the FP64 oracle


@pytest.fixture(scope="module")
def gks():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2306_04467_amd as g

    g.load()
    return g


def rel_l1(W, Wr, area, G=9.81):
    out = []
    for o_ in (0, 3):
        h = Wr[o_]
        out.append((area * np.abs(W[o_] - h)).sum() / (area * np.abs(h)).sum())
        den = (area * h * np.sqrt(G * h)).sum()
        for v in (o_ + 1, o_ + 2):
            out.append((area * np.abs(W[v] - Wr[v])).sum() / den)
    return np.array(out)


@pytest.mark.parametrize("make", [lambda: w.dam_break(24, bump_amp=0.2),
                                  lambda: w.lake_at_rest(24, perturb=1e-2, seed=4),
                                  lambda: w.smooth_periodic(20)])
def test_mixed_precision_error_against_oracle(gks, make):
    sc = make()
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc, precision="fp32")
    om = o.Mesh.from_scenario(sc)
    p = o.params_of(sc)
    a, _, _ = om.geometry()
    W, gW = sc.W0.copy(), sc.gradW0.copy()
    for n in range(20):
        dt = o.dt(om, p, W)
        st.stage(0, dt)
        st.stage(1)
        W, gW = o.step(om, p, dt, W, gW)
    Wg, _, _ = st.read()
    err = rel_l1(Wg, W, a)
    print(f"[mixed] {sc.name}: rel-L1 after 20 steps {err.max():.2e}", flush=True)
    assert err.max() < TOL_FP32_REL_L1, err


def test_mixed_precision_lake_at_rest(gks):
    sc = w.lake_at_rest(16, chi=0.98)
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc, precision="fp32")
    st.step(200)
    W, gW, _ = st.read()
    mom = np.abs(W[[1, 2, 4, 5]]).max()
    dh = np.abs(W[[0, 3]] - sc.W0[[0, 3]]).max()
    print(f"[mixed] lake at rest 200 steps: max|hU| {mom:.2e}, max|dh| {dh:.2e}", flush=True)
    # the hydrostatic balance is FP64 and every FP32 term vanishes exactly at rest (mirror-image
    # left/right sums, closed-form bottom moments), so the bound is the FP64 path's
    assert mom < 1e-13
    assert dh < 1e-13


def test_mixed_precision_mass(gks):
    sc = w.dam_break(16, bump_amp=0.2)
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc, precision="fp32")
    m0 = st.mass()
    st.step(30)
    m1 = st.mass()
    assert np.all(np.abs(m1 - m0) <= 30 * 1e-14 * m0), (m1 - m0) / m0


def _small_ensemble():
    return [w.lake_at_rest(6, seed=31, chi=0.93, perturb=3e-3),
            w.dam_break(9, seed=32, chi=0.97),
            w.lake_at_rest(11, seed=33, chi=0.91, perturb=1e-2)]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_matches_individual_runs(gks, precision):
    scs = _small_ensemble()
    singles = []
    for sc in scs:
        m = gks.Mesh.from_scenario(sc)
        st = gks.State.from_scenario(m, sc, precision=precision)
        st.step(6)
        singles.append((st.read(), st.time()))
    meshes = [gks.Mesh.from_scenario(sc) for sc in scs]
    bm = gks.Mesh.batch(meshes)
    assert bm.n_scenarios == len(scs) and bm.n_tri == sum(s.n_tri for s in scs)
    bs = gks.State.from_scenarios(bm, scs, precision=precision)
    bs.step(6)
    Wb, gWb, _ = bs.read()
    for i, sc in enumerate(scs):
        c0, n = bm.scenario_range(i)
        (W, gW, _), (t, dt) = singles[i]
        assert np.array_equal(Wb[:, c0:c0 + n], W), i
        assert np.array_equal(gWb[:, :, c0:c0 + n], gW), i
        assert bs.time(i) == (t, dt)


def test_batch_graph_replay_matches_eager_steps(gks):
    scs = _small_ensemble()
    out = []
    for graph in (False, True):
        bm = gks.Mesh.batch([gks.Mesh.from_scenario(sc) for sc in scs])
        bs = gks.State.from_scenarios(bm, scs, precision="fp32")
        if graph:
            bs.batch_step(5)
            bs.batch_step(3)
        else:
            bs.step(8)
        out.append(bs.read())
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_two_batches_on_two_streams_match_the_whole_batch(gks, precision):
    """An ensemble split into two batch states on two streams, their graph replays interleaved so
    that the GPU may run both at once, gives every scenario the state the whole batch gives it, bit
    for bit: the states share no device memory."""
    import ctypes

    import torch

    scs = [w.lake_at_rest(40, seed=41, chi=0.93, perturb=3e-3), w.dam_break(50, seed=42, chi=0.97),
           w.lake_at_rest(45, seed=43, chi=0.91, perturb=1e-2), w.dam_break(35, seed=44, chi=0.95)]
    bm = gks.Mesh.batch([gks.Mesh.from_scenario(sc) for sc in scs])
    whole = gks.State.from_scenarios(bm, scs, precision=precision)
    whole.batch_step(7)
    Ww, gWw, _ = whole.read()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    parts = []
    for idx, strm in zip(([0, 2], [1, 3]), streams):
        sub = [scs[i] for i in idx]
        m = gks.Mesh.batch([gks.Mesh.from_scenario(sc) for sc in sub])
        st = gks.State.from_scenarios(m, sub, precision=precision, stream=ctypes.c_void_p(strm.cuda_stream))
        parts.append((idx, m, st))
    for _ in range(7):
        for _, _, st in parts:
            st.batch_step(1)
    torch.cuda.synchronize()
    for idx, m, st in parts:
        W, gW, _ = st.read()
        for j, i in enumerate(idx):
            c0, n = bm.scenario_range(i)
            d0, dn = m.scenario_range(j)
            assert dn == n
            assert np.array_equal(W[:, d0:d0 + n], Ww[:, c0:c0 + n]), i
            assert np.array_equal(gW[:, :, d0:d0 + n], gWw[:, :, c0:c0 + n]), i
            assert st.time(j) == whole.time(i), i


def test_scenarios_stop_at_their_end_times(gks):
    """A scenario that reaches its t_end stays unchanged by later steps while the others go on:
    the finished one equals its own single run stopped at t_end, bit for bit."""
    scs = _small_ensemble()
    t_ends = [0.004, 0.0, 0.011]              # 0: no end time
    for sc, te in zip(scs, t_ends):
        sc.t_end = te if te > 0 else 1e300
    singles = []
    for sc, te in zip(scs, t_ends):
        st = gks.State.from_scenario(gks.Mesh.from_scenario(sc), sc, t_end=te)
        st.step(30)
        singles.append(st.read())
    bm = gks.Mesh.batch([gks.Mesh.from_scenario(sc) for sc in scs])
    bs = gks.State.from_scenarios(bm, scs)
    bs.batch_step(30)
    Wb, gWb, _ = bs.read()
    for i, (sc, te) in enumerate(zip(scs, t_ends)):
        c0, n = bm.scenario_range(i)
        W, gW, t = singles[i]
        assert np.isfinite(Wb).all()
        assert np.array_equal(Wb[:, c0:c0 + n], W) and np.array_equal(gWb[:, :, c0:c0 + n], gW), i
        tb, _ = bs.time(i)
        if te > 0:
            assert tb == te and t == te, (i, tb, t)
        else:
            assert tb > 0.011


def test_autotune_restores_the_state_and_changes_no_result(gks):
    """The autotuner times several launch shapes on the state itself; afterwards the state is the
    one it was given, and the chosen shapes give the same results bit for bit (graph replay)."""
    scs = _small_ensemble()
    bm = gks.Mesh.batch([gks.Mesh.from_scenario(sc) for sc in scs])
    ref = gks.State.from_scenarios(bm, scs, precision="fp32")
    tuned = gks.State.from_scenarios(bm, scs, precision="fp32")
    tuned.step(2)
    ref.step(2)
    W0, gW0, _ = tuned.read()
    t0 = [tuned.time(i) for i in range(len(scs))]
    chosen = tuned.autotune(reps=2)
    W1, gW1, _ = tuned.read()
    assert np.array_equal(W0, W1) and np.array_equal(gW0, gW1)
    assert [tuned.time(i) for i in range(len(scs))] == t0
    for k in ("ghost", "hhat", "plane", "flux", "update"):
        assert chosen[k] in (64, 128, 256), chosen
    tuned.batch_step(4)
    ref.batch_step(4)
    Wa, gWa, _ = tuned.read()
    Wr, gWr, _ = ref.read()
    assert np.array_equal(Wa, Wr) and np.array_equal(gWa, gWr)


def test_batch_scenario_against_oracle(gks):
    scs = _small_ensemble()
    bm = gks.Mesh.batch([gks.Mesh.from_scenario(sc) for sc in scs])
    bs = gks.State.from_scenarios(bm, scs)
    bs.batch_step(3)
    Wb, gWb, _ = bs.read()
    for i, sc in enumerate(scs):
        om = o.Mesh.from_scenario(sc)
        p = o.params_of(sc)
        W, gW = sc.W0.copy(), sc.gradW0.copy()
        for _ in range(3):
            W, gW = o.step(om, p, o.dt(om, p, W), W, gW)
        c0, n = bm.scenario_range(i)
        assert state_err(Wb[:, c0:c0 + n], W).max() < 3 * TOL_FP64
        assert grad_err(gWb[:, :, c0:c0 + n], gW, W).max() < 3 * TOL_FP64
        m0 = o.mass(om, sc.W0)
        np.testing.assert_allclose(bs.mass(i), m0, rtol=1e-13)
