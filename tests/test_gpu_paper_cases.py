"""The paper's own test cases run on the GPU: the accuracy table of the translating two-layer
Gaussian (Sec. 4.1, table of L1 errors at t = 0.1) in both precisions, the lake at rest over a
bump (Sec. 4.2) over 1000 steps on the 520,200-triangle mesh, and the well-balance test's
geometry run to its end time t = 100."""
import json
import math
import os

import numpy as np
import pytest

import workloads as w

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def gks():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2306_04467_amd as g

    g.load()
    return g


def _e1_error(gks, n, precision):
    sc = w.accuracy_e1(n)
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc, precision=precision, t_end=sc.t_end)
    st.step(10000 // n)            # the CFL step needs fewer; steps after t_end stay at t_end
    W, _, t = st.read()
    assert abs(t - sc.t_end) < 1e-14
    ex = sc.exact(t)
    xy = sc.node_xy[sc.tri]
    a = 0.5 * np.abs((xy[:, 1, 0] - xy[:, 0, 0]) * (xy[:, 2, 1] - xy[:, 0, 1])
                     - (xy[:, 1, 1] - xy[:, 0, 1]) * (xy[:, 2, 0] - xy[:, 0, 0]))
    return [(a * np.abs(W[v] - ex[v])).sum() / a.sum() for v in (3, 0)]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_accuracy_table_on_gpu(gks, precision):
    """At most 3 times and at least a quarter of the printed errors, mean order >= 1.9 (see the
    oracle pin of the same table: the nonlinear weights cost the paper's order on this problem)."""
    with open(os.path.join(GOLDEN, "accuracy_table.json")) as f:
        gold = json.load(f)
    errs = {"1/8": _e1_error(gks, 16, precision), "1/16": _e1_error(gks, 32, precision),
            "1/32": _e1_error(gks, 64, precision)}
    print(f"[paper] E1 {precision}: {errs}", flush=True)
    for v, key in ((0, "h1"), (1, "h2")):
        for row, e in errs.items():
            ref = gold["rows"][row][key]
            assert ref / 4 < e[v] < 3 * ref, (key, row, e[v], ref)
        assert 0.5 * math.log2(errs["1/8"][v] / errs["1/32"][v]) > 1.9


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_lake_at_rest_1000_steps(gks, precision):
    """The unperturbed 520,200-triangle lake at rest (bump 0.5 exp(-50 r^2), lower level 0.8, upper
    layer 0.2, density ratio 0.98, walls) over 1000 steps: momenta against h sqrt(G h), levels
    against h.  The state is an exact fixed point of the scheme.  Round-off seeds modes that the
    compact gradient update amplifies at a few obtuse cells of this jittered mesh while the
    reconstruction runs on its linear weights (the oracle does the same on a patch of the mesh);
    the nonlinear weights engage at the floor of the smoothness indicators, which sits near
    round-off for a momentum at rest, and hold the deviation there: 1e-12 of the scale in FP64
    (measured 7e-14 / 2e-13), 1e-10 in the mixed path, whose momenta are single precision."""
    sc = w.lake_at_rest(510)
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc, precision=precision)
    G = sc.G
    for k in range(4):
        st.batch_step(250)
        W, gW, _ = st.read()
        assert np.isfinite(W).all() and np.isfinite(gW).all()
        mom = max(np.abs(W[1:3]).max() / (0.2 * math.sqrt(G * 0.2)),
                  np.abs(W[4:6]).max() / (0.3 * math.sqrt(G * 0.3)))
        dh = max(np.abs(W[3] - sc.W0[3]).max() / 0.3, np.abs(W[0] - sc.W0[0]).max() / 0.2)
        print(f"[paper] lake at rest {precision} {250 * (k + 1)} steps: scaled max|hU| {mom:.2e} "
              f"max|dh| {dh:.2e}", flush=True)
        bound = 1e-12 if precision == "fp64" else 1e-10
        assert mom < bound and dh < bound


@pytest.mark.parametrize("chi,precision,bound", [(0.9, "fp64", 1e-11), (0.9, "fp32", 1e-6),
                                                 (1.0, "fp64", 1e-8), (1.0, "fp32", 1e-4)])
def test_well_balance_test_to_t100(gks, chi, precision, bound):
    """The well-balance test of Sec. 4 ([0, 2]^2, cell size 0.05, bump 0.5 exp(-50 r^2) at the
    centre, h1 = 0.8 - B, h2 = 0.2, CFL 0.5, walls) run to its end time t = 100, about 46,000
    steps.  At the paper's density ratio 1 the internal mode has no restoring force and the linear
    scheme lets it grow from round-off; the nonlinear weights hold it near their floor, 1e-9 of the
    level in FP64: under the paper's bound (< 1e-8; measured 1e-9).  The mixed path's floor sits at
    1e-5 of the level, above single-precision rounding (measured 9e-6).  At 0.9 the deviation
    stays at round-off in FP64 (measured 2.6e-13) and at single-precision rounding in the mixed
    path, whose momenta are single precision."""
    import dataclasses

    sc = dataclasses.replace(w.well_balance_bump(40), chi=chi)
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc, precision=precision, t_end=sc.t_end)
    worst, t = 0.0, 0.0
    for k in range(30):
        st.batch_step(2000)
        t, _ = st.time()
        W, gW, _ = st.read()
        assert np.isfinite(W).all() and np.isfinite(gW).all(), t
        dev = max(np.abs(W[3] - sc.W0[3]).max(), np.abs(W[0] - sc.W0[0]).max(), np.abs(W[[1, 2, 4, 5]]).max())
        worst = max(worst, dev)
        if t >= sc.t_end:
            break
    print(f"[paper] well balance chi {chi} {precision}: t {t:.2f}, max deviation {worst:.2e}", flush=True)
    assert t >= sc.t_end
    assert worst < bound, worst
