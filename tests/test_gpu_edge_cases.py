"""Edge cases of the HIP path through the C ABI: malformed meshes and call orders are rejected
with status codes, the smallest meshes (a stencil that wraps onto itself, a wall mesh made mostly
of mirror cells) match the FP64 oracle, and the mixed path matches the oracle at full size."""
import numpy as np
import pytest

import oracle as o
import workloads as w
from tests._parity import TOL_FP64, grad_err, state_err

pytestmark = pytest.mark.gpu

GKS_EINVAL, GKS_EMESH = 1, 4


@pytest.fixture(scope="module")
def gks():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2306_04467_amd as g

    g.load()
    return g


def _square():
    xy = np.array([[0, 0], [1, 0], [1, 1], [0, 1], [0.5, 0.5]], dtype=float)
    tri = np.array([[0, 1, 4], [1, 2, 4], [2, 3, 4], [3, 0, 4]], dtype=np.int32)
    return xy, tri


def test_rejects_malformed_meshes(gks):
    xy, tri = _square()
    gks.Mesh(xy, tri)                                   # the well-formed square is accepted
    with pytest.raises(gks.GksError) as ei:
        gks.Mesh(xy, tri[:0])                           # no triangles
    assert ei.value.code == GKS_EINVAL
    bad = tri.copy()
    bad[1, 2] = 7                                       # node index out of range
    with pytest.raises(gks.GksError) as ei:
        gks.Mesh(xy, bad)
    assert ei.value.code == GKS_EMESH
    with pytest.raises(gks.GksError) as ei:
        gks.Mesh(xy, tri[:, ::-1].copy())               # clockwise triangles
    assert ei.value.code == GKS_EMESH
    fan = np.concatenate([tri, [[0, 1, 2]]]).astype(np.int32)  # overlaps: edge 0-1 twice in one direction
    with pytest.raises(gks.GksError) as ei:
        gks.Mesh(xy, fan)
    assert ei.value.code == GKS_EMESH
    flat = xy.copy()
    flat[4] = [0.5, 0.0]                                # degenerate (zero-area) triangle
    with pytest.raises(gks.GksError) as ei:
        gks.Mesh(flat, tri)
    assert ei.value.code == GKS_EMESH


def test_rejects_wrong_call_order(gks):
    scs = [w.lake_at_rest(4, seed=41, perturb=1e-2), w.lake_at_rest(5, seed=42, perturb=1e-2)]
    m = gks.Mesh.from_scenario(scs[0])
    st = gks.State.from_scenario(m, scs[0])
    with pytest.raises(gks.GksError):
        st.stage(1)                                     # stage 1 before stage 0
    st.stage(0)
    with pytest.raises(gks.GksError):
        st.stage(0)                                     # stage 0 twice
    with pytest.raises(gks.GksError):
        st.step(1)                                      # a step between the stages
    with pytest.raises(gks.GksError):
        st.autotune(1)
    st.stage(1)
    bm = gks.Mesh.batch([gks.Mesh.from_scenario(sc) for sc in scs])
    bs = gks.State.from_scenarios(bm, scs)
    with pytest.raises(gks.GksError):
        bs.stage(0, 1e-3)                               # an explicit dt needs a single scenario
    with pytest.raises(gks.GksError):
        bs.buffer("skip")                               # the indicator was never switched on


def test_periodic_mesh_too_small_to_pair_its_edges(gks):
    """On a 2 x 2 periodic lattice an edge and its periodic image coincide, so one edge would join
    four triangles: both the oracle and the library reject the mesh."""
    sc = w.smooth_periodic(2)
    with pytest.raises(ValueError):
        o.Mesh.from_scenario(sc)
    with pytest.raises(gks.GksError) as ei:
        gks.Mesh.from_scenario(sc)
    assert ei.value.code == GKS_EMESH


TINY = {
    "periodic_n3": lambda: w.smooth_periodic(3),       # 18 triangles: stencils wrap onto themselves
    "wall_n2": lambda: w.lake_at_rest(2, perturb=1e-2, seed=5),   # every cell touches a wall
    "wall_n3_dam": lambda: w.dam_break(3, bump_amp=0.2),
}


@pytest.mark.parametrize("case", list(TINY))
def test_tiny_meshes_match_oracle(gks, case):
    sc = TINY[case]()
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc)
    om = o.Mesh.from_scenario(sc)
    p = o.params_of(sc)
    W, gW = sc.W0.copy(), sc.gradW0.copy()
    for n in range(4):
        dt = o.dt(om, p, W)
        st.stage(0, dt)
        st.stage(1)
        W, gW = o.step(om, p, dt, W, gW)
    Wg, gWg, _ = st.read()
    e, g = state_err(Wg, W), grad_err(gWg, gW, W)
    assert e.max() < 4 * TOL_FP64 and g.max() < 4 * TOL_FP64, (case, e, g)


def test_mixed_precision_full_size_step(gks):
    """The benchmarked workload at full size in the mixed path: one step against the oracle, at the
    relative L1 bound of the mixed path."""
    sc = w.lake_at_rest(510, seed=20230604, perturb=1e-3, disk=(0.3, 0.3, 0.1))
    print(f"[edge] full size fp32 T={sc.n_tri}", flush=True)
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc, precision="fp32")
    om = o.Mesh.from_scenario(sc)
    p = o.params_of(sc)
    dt = o.dt(om, p, sc.W0)
    st.stage(0, dt)
    st.stage(1)
    W, _, _ = st.read()
    Wr, _ = o.step(om, p, dt, sc.W0, sc.gradW0)
    a, _, _ = om.geometry()
    err = []
    for q in (0, 3):
        h = Wr[q]
        err.append((a * np.abs(W[q] - h)).sum() / (a * np.abs(h)).sum())
        den = (a * h * np.sqrt(9.81 * h)).sum()
        for v in (q + 1, q + 2):
            err.append((a * np.abs(W[v] - Wr[v])).sum() / den)
    print(f"   rel-L1 {max(err):.2e}", flush=True)
    assert max(err) <= 1e-5, err


def test_explicit_step_past_t_end_is_clipped(gks):
    """An explicit stage-0 step that would pass t_end is clipped to it, and later CFL steps are
    empty (step size 0, state unchanged), never negative."""
    sc = w.lake_at_rest(8, perturb=1e-2, seed=4)
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc, t_end=0.01)
    st.stage(0, 0.004)
    st.stage(1)
    st.stage(0, 0.05)             # 0.004 + 0.05 passes t_end = 0.01
    st.stage(1)
    t, dt = st.time()
    assert t == 0.01 and abs(dt - 0.006) < 1e-15, (t, dt)
    W1, gW1, _ = st.read()
    assert st.step(3, want_dt=True) == 0.0
    st.stage(0, 0.02)
    st.stage(1)
    W2, gW2, t2 = st.read()
    assert t2 == 0.01 and np.array_equal(W1, W2) and np.array_equal(gW1, gW2)
