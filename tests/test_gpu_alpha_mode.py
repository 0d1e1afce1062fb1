"""The paper's printed constants alpha_{k,m} (Sec. 2.2) as the alternative mode of the library:
GPU against the oracle in the same mode, one and three steps at the FP64 bound, on the perturbed
lake at rest over a bump and on a dam break; and the lake at rest kept."""
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


@pytest.mark.parametrize("case", ["lake", "dam"])
@pytest.mark.parametrize("nsteps", [1, 3])
def test_paper_alpha_mode_matches_oracle(gks, case, nsteps):
    sc = w.lake_at_rest(24, perturb=1e-2, seed=41) if case == "lake" else w.dam_break(20, seed=42)
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc, alpha_mode="paper")
    om = o.Mesh.from_scenario(sc)
    p = o.params_of(sc, alpha_mode="paper")
    Wr, gWr = sc.W0, sc.gradW0
    for _ in range(nsteps):
        dt = st.step(1, want_dt=True)
        Wr, gWr = o.step(om, p, dt, Wr, gWr)
    W, gW, _ = st.read()
    e, g = state_err(W, Wr).max(), grad_err(gW, gWr, Wr).max()
    print(f"[alpha] paper mode {case} {nsteps} steps: state {e:.2e} grad {g:.2e}", flush=True)
    assert e < nsteps * TOL_FP64 and g < nsteps * TOL_FP64 * 10
    # the modes differ on these flows
    ref = gks.State.from_scenario(m, sc)
    ref.step(nsteps)
    assert not np.array_equal(ref.read()[0], W)


def test_paper_alpha_mode_lake_at_rest(gks):
    sc = w.lake_at_rest(32, seed=43)
    st = gks.State.from_scenario(gks.Mesh.from_scenario(sc), sc, alpha_mode="paper")
    st.step(200)
    W, _, _ = st.read()
    assert np.abs(W[[1, 2, 4, 5]]).max() < 1e-12 and np.abs(W[[0, 3]] - sc.W0[[0, 3]]).max() < 1e-12


def test_paper_alpha_mode_mixed_precision(gks):
    """The paper's constants in the mixed FP32/FP64 path: three steps of a dam break within the mixed
    path's relative L1 bound of the FP64 oracle in the same mode."""
    sc = w.dam_break(20, seed=44)
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc, precision="fp32", alpha_mode="paper")
    om = o.Mesh.from_scenario(sc)
    p = o.params_of(sc, alpha_mode="paper")
    a, _, _ = om.geometry()
    Wr, gWr = sc.W0, sc.gradW0
    for _ in range(3):
        dt = o.dt(om, p, Wr)
        st.stage(0, dt)
        st.stage(1)
        Wr, gWr = o.step(om, p, dt, Wr, gWr)
    W, _, _ = st.read()
    err = []
    for q in (0, 3):
        h = Wr[q]
        err.append((a * np.abs(W[q] - h)).sum() / (a * np.abs(h)).sum())
        den = (a * h * np.sqrt(sc.G * h)).sum()
        for v in (q + 1, q + 2):
            err.append((a * np.abs(W[v] - Wr[v])).sum() / den)
    print(f"[alpha] paper mode fp32 3 steps: rel-L1 {max(err):.2e}", flush=True)
    assert max(err) <= 1e-5, err
