"""Free (zero-gradient) boundaries on the GPU against the oracle: a smooth hump flowing out of a
jittered box over a bump (one step at the FP64 bound, then five steps), the uniform stream kept to
round-off, and a batch that mixes a free-boundary scenario with a walled one."""
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


@pytest.mark.parametrize("nsteps", [1, 5])
def test_free_outflow_matches_oracle(gks, nsteps):
    sc = w.free_outflow(24)
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc)
    om = o.Mesh.from_scenario(sc)
    p = o.params_of(sc)
    Wr, gWr = sc.W0, sc.gradW0
    for _ in range(nsteps):
        dt = st.step(1, want_dt=True)
        Wr, gWr = o.step(om, p, dt, Wr, gWr)
    W, gW, _ = st.read()
    e, g = state_err(W, Wr).max(), grad_err(gW, gWr, Wr).max()
    print(f"[free] outflow {nsteps} steps: state {e:.2e} grad {g:.2e}", flush=True)
    assert e < nsteps * TOL_FP64 and g < nsteps * TOL_FP64 * 10


def test_uniform_stream_kept(gks):
    for precision, tol in (("fp64", 1e-14), ("fp32", 1e-6)):
        sc = w.uniform_stream(16)
        st = gks.State.from_scenario(gks.Mesh.from_scenario(sc), sc, precision=precision)
        st.step(20)
        W, _, _ = st.read()
        assert np.abs(W - sc.W0).max() < tol, (precision, np.abs(W - sc.W0).max())


def test_batch_mixes_free_and_wall_scenarios(gks):
    scs = [w.free_outflow(12), w.lake_at_rest(10, perturb=1e-2, seed=4)]
    meshes = [gks.Mesh.from_scenario(s) for s in scs]
    bm = gks.Mesh.batch(meshes)
    st = gks.State.from_scenarios(bm, scs)
    st.batch_step(3)
    W, gW, _ = st.read()
    for k, sc in enumerate(scs):
        a, n = bm.scenario_range(k)
        single = gks.State.from_scenario(meshes[k], sc)
        single.step(3)
        Ws, gWs, _ = single.read()
        assert np.array_equal(W[:, a:a + n], Ws) and np.array_equal(gW[:, :, a:a + n], gWs), k
