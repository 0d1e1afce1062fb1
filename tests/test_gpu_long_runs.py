"""Long runs of the headline workload on the GPU: the 520,200-triangle lake at rest with its 1e-3
interface perturbation in a disk (walls, bump, density ratio 0.98) for 3000 steps (t = 0.13), in
both precisions.  The run must stay finite with its layer masses conserved to round-off, and the
disk's waves must keep their size (the largest momentum stays within a factor 2 of its value after
250 steps)."""
import numpy as np
import pytest

import workloads as w

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gks():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2306_04467_amd as g

    g.load()
    return g


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_perturbed_headline_workload_3000_steps(gks, precision):
    sc = w.lake_at_rest(510, perturb=1e-3)
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc, precision=precision)
    m0 = st.mass()
    first = None
    for k in range(12):
        st.batch_step(250)
        W, gW, t = st.read()
        assert np.isfinite(W).all() and np.isfinite(gW).all(), (precision, 250 * (k + 1))
        peak = np.abs(W[[1, 2, 4, 5]]).max()
        first = peak if first is None else first
        dm = (np.abs(st.mass() - m0) / m0).max()
        print(f"[long] {precision} step {250 * (k + 1)} t {t:.4f} max|hU| {peak:.3e} mass drift {dm:.1e}",
              flush=True)
        assert dm < 1e-13, dm
        assert 0.5 * first < peak < 2 * first, (peak, first)
