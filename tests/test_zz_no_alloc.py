"""The allocation-free mass query against the ordinary one, through the C ABI: two calls in a
row on the same device, the second on a smaller state, for all cells and for one scenario of a
batch.  Same kernel and block grid, so the sums agree bit for bit."""
import ctypes

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


def _both(gks, st, scen):
    lib = gks.load()
    a, b = np.zeros(2), np.zeros(2)
    assert lib.gks_state_mass(st._h, int(scen), a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == 0
    assert lib.gks_state_mass_noalloc(st._h, int(scen), b.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == 0
    return a, b


def test_noalloc_mass_matches_the_allocating_query(gks):
    big = w.lake_at_rest(64, perturb=1e-2, seed=5)       # 8192 triangles
    small = w.lake_at_rest(12, perturb=1e-2, seed=6)     # 288 triangles
    for sc in (big, small):
        m = gks.Mesh.from_scenario(sc)
        st = gks.State.from_scenario(m, sc)
        st.step(3)
        a, b = _both(gks, st, -1)
        print(f"[noalloc] {sc.n_tri} triangles: {a} vs {b}", flush=True)
        assert np.array_equal(a, b), (a, b)
        assert np.all(a > 0)


def test_noalloc_mass_of_one_scenario_of_a_batch(gks):
    scs = [w.lake_at_rest(20, perturb=1e-3, seed=7), w.lake_at_rest(9, perturb=1e-3, seed=8)]
    meshes = [gks.Mesh.from_scenario(s) for s in scs]
    bm = gks.Mesh.batch(meshes)
    st = gks.State.from_scenarios(bm, scs)
    st.batch_step(2)
    for scen in (0, 1, -1):
        a, b = _both(gks, st, scen)
        assert np.array_equal(a, b), (scen, a, b)
    lib = gks.load()
    out = np.zeros(2)
    assert lib.gks_state_mass_noalloc(st._h, 2, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) != 0
