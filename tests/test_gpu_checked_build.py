"""The checked build of the library (GKS_CHECKED: every index the kernels read from a mesh table is
range-checked on the device) on periodic, wall, free, mixed-precision, higher-order-coupling and
batched cases: no index is out of range, and the states equal those of the ordinary build bit for
bit.  The checked build runs in one helper process (tests/checked_build_cases.py) so that it is the
library that process loads; the ordinary build runs the same cases here."""
import os
import subprocess
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def gks():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2306_04467_amd as g

    g.load()
    return g


def test_checked_build_finds_no_index_out_of_range_and_changes_no_result(gks, tmp_path):
    from paper_2306_04467_amd.gks import GksError, debug_bounds

    lib = os.path.join(os.path.dirname(HERE), "paper_2306_04467_amd", "libgks_checked.so")
    assert os.path.exists(lib), "the checked build is missing (run the build first)"
    out = tmp_path / "checked.npz"
    env = dict(os.environ, GKS_LIBRARY=lib)
    print("[checked] running the checked build", flush=True)
    r = subprocess.run([sys.executable, os.path.join(HERE, "checked_build_cases.py"), str(out)], env=env,
                       capture_output=True, text=True, timeout=240)
    print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0
    assert "violations 0" in r.stdout
    chk = np.load(out)
    # the ordinary build: no checks to ask for
    with pytest.raises(GksError) as ei:
        debug_bounds()
    assert ei.value.code == gks.GKS_EUNSUPPORTED
    sys.path.insert(0, HERE)
    import checked_build_cases as cbc

    import workloads as w

    for name, (sc, kw) in cbc.cases().items():
        st = gks.State.from_scenario(gks.Mesh.from_scenario(sc), sc, **kw)
        st.step(3)
        W, gW, _ = st.read()
        assert np.array_equal(W, chk[name + "_W"]), name
        assert np.array_equal(gW, chk[name + "_gW"]), name
    scs = [w.lake_at_rest(8, perturb=1e-2, seed=30 + k) for k in range(3)]
    bm = gks.Mesh.batch([gks.Mesh.from_scenario(s) for s in scs])
    bst = gks.State.from_scenarios(bm, scs)
    bst.batch_step(3)
    assert np.array_equal(bst.read()[0], chk["batch_W"])
