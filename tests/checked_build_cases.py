"""Cases run by tests/test_gpu_checked_build.py, in a process of their own so that the library
named by GKS_LIBRARY (the checked build, or the ordinary one) is the one loaded.  Writes the final
states of every case to the .npz path given as the first argument and prints the index-check flag
(-1 where the build has no checks)."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import workloads as w  # noqa: E402


def cases():
    return {
        "periodic": (w.smooth_periodic(10), {}),
        "wall_bump": (w.lake_at_rest(12, perturb=1e-2, seed=3), {}),
        "free": (w.free_outflow(10), {}),
        "dam_fp32": (w.dam_break(12, seed=5), {"precision": "fp32"}),
        "src4": (w.smooth_jittered(10), {"src_order": 4}),
        "grad_mode": (w.dam_break(10, seed=6), {"grad_mode": "discontinuous"}),
        "wet_dry": (w.dam_break_dry(16, chi=0.2), {}),
        "wet_dry_breach": (w.dam_break_breach("dry", n=12), {"grad_mode": "discontinuous"}),
    }


def main(out):
    import torch

    import paper_2306_04467_amd as g
    from paper_2306_04467_amd.gks import GksError, debug_bounds

    torch.cuda.set_device(0)
    g.load()
    try:
        debug_bounds(reset=True)
        checked = True
    except GksError:
        checked = False
    res = {}
    for name, (sc, kw) in cases().items():
        st = g.State.from_scenario(g.Mesh.from_scenario(sc), sc, **kw)
        st.step(3)
        W, gW, _ = st.read()
        res[name + "_W"], res[name + "_gW"] = W, gW
        print(f"[checked] {name} done", flush=True)
    scs = [w.lake_at_rest(8, perturb=1e-2, seed=30 + k) for k in range(3)]
    bm = g.Mesh.batch([g.Mesh.from_scenario(s) for s in scs])
    bst = g.State.from_scenarios(bm, scs)
    bst.batch_step(3)
    res["batch_W"] = bst.read()[0]
    np.savez(out, **res)
    print(f"violations {debug_bounds() if checked else -1}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1])
