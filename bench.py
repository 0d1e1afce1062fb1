#!/usr/bin/env python
"""Throughput of the two-layer compact GKS on one MI355X: triangle-stage updates per second.

One step = the whole hot path once: device CFL time step, then the two S2O4 stages, each running
ghost refresh, reconstruction, force-model heights and planes, gas-kinetic flux at every Gauss
point and the gather/source/update kernel.  Inputs are resident on the GPU before timing starts.

Default workload: FP64 plain path on the 520,200-triangle jittered Delaunay mesh of [0,1]^2 with a
Gaussian bottom bump, lake at rest plus a 1e-3 interface perturbation in a disk, reflecting walls.

Prints ONE JSON line (see the design doc for the fields).  Kernel durations for the roofline come from
HIP events recorded by the library around each launch on its stream; the CPU baseline times the
FP64 oracle on the host for one full step of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "triangle-stage updates/s, FP64 plain vs FP32+learned-indicator, at rel-L1 err"
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes_fp64(T, E, NG):
    """Bytes each kernel must move per launch if every input is read once and every output
    written once (neighbour re-reads served by caches).  FP64 words, int32 indices."""
    return {
        "recon": T * (8 * (6 + 12 + 153 + 6 + 1 + 6) + 4 * 9 + 8 * (108 + 2)),
        "flux": T * 8 * (108 + 2 + 4) + E * (4 * 3 + 8 * 6 + 8 * 24),
        "hhat": T * 8 * 36 + E * (4 * 3 + 8 * 4 + 8 * 2),
        "plane": T * (4 * 3 + 8 * 6 + 8 * 4) + E * 8 * 2,
        "update": T * (4 * 3 + 8 * 12) + E * 8 * 24 + T * 8 * 36,  # stage average of 6+36 / 36+18 words
        "ghost": NG * (8 * 36 + 8 * 4 + 4),
        "dt": T * 8 * 4,
    }


def rel_l1(W, Wr, area, G):
    import numpy as np

    out = []
    for o in (0, 3):
        h = Wr[o]
        out.append((area * np.abs(W[o] - h)).sum() / (area * np.abs(h)).sum())
        den = (area * h * np.sqrt(G * h)).sum()
        for v in (o + 1, o + 2):
            out.append((area * np.abs(W[v] - Wr[v])).sum() / den)
    return max(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=510, help="lattice size: 2 n^2 triangles")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip the event-timed pass")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 5 times (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch

        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": x.numel() * 8, "copy_bytes_written_per_launch": x.numel() * 8}))
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU decomposition is described in DESIGN.md but not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads
    from paper_2306_04467_amd import Mesh, State

    torch.cuda.set_device(0)
    t0 = time.time()
    sc = workloads.lake_at_rest(args.n, seed=20230604, perturb=1e-3, disk=(0.3, 0.3, 0.1))
    print(f"[bench] workload built: {sc.n_tri} triangles ({time.time() - t0:.1f}s)", file=sys.stderr, flush=True)
    t0 = time.time()
    mesh = Mesh.from_scenario(sc)
    print(f"[bench] mesh setup: {mesh.n_edges} edges, {mesh.n_ghost} ghosts ({time.time() - t0:.1f}s)",
          file=sys.stderr, flush=True)
    st = State.from_scenario(mesh, sc)
    stream = torch.cuda.current_stream()

    st.step(args.warmup)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_wall = time.time()
    ev0.record(stream)
    st.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_wall = time.time() - t_wall
    ms = ev0.elapsed_time(ev1)
    ms_per_step = ms / args.steps
    T, E, NG = mesh.n_tri, mesh.n_edges, mesh.n_ghost
    value = T * 2 * args.steps / (ms / 1e3)
    print(f"[bench] {args.steps} steps: {ms:.2f} ms (wall {t_wall * 1e3:.1f} ms), {value / 1e9:.3f} G tri-stage/s",
          file=sys.stderr, flush=True)

    # per-kernel durations from HIP events on the library's stream, same steps again
    roofline, kernels = None, {}
    if not args.no_profile:
        st.profile(True)
        st.step(args.steps)
        prof = st.profile_read()
        st.profile(False)
        alg = algorithmic_bytes_fp64(T, E, NG)
        for k, (tot, n) in prof.items():
            if n:
                avg = tot / n
                kernels[k] = {"avg_ms": round(avg, 5), "launches": n,
                              "alg_GBs": round(alg[k] / (avg / 1e3) / 1e9, 1)}
        dom = max(kernels, key=lambda k: kernels[k]["avg_ms"] * kernels[k]["launches"])
        avg = kernels[dom]["avg_ms"]
        achieved = alg[dom] / (avg / 1e3) / 1e9
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                    "alg_bytes_per_launch": alg[dom]}
        print(f"[bench] kernels: {json.dumps(kernels)}", file=sys.stderr, flush=True)

    cpu = None
    err = None
    if not args.no_cpu_baseline:
        import oracle

        W1 = State.from_scenario(mesh, sc)
        om = oracle.Mesh.from_scenario(sc)
        p = oracle.params_of(sc)
        dt = oracle.dt(om, p, sc.W0)
        tc = time.time()
        Wr, _ = oracle.step(om, p, dt, sc.W0, sc.gradW0)
        tc = time.time() - tc
        W1.stage(0, dt)
        W1.stage(1)
        Wg, _, _ = W1.read()
        area = sc_area(sc)
        err = rel_l1(Wg, Wr, area, sc.G)
        cpu = {"value": round(T * 2 / tc, 1), "unit": "triangle-stage/s", "cores": 1, "kind": "oracle",
               "sample": f"one full S2O4 step (2 stages) of the same {T}-triangle workload, single-threaded "
                         f"FP64 C oracle, {tc:.1f} s"}
        print(f"[bench] oracle step {tc:.1f}s, rel-L1 GPU vs oracle {err:.3e}", file=sys.stderr, flush=True)

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "triangle-stage/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"fp64 plain: jittered-node Delaunay [0,1]^2, {T} triangles, Gaussian bottom "
                               f"bump 0.5exp(-50r^2), lake at rest eta1=0.8 h2=0.2 + 1e-3 interface "
                               f"perturbation in a disk, walls, chi=0.98, CFL 0.3",
                   "n_tri": T, "n_edges": E, "precision": "fp64", "rel_l1_vs_oracle_1step": err},
        "roofline": roofline, "cpu_baseline": cpu, "kernels": kernels,
    }
    print(json.dumps(line), flush=True)


def sc_area(sc):
    import numpy as np

    a, b, c = (sc.node_xy[sc.tri[:, k]] for k in range(3))
    return 0.5 * ((b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0]))


if __name__ == "__main__":
    main()
