"""The benchmark configurations C1-C5 as named scenario specifications.

Each entry names the generator of `workloads.scenarios` and its arguments, so that the benchmark,
the tests and a user build the same inputs from one table; `spec()` gives the table as plain data
(JSON-ready) and `build()` makes the scenario (a list of scenarios for the ensemble).
"""
from __future__ import annotations

import copy

from . import scenarios as _sc

CONFIGS = {
    "C1": {"generator": "smooth_periodic", "args": {"n": 20},
           "what": "periodic [0,2]^2, 800 right triangles, smooth two-layer plane waves, chi 0.98, CFL 0.3"},
    "C2": {"generator": "lake_at_rest",
           "args": {"n": 510, "seed": 20230604, "perturb": 1e-3, "disk": [0.3, 0.3, 0.1]},
           "what": "520,200-triangle jittered Delaunay [0,1]^2, bump 0.5 exp(-50 r^2), lake at rest "
                   "eta1 = 0.8, h2 = 0.2 with a 1e-3 interface perturbation in a disk, walls, chi 0.98"},
    "C3": {"generator": "dam_break", "args": {"n": 707, "seed": 20230605},
           "what": "999,698-triangle two-layer dam break over a sinusoidal bottom, chi 0.95, walls"},
    "C4": {"generator": "ensemble", "args": {"n_scen": 256, "seed": 20230606},
           "what": "256 lake-at-rest scenarios of 5k-200k triangles (log-uniform), 13.65 M in all"},
    "C5": {"generator": "dam_break", "args": {"n": 1000, "seed": 20230608, "sin_amp": 0.1, "bump_amp": 0.2},
           "what": "2,000,000-triangle dam break over a bump (the learned indicator's gain case)"},
}


def spec(name: str) -> dict:
    """The configuration as plain data: generator name, arguments, description."""
    return copy.deepcopy(CONFIGS[name])


def build(name: str, **overrides):
    """Build configuration `name` (arguments may be overridden, e.g. a smaller n for a test)."""
    c = CONFIGS[name]
    args = dict(c["args"], **overrides)
    if "disk" in args and isinstance(args["disk"], list):
        args["disk"] = tuple(args["disk"])
    return getattr(_sc, c["generator"])(**args)
