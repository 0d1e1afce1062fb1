"""Seeded synthetic inputs shared by the HIP path, its tests, the bench and the oracle's tests.

This package builds triangular meshes and initial cell data for the two-layer shallow water
problems (meshes, bottom topography at nodes, cell averages and cell-averaged gradients of the
initial state).  It holds none of the scheme's arithmetic: no reconstruction, flux, source or
time-stepping code lives here, only geometry generation and quadrature of analytic initial data.
"""
from .meshes import periodic_square, jittered_square, jittered_rect  # noqa: F401
from .scenarios import (  # noqa: F401
    Scenario,
    smooth_periodic,
    accuracy_e1,
    accuracy_e1_free,
    uniform_stream,
    free_outflow,
    smooth_jittered,
    lake_at_rest,
    well_balance_bump,
    dam_break,
    ensemble,
    riemann_exchange,
    riemann_interface,
    circular_interface,
    dam_break_dry,
    ritter_channel,
    dam_break_breach,
    dry_bump_dam_break,
    COMPONENTS,
)
from .configs import CONFIGS, build as build_config, spec as config_spec  # noqa: F401,E402
