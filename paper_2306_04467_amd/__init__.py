"""MI355X (gfx950) implementation of the compact gas-kinetic scheme for the two-layer shallow
water equations on triangular meshes: HIP kernels behind a C ABI (include/gks.h) and a thin
Python binding."""
from .gks import (GKS_EINVAL, GKS_ENONFINITE, GKS_EUNSUPPORTED, GKS_OK, GksError, Mesh, State,  # noqa: F401
                  Trainer, debug_bounds, load, make_params)
