"""MI355X (gfx950) implementation of the compact gas-kinetic scheme for the two-layer shallow
water equations on triangular meshes: HIP kernels behind a C ABI (include/gks.h) and a thin
Python binding."""
from .gks import GksError, Mesh, State, Trainer, load  # noqa: F401
