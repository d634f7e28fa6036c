"""Exponential-free open GRAPE on AMD Instinct MI355X (gfx950).

Python front end of libopengrape.so: RK4 propagation of the density matrix
under the Lindblad equation with piecewise-constant controls, the backward
adjoint sweep and the per-slice gradient (Boutin et al., Secs. II-III), all
in hand-written HIP kernels behind a C ABI (include/opengrape.h).
"""
from .api import (  # noqa: F401
    EXPORTS,
    LIB_PATH,
    OgError,
    OpenGrapeCost,
    Problem,
    load_library,
    open_grape_cost,
)
