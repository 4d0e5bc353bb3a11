"""MI355X (gfx950) Eikonal travel-time solver: asynchronous soft-priority
marching with an exactly monotone update operator, its adjoint, and batched
multi-shot solves.  The compute path is the HIP library libeik.so (C ABI in
include/eik.h); this package is its thin Python binding.
"""
from ._lib import EikError  # noqa: F401
from .api import (  # noqa: F401
    Batch, EikonalFn, adjoint, adjoint_packed, eikonal, make_opts, num_tiles, pack, parents_of,
    release, reserve, residual, solve, solve_batched, solve_packed, solve_rect, source_indices, status, timeline,
)

__all__ = [
    "EikError", "Batch", "EikonalFn", "adjoint", "adjoint_packed", "eikonal", "make_opts",
    "num_tiles", "pack", "parents_of", "release", "reserve", "residual", "solve", "solve_batched",
    "solve_packed", "solve_rect", "source_indices", "status", "timeline",
]
