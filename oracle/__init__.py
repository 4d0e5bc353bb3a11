"""CPU oracle for the Eikonal solve and its adjoint.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product path (the HIP library and
its Python binding) never imports this package, and this package never imports
the product path.
"""
from .oracle import *  # noqa: F401,F403
