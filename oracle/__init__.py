"""CPU FP64 oracle for the finite-array MoM solver.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the benchmark's
CPU-baseline leg, never by the GPU product path.  See mom.py for what it
computes and gmres.py for the reference iterative solver.
"""
from . import mom, gmres  # noqa: F401
