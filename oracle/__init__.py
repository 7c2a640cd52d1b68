"""FP64 CPU oracle of the damped-gradient Skyrme iteration.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything under this package; only the tests, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP library.

Every function here is written plainly from the paper (Afibuzzaman,
Schuetrumpf, Aktulga, "Scalable Nuclear Density Functional Theory with
Sky3D"), in FP64, with numpy/scipy FFTs and dense linear algebra as the only
library steps.  Where the paper is schematic the reading used is stated in
the docstring of the function that takes it.
"""
from .grid import Grid  # noqa: F401
from . import grid, physics, precond, solver  # noqa: F401
