"""Seeded synthetic inputs shared by the oracle and the library's tests and benchmark.

This package produces input arrays only (meshes, coefficient fields,
stimulus node lists, initial states, solver settings).  It holds none of the
method's arithmetic and imports neither the oracle nor the library.
"""
from .configs import Problem, make, config0, config1, config2, config4, AP_PARAMS  # noqa: F401
from .emi import EmiProblem, config3, config5, emi_mesh, emi_mesh3d  # noqa: F401
