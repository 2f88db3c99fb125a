"""MI355X-native adaptive spectral deferred correction for monodomain models.

The compute path is the HIP library ``libsdc.so`` (C ABI in include/sdc.h),
built in-tree by :func:`build.build`; :class:`Solver` is its thin binding.
"""
from .solver import SDCError, Solver, collocation, select_noalloc  # noqa: F401
