"""MI355X-native N-shaped partition Crank-Nicolson solver (arXiv 2205.00856).

The solver itself is the HIP library libcntri.so (C ABI in include/cntri.h); this package
binds it for torch device tensors and adds autograd wrappers.
"""
from .api import (Handle, Layout, assemble, radial_step, autotune, describe_plan, get_status, handle,  # noqa: F401
                  profile, profile_report, propagate, propagate_adjoint, propagate_adjoint_reconstruct,
                  propagate_resident,
                  reserve, rhs, solve, solve_adjoint,
                  solve_noalloc, step, tune_cache,
                  step_adjoint)

__version__ = "0.1.0"
