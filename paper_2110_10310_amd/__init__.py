"""MI355X-native hot path of open-system optimal control (Lindblad master
equation, implicit midpoint rule, discrete adjoint) behind the C ABI of
liblbx.so.  See include/lbx.h for the ABI; ``api`` holds the Python binding.
"""
from . import _native  # noqa: F401  (raises ImportError when liblbx.so is missing)
from .api import (  # noqa: F401
    Plan,
    control_table,
    sweep_counts,
    lindblad_apply,
    imr_step,
    imr_step_noalloc,
    forward_solve,
    objective,
    adjoint_gradient,
    adjoint_backward,
    LindbladObjective,
    lindblad_objective,
)
from .optim import optimize  # noqa: F401
