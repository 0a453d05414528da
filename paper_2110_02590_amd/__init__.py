"""MI355X-native reduced-space power-flow derivatives (FP64, HIP/gfx950).

Python face of the C ABI declared in include/rpf.h: power flow, AL value,
reduced gradient, batched reduced Hessian-vector products, dense reduced
Hessian and Cholesky step.  All computation runs in librpf.so.
"""
from .binding import Grid, RpfError, lib, presolve_info, presolve_pattern  # noqa: F401
from .problem import Problem  # noqa: F401
