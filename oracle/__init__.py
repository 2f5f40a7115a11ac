"""CPU oracle (test infrastructure only): plain FP64 NumPy implementation of the discrete
acoustic forward operator, its adjoint, the Born operator and the adjoint-state gradient.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark import it; the
HIP library and its Python binding never do.
"""
from .awe_oracle import *  # noqa: F401,F403
from .awe_oracle import __all__  # noqa: F401
