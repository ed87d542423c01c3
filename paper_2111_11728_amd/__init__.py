"""MI355X-native FETI solvers (TFETI / FETI-DP with k-scaling, full orthogonalisation and
simultaneous search directions) for SIMP linear elasticity, after arXiv 2111.11728.

The compute path is the HIP library libfeti.so (C ABI in include/feti.h); ``feti`` is its
ctypes binding and ``autograd`` wraps compliance and its gradient for torch.
"""
from . import feti  # noqa: F401
from . import autograd  # noqa: F401
