"""tetmf: matrix-free finite-element operators on uniformly refined
macro-tetrahedra for AMD Instinct MI355X (gfx950).

The compute path is the HIP library libtetmf.so (C ABI in include/tetmf.h);
this package marshals PyTorch device tensors and streams into it.
"""
from ._lib import TetmfError, check, lib  # noqa: F401
from .operators import (Mesh, Operator, P1_LAPLACE, P1_DIVKGRAD, P2_LAPLACE, P2_DIVKGRAD, N1_CURLCURL,  # noqa: F401
                        P2V_EPSILON, F64, F32, BC_NONE, BC_DIRICHLET_ZERO, MAP_AFFINE,
                        MAP_SHELL_RADIAL, KIND_NAMES)
from .batch import Batch, IRSolver, PRECOND_NONE, PRECOND_JACOBI  # noqa: F401,E402
from .autograd import TmfApply  # noqa: F401,E402
