"""Independent FP64 CPU oracle for the matrix-free tetrahedral operators.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package; the product library
(paper_2404_08371_amd) never imports it and shares no code with it.

Modules: lattice (refinement, layout, keys), elements (element matrices from
their definitions), apply (matrix-free y = A x, sparse assembly, gradients,
conjugate gradients).
"""
from .apply import (Problem, P1_LAPLACE, P1_DIVKGRAD, P2_LAPLACE, P2_DIVKGRAD, P2V_EPSILON, N1_CURLCURL,  # noqa: F401
                    BC_NONE, BC_DIRICHLET_ZERO, MAP_AFFINE, MAP_SHELL_RADIAL)
