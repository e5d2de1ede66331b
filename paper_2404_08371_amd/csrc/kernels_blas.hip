// Vector kernels for the Krylov solvers (filled in with the solver).
#include "tmf_internal.h"
