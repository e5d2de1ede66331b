// Declarations of the batch solver's vector kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tmf {

constexpr int kBlasThreads = 256;
constexpr int kChunkLen = 8192;  // vector entries per reduction chunk

struct ChunkDesc {
  int64_t start;  // first entry in the concatenated vector
  int len;
  int inst;
};

// per-instance CG state (device arrays of `count` entries)
struct CgScalars {
  double *rnorm, *bnorm, *rr, *rr0, *alpha, *beta;
  int *it;
  uint8_t *oact, *iact;  // outer / inner activity
};

struct BlasCtx {
  const ChunkDesc *chunks;
  int nchunks;
  const int *first;      // count + 1 chunk offsets per instance
  int count;
  const uint8_t *owner;  // NULL when every slot is the only copy of its DoF
  const float *dinv;     // Jacobi preconditioner 1 / diag(A) (0 on Dirichlet rows), or NULL for none
  CgScalars sc;
};

hipError_t blas_residual(const BlasCtx &c, const double *b, const double *Ax, double *r, double *prr, double *pbb,
                         double tol, hipStream_t s);
hipError_t blas_start_inner(const BlasCtx &c, const double *r64, float *r32, float *p, float *d, double *part,
                            hipStream_t s);
hipError_t blas_cg_step_after_apply(const BlasCtx &c, float *d, float *r, float *p, const float *q, double *part,
                                    double rtol2, int maxit, hipStream_t s);
hipError_t blas_update_x(const BlasCtx &c, double *x, const float *d, hipStream_t s);
// dinv = 1 / d where d > 0, else 0 (FP64 diagonal in, FP32 out)
hipError_t blas_inverse_diagonal(const BlasCtx &c, const double *d, float *dinv, hipStream_t s);

}  // namespace tmf
