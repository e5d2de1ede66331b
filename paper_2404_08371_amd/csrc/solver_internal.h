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

// per-instance CG state (device arrays of `count` entries; rr holds two
// slots of `count`, used alternately by consecutive inner iterations)
struct CgScalars {
  double *rnorm, *bnorm, *rr, *rr0, *alpha, *beta;
  int *it;
  uint8_t *oact, *iact;  // outer / inner activity
  int count;
};

struct BlasCtx {
  const ChunkDesc *chunks;
  int nchunks;
  const int *first;      // count + 1 chunk offsets per instance
  int count;
  const uint8_t *owner;  // NULL when every slot is the only copy of its DoF
  const void *dinv;      // Jacobi preconditioner 1 / diag(A) (0 on Dirichlet rows) in the inner type, or NULL
  CgScalars sc;
};

hipError_t blas_residual(const BlasCtx &c, const double *b, const double *Ax, double *r, double *prr, double *pbb,
                         double tol, hipStream_t s);
// V = float (FP32 inner iteration) or double (FP64 inner iteration)
template <typename V>
hipError_t blas_start_inner(const BlasCtx &c, const double *r64, V *r, V *p, V *d, double *part, hipStream_t s);
// the inner iteration after q = A p: p.q, alpha and the update, beta and the
// new direction; ppq and prz hold the per-chunk partials, par the slot parity
template <typename V>
hipError_t blas_cg_step_after_apply(const BlasCtx &c, V *d, V *r, V *p, const V *q, double *ppq, double *prz,
                                    double rtol2, int maxit, int par, hipStream_t s);
template <typename V>
hipError_t blas_update_x(const BlasCtx &c, double *x, const V *d, hipStream_t s);
// dinv = 1 / d where d > 0, else 0 (FP64 diagonal in)
template <typename V>
hipError_t blas_inverse_diagonal(const BlasCtx &c, const double *d, V *dinv, hipStream_t s);

}  // namespace tmf
