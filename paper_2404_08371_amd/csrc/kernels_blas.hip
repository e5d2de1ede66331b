// Vector kernels of the batched Krylov solver.
//
// A batch concatenates the vectors of its instances; every kernel walks a
// fixed list of chunks (instance, start, length), one workgroup per chunk,
// so per-instance reductions are two-pass and deterministic: each chunk
// writes one FP64 partial (fixed tree order inside the workgroup), and a
// second pass adds an instance's partials in chunk order.  CG scalars live
// per instance in device memory; an instance whose inner iteration has
// converged keeps its vectors unchanged (alpha = 0 and p frozen), and its q
// is never read (the solver's applies skip inactive instances).
//
// With a Jacobi preconditioner (dinv = 1 / diag(A), 0 on Dirichlet rows) the
// inner iteration is preconditioned CG: z = dinv r is formed on the fly where
// it is used, rr holds r.z, and the inner stopping test compares r.z with its
// initial value.
#include "solver_internal.h"

namespace tmf {

namespace {

__device__ inline double block_sum(double v, double *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
#pragma unroll
  for (int s = kBlasThreads / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  return sh[0];
}

template <typename TA, typename TB>
__global__ __launch_bounds__(kBlasThreads) void k_dot_partial(const TA *a, const TB *b, const uint8_t *owner,
                                                               const ChunkDesc *ch, double *partial) {
  __shared__ double sh[kBlasThreads];
  const ChunkDesc c = ch[blockIdx.x];
  double s = 0;
  for (int i = threadIdx.x; i < c.len; i += kBlasThreads) {
    const int64_t g = c.start + i;
    const double v = double(a[g]) * double(b[g]);
    s += (owner == nullptr || owner[g]) ? v : 0.0;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Sum of the partials of instance i, by one wavefront: lane l adds partials
// first[i] + l, + 64, ... in order, then a fixed xor butterfly.  Every lane
// ends with the same bits (a + b == b + a exactly), and the order depends only
// on the chunk list, so the result is reproducible run to run.
__device__ inline double inst_sum(const double *partial, const int *first, int i) {
  const int lane = threadIdx.x & 63;
  double s = 0;
  for (int q = first[i] + lane; q < first[i + 1]; q += 64) s += partial[q];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  return s;
}

// r64 = b - Ax, partials of r.r and b.b
__global__ __launch_bounds__(kBlasThreads) void k_residual(const double *b, const double *Ax, double *r,
                                                            const uint8_t *owner, const ChunkDesc *ch,
                                                            double *prr, double *pbb) {
  __shared__ double sh[kBlasThreads];
  const ChunkDesc c = ch[blockIdx.x];
  double srr = 0, sbb = 0;
  for (int i = threadIdx.x; i < c.len; i += kBlasThreads) {
    const int64_t g = c.start + i;
    const double rv = b[g] - Ax[g];
    r[g] = rv;
    if (owner == nullptr || owner[g]) {
      srr += rv * rv;
      sbb += b[g] * b[g];
    }
  }
  srr = block_sum(srr, sh);
  if (threadIdx.x == 0) prr[blockIdx.x] = srr;
  __syncthreads();
  sbb = block_sum(sbb, sh);
  if (threadIdx.x == 0) pbb[blockIdx.x] = sbb;
}

// per instance: |r|, |b|, outer activity (|r| > tol |b|)
__global__ void k_outer_norms(const double *prr, const double *pbb, const int *first, int count, double tol,
                              CgScalars s) {
  const int i = blockIdx.x;
  if (i >= count) return;
  const double rn = sqrt(inst_sum(prr, first, i)), bn = sqrt(inst_sum(pbb, first, i));
  if (threadIdx.x != 0) return;
  s.rnorm[i] = rn;
  s.bnorm[i] = bn;
  s.oact[i] = (rn > tol * bn) ? 1 : 0;
}

// r32 = r64 / |r| for active instances (0 otherwise), p = z = dinv r32, d = 0;
// partial r32.z
__global__ __launch_bounds__(kBlasThreads) void k_scale_cast(const double *r64, float *r32, float *p, float *d,
                                                              const float *dinv, const uint8_t *owner,
                                                              const ChunkDesc *ch, CgScalars s, double *partial) {
  __shared__ double sh[kBlasThreads];
  const ChunkDesc c = ch[blockIdx.x];
  const bool act = s.oact[c.inst] != 0;
  const double inv = act ? 1.0 / s.rnorm[c.inst] : 0.0;
  double acc = 0;
  for (int i = threadIdx.x; i < c.len; i += kBlasThreads) {
    const int64_t g = c.start + i;
    const float v = act ? float(r64[g] * inv) : 0.0f;
    const float z = dinv ? dinv[g] * v : v;
    r32[g] = v;
    p[g] = z;
    d[g] = 0.0f;
    if (owner == nullptr || owner[g]) acc += double(v) * double(z);
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

__global__ void k_cg_init(const double *partial, const int *first, int count, CgScalars s) {
  const int i = blockIdx.x;
  if (i >= count) return;
  const double rr = inst_sum(partial, first, i);
  if (threadIdx.x != 0) return;
  s.rr[i] = rr;
  s.rr0[i] = rr;
  s.iact[i] = (s.oact[i] && rr > 0) ? 1 : 0;
  s.it[i] = 0;
}

// alpha = rr / (p.q) for inner-active instances, else 0
__global__ void k_cg_alpha(const double *partial, const int *first, int count, CgScalars s) {
  const int i = blockIdx.x;
  if (i >= count) return;
  const double pq = inst_sum(partial, first, i);
  if (threadIdx.x != 0) return;
  s.alpha[i] = (s.iact[i] && pq > 0) ? s.rr[i] / pq : 0.0;
}

// d += alpha p, r -= alpha q; partial r.z.  A chunk whose instance takes no
// step (alpha = 0) is left alone: its q was not computed.
__global__ __launch_bounds__(kBlasThreads) void k_cg_update(float *d, float *r, const float *p, const float *q,
                                                             const float *dinv, const uint8_t *owner,
                                                             const ChunkDesc *ch, CgScalars s, double *partial) {
  __shared__ double sh[kBlasThreads];
  const ChunkDesc c = ch[blockIdx.x];
  if (s.alpha[c.inst] == 0.0) {
    if (threadIdx.x == 0) partial[blockIdx.x] = 0.0;
    return;
  }
  const float a = float(s.alpha[c.inst]);
  double acc = 0;
  for (int i = threadIdx.x; i < c.len; i += kBlasThreads) {
    const int64_t g = c.start + i;
    const float rv = r[g] - a * q[g];
    d[g] += a * p[g];
    r[g] = rv;
    const float z = dinv ? dinv[g] * rv : rv;
    if (owner == nullptr || owner[g]) acc += double(rv) * double(z);
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// beta = rr_new / rr; convergence test of the inner iteration
__global__ void k_cg_beta(const double *partial, const int *first, int count, double rtol2, int maxit,
                          CgScalars s) {
  const int i = blockIdx.x;
  if (i >= count) return;
  if (!s.iact[i]) {
    if (threadIdx.x == 0) s.beta[i] = 0.0;
    return;
  }
  const double rrn = inst_sum(partial, first, i);
  if (threadIdx.x != 0) return;
  s.beta[i] = rrn / s.rr[i];
  s.rr[i] = rrn;
  const int it = s.it[i] + 1;
  s.it[i] = it;
  s.iact[i] = (rrn > rtol2 * s.rr0[i] && it < maxit) ? 1 : 0;
}

// p = z + beta p (z = dinv r) for instances that took the step
__global__ __launch_bounds__(kBlasThreads) void k_cg_p(float *p, const float *r, const float *dinv,
                                                        const ChunkDesc *ch, CgScalars s) {
  const ChunkDesc c = ch[blockIdx.x];
  if (s.alpha[c.inst] == 0.0) return;
  const float b = float(s.beta[c.inst]);
  for (int i = threadIdx.x; i < c.len; i += kBlasThreads) {
    const int64_t g = c.start + i;
    const float z = dinv ? dinv[g] * r[g] : r[g];
    p[g] = z + b * p[g];
  }
}

// dinv = 1 / d where d > 0 (0 on Dirichlet rows, whose diagonal is 0)
__global__ __launch_bounds__(kBlasThreads) void k_inv_diag(const double *d, float *dinv, const ChunkDesc *ch) {
  const ChunkDesc c = ch[blockIdx.x];
  for (int i = threadIdx.x; i < c.len; i += kBlasThreads) {
    const int64_t g = c.start + i;
    dinv[g] = d[g] > 0.0 ? float(1.0 / d[g]) : 0.0f;
  }
}

// x += |r| d for instances refined in this outer step
__global__ __launch_bounds__(kBlasThreads) void k_update_x(double *x, const float *d, const ChunkDesc *ch,
                                                            CgScalars s) {
  const ChunkDesc c = ch[blockIdx.x];
  if (!s.oact[c.inst]) return;
  const double sc = s.rnorm[c.inst];
  for (int i = threadIdx.x; i < c.len; i += kBlasThreads) {
    const int64_t g = c.start + i;
    x[g] += sc * double(d[g]);
  }
}

}  // namespace

#define TMF_LAUNCH(kernel, grid, block, s, ...)                               \
  do {                                                                        \
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, s, __VA_ARGS__); \
    hipError_t e_ = hipGetLastError();                                        \
    if (e_ != hipSuccess) return e_;                                          \
  } while (0)

hipError_t blas_residual(const BlasCtx &c, const double *b, const double *Ax, double *r, double *prr, double *pbb,
                         double tol, hipStream_t s) {
  TMF_LAUNCH(k_residual, c.nchunks, kBlasThreads, s, b, Ax, r, c.owner, c.chunks, prr, pbb);
  TMF_LAUNCH(k_outer_norms, c.count, 64, s, prr, pbb, c.first, c.count, tol, c.sc);
  return hipSuccess;
}

hipError_t blas_start_inner(const BlasCtx &c, const double *r64, float *r32, float *p, float *d, double *part,
                            hipStream_t s) {
  TMF_LAUNCH(k_scale_cast, c.nchunks, kBlasThreads, s, r64, r32, p, d, c.dinv, c.owner, c.chunks, c.sc, part);
  TMF_LAUNCH(k_cg_init, c.count, 64, s, part, c.first, c.count, c.sc);
  return hipSuccess;
}

hipError_t blas_cg_step_after_apply(const BlasCtx &c, float *d, float *r, float *p, const float *q, double *part,
                                    double rtol2, int maxit, hipStream_t s) {
  TMF_LAUNCH((k_dot_partial<float, float>), c.nchunks, kBlasThreads, s, p, q, c.owner, c.chunks, part);
  TMF_LAUNCH(k_cg_alpha, c.count, 64, s, part, c.first, c.count, c.sc);
  TMF_LAUNCH(k_cg_update, c.nchunks, kBlasThreads, s, d, r, p, q, c.dinv, c.owner, c.chunks, c.sc, part);
  TMF_LAUNCH(k_cg_beta, c.count, 64, s, part, c.first, c.count, rtol2, maxit, c.sc);
  TMF_LAUNCH(k_cg_p, c.nchunks, kBlasThreads, s, p, r, c.dinv, c.chunks, c.sc);
  return hipSuccess;
}

hipError_t blas_inverse_diagonal(const BlasCtx &c, const double *d, float *dinv, hipStream_t s) {
  TMF_LAUNCH(k_inv_diag, c.nchunks, kBlasThreads, s, d, dinv, c.chunks);
  return hipSuccess;
}

hipError_t blas_update_x(const BlasCtx &c, double *x, const float *d, hipStream_t s) {
  TMF_LAUNCH(k_update_x, c.nchunks, kBlasThreads, s, x, d, c.chunks, c.sc);
  return hipSuccess;
}

}  // namespace tmf
