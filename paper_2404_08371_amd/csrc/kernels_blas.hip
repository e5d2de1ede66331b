// Vector kernels of the batched Krylov solver.
//
// A batch concatenates the vectors of its instances; every kernel walks a
// fixed list of chunks (instance, start, length), one workgroup per chunk,
// so per-instance reductions are two-pass and deterministic: each chunk
// writes one FP64 partial (a fixed butterfly inside each wavefront, then the
// wavefronts in order), and a second pass adds an instance's partials in
// chunk order.  CG scalars live per instance in device memory; an instance
// whose inner iteration has converged keeps its vectors unchanged (alpha = 0
// and p frozen), and its q is never read (the solver's applies skip inactive
// instances).
//
// The inner vectors are of type V: float (the FP32 inner iteration of
// iterative refinement) or double (plain FP64 CG, the comparison form).  One
// inner iteration after the apply q = A p is three launches: the partials of
// p.q; the update, where every workgroup forms its instance's alpha from
// those partials (the first chunk of the instance also stores it) and then
// sets d += alpha p, r -= alpha q and the partials of r.z; and the direction
// update, where every workgroup forms beta = (r.z)_new / (r.z)_old and sets
// p = z + beta p, the first chunk storing (r.z)_new and the iteration state.
// (r.z) is kept in two slots that alternate between iterations (parity par),
// so that no workgroup of the direction update reads a value another one has
// already replaced.
//
// With a Jacobi preconditioner (dinv = 1 / diag(A), 0 on Dirichlet rows) the
// inner iteration is preconditioned CG: z = dinv r is formed on the fly where
// it is used, rr holds r.z, and the inner stopping test compares r.z with its
// initial value.
#include "solver_internal.h"

namespace tmf {

namespace {

// Sum over the workgroup (kBlasThreads threads): xor butterfly inside each
// wavefront, then the wavefront sums in order.  Deterministic; the result is
// valid in thread 0.  `sh` holds one value per wavefront and may be reused
// after the call (the trailing barrier).
__device__ inline double block_sum(double v, double *sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int t = threadIdx.x;
  if ((t & 63) == 0) sh[t >> 6] = v;
  __syncthreads();
  double s = 0;
#pragma unroll
  for (int w = 0; w < kBlasThreads / 64; ++w) s += sh[w];
  __syncthreads();
  return s;
}

// Sum of the partials of instance i, by one wavefront: lane l adds partials
// first[i] + l, + 64, ... in order, then a fixed xor butterfly.  Every lane
// ends with the same bits (a + b == b + a exactly), and the order depends only
// on the chunk list, so the result is reproducible run to run and identical in
// every workgroup that forms it.
__device__ inline double inst_sum(const double *partial, const int *first, int i) {
  const int lane = threadIdx.x & 63;
  double s = 0;
  for (int q = first[i] + lane; q < first[i + 1]; q += 64) s += partial[q];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  return s;
}

template <typename TA, typename TB>
__global__ __launch_bounds__(kBlasThreads) void k_dot_partial(const TA *a, const TB *b, const uint8_t *owner,
                                                               const ChunkDesc *ch, double *partial) {
  __shared__ double sh[kBlasThreads / 64];
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

// r64 = b - Ax, partials of r.r and b.b
__global__ __launch_bounds__(kBlasThreads) void k_residual(const double *b, const double *Ax, double *r,
                                                            const uint8_t *owner, const ChunkDesc *ch,
                                                            double *prr, double *pbb) {
  __shared__ double sh[kBlasThreads / 64];
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
  sbb = block_sum(sbb, sh);
  if (threadIdx.x == 0) {
    prr[blockIdx.x] = srr;
    pbb[blockIdx.x] = sbb;
  }
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

// r = r64 / |r| for active instances (0 otherwise), p = z = dinv r, d = 0;
// partial r.z
template <typename V>
__global__ __launch_bounds__(kBlasThreads) void k_scale_cast(const double *r64, V *r, V *p, V *d, const V *dinv,
                                                              const uint8_t *owner, const ChunkDesc *ch, CgScalars s,
                                                              double *partial) {
  __shared__ double sh[kBlasThreads / 64];
  const ChunkDesc c = ch[blockIdx.x];
  const bool act = s.oact[c.inst] != 0;
  const double inv = act ? 1.0 / s.rnorm[c.inst] : 0.0;
  double acc = 0;
  for (int i = threadIdx.x; i < c.len; i += kBlasThreads) {
    const int64_t g = c.start + i;
    const V v = act ? V(r64[g] * inv) : V(0);
    const V z = dinv ? dinv[g] * v : v;
    r[g] = v;
    p[g] = z;
    d[g] = V(0);
    if (owner == nullptr || owner[g]) acc += double(v) * double(z);
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// initial r.z in slot 0 of the alternating pair, the inner stopping reference
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

// alpha = (r.z) / (p.q) for inner-active instances, else 0 (formed in every
// workgroup from the p.q partials, stored by the instance's first chunk);
// then d += alpha p, r -= alpha q and the partials of r.z.  A chunk whose
// instance takes no step (alpha = 0) is left alone: its q was not computed.
template <typename V>
__global__ __launch_bounds__(kBlasThreads) void k_cg_update(V *d, V *r, const V *p, const V *q, const V *dinv,
                                                             const uint8_t *owner, const ChunkDesc *ch,
                                                             const int *first, CgScalars s, const double *ppq,
                                                             double *prz, int par) {
  __shared__ double sh[kBlasThreads / 64];
  const ChunkDesc c = ch[blockIdx.x];
  const int i = c.inst;
  double alpha = 0.0;
  if (s.iact[i]) {
    const double pq = inst_sum(ppq, first, i);
    alpha = pq > 0 ? s.rr[par * s.count + i] / pq : 0.0;
  }
  if (threadIdx.x == 0 && static_cast<int>(blockIdx.x) == first[i]) s.alpha[i] = alpha;
  if (alpha == 0.0) {
    if (threadIdx.x == 0) prz[blockIdx.x] = 0.0;
    return;
  }
  const V a = V(alpha);
  double acc = 0;
  for (int t = threadIdx.x; t < c.len; t += kBlasThreads) {
    const int64_t g = c.start + t;
    const V rv = r[g] - a * q[g];
    d[g] += a * p[g];
    r[g] = rv;
    const V z = dinv ? dinv[g] * rv : rv;
    if (owner == nullptr || owner[g]) acc += double(rv) * double(z);
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) prz[blockIdx.x] = acc;
}

// beta = (r.z)_new / (r.z)_old and p = z + beta p (z = dinv r) for instances
// that took the step; the instance's first chunk stores (r.z)_new in the other
// slot and advances the iteration state (count, inner activity)
template <typename V>
__global__ __launch_bounds__(kBlasThreads) void k_cg_p(V *p, const V *r, const V *dinv, const ChunkDesc *ch,
                                                        const int *first, CgScalars s, const double *prz,
                                                        double rtol2, int maxit, int par) {
  const ChunkDesc c = ch[blockIdx.x];
  const int i = c.inst;
  if (s.alpha[i] == 0.0) return;
  const double rrn = inst_sum(prz, first, i);
  const double rro = s.rr[par * s.count + i];
  const double beta = rrn / rro;
  if (threadIdx.x == 0 && static_cast<int>(blockIdx.x) == first[i]) {
    s.rr[(1 - par) * s.count + i] = rrn;
    s.beta[i] = beta;
    const int it = s.it[i] + 1;
    s.it[i] = it;
    s.iact[i] = (rrn > rtol2 * s.rr0[i] && it < maxit) ? 1 : 0;
  }
  const V b = V(beta);
  for (int t = threadIdx.x; t < c.len; t += kBlasThreads) {
    const int64_t g = c.start + t;
    const V z = dinv ? dinv[g] * r[g] : r[g];
    p[g] = z + b * p[g];
  }
}

// dinv = 1 / d where d > 0 (0 on Dirichlet rows, whose diagonal is 0)
template <typename V>
__global__ __launch_bounds__(kBlasThreads) void k_inv_diag(const double *d, V *dinv, const ChunkDesc *ch) {
  const ChunkDesc c = ch[blockIdx.x];
  for (int i = threadIdx.x; i < c.len; i += kBlasThreads) {
    const int64_t g = c.start + i;
    dinv[g] = d[g] > 0.0 ? V(1.0 / d[g]) : V(0);
  }
}

// x += |r| d for instances refined in this outer step
template <typename V>
__global__ __launch_bounds__(kBlasThreads) void k_update_x(double *x, const V *d, const ChunkDesc *ch, CgScalars s) {
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

template <typename V>
hipError_t blas_start_inner(const BlasCtx &c, const double *r64, V *r, V *p, V *d, double *part, hipStream_t s) {
  TMF_LAUNCH((k_scale_cast<V>), c.nchunks, kBlasThreads, s, r64, r, p, d, static_cast<const V *>(c.dinv), c.owner,
             c.chunks, c.sc, part);
  TMF_LAUNCH(k_cg_init, c.count, 64, s, part, c.first, c.count, c.sc);
  return hipSuccess;
}

template <typename V>
hipError_t blas_cg_step_after_apply(const BlasCtx &c, V *d, V *r, V *p, const V *q, double *ppq, double *prz,
                                    double rtol2, int maxit, int par, hipStream_t s) {
  const V *dinv = static_cast<const V *>(c.dinv);
  TMF_LAUNCH((k_dot_partial<V, V>), c.nchunks, kBlasThreads, s, p, q, c.owner, c.chunks, ppq);
  TMF_LAUNCH((k_cg_update<V>), c.nchunks, kBlasThreads, s, d, r, p, q, dinv, c.owner, c.chunks, c.first, c.sc, ppq,
             prz, par);
  TMF_LAUNCH((k_cg_p<V>), c.nchunks, kBlasThreads, s, p, r, dinv, c.chunks, c.first, c.sc, prz, rtol2, maxit, par);
  return hipSuccess;
}

template <typename V>
hipError_t blas_inverse_diagonal(const BlasCtx &c, const double *d, V *dinv, hipStream_t s) {
  TMF_LAUNCH((k_inv_diag<V>), c.nchunks, kBlasThreads, s, d, dinv, c.chunks);
  return hipSuccess;
}

template <typename V>
hipError_t blas_update_x(const BlasCtx &c, double *x, const V *d, hipStream_t s) {
  TMF_LAUNCH((k_update_x<V>), c.nchunks, kBlasThreads, s, x, d, c.chunks, c.sc);
  return hipSuccess;
}

#define TMF_BLAS_INST(V)                                                                                           \
  template hipError_t blas_start_inner<V>(const BlasCtx &, const double *, V *, V *, V *, double *, hipStream_t); \
  template hipError_t blas_cg_step_after_apply<V>(const BlasCtx &, V *, V *, V *, const V *, double *, double *,  \
                                                  double, int, int, hipStream_t);                                 \
  template hipError_t blas_inverse_diagonal<V>(const BlasCtx &, const double *, V *, hipStream_t);                \
  template hipError_t blas_update_x<V>(const BlasCtx &, double *, const V *, hipStream_t);
TMF_BLAS_INST(float)
TMF_BLAS_INST(double)
#undef TMF_BLAS_INST

}  // namespace tmf
