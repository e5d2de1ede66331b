// P1 operators: vertex-centric ("owner computes") matrix-free kernels.
//
// Each thread owns one lattice point p of one macro and forms row p of
// A x directly: y_p = sum over the (up to 24) micro-tets T containing p of
// (A_T x_T)_p (equation (4.1) restricted to one row).  Every row is written
// exactly once, so there are no write conflicts, no atomics and the
// summation order is fixed.  The 15-point neighbourhood of p is loaded once
// into registers; the local matrices are the per-(macro, type) constants
// Gp = |T| grad(lambda_a).grad(lambda_b) (affine macros: every micro-tet of a
// type has the same Jacobian -- the loop-invariant hoisting of section
// "Automatic Identification of Loop Invariants" done once on the host).
//
// Points at distance >= 2 from every macro face take a fast path: all 24
// micro-tets exist and no neighbour is a Dirichlet DoF, so the constant
// coefficient operator is a 15-point stencil.  Other points test each
// candidate micro-tet and mask boundary neighbours.
#include "tmf_internal.h"

namespace tmf {

namespace {

struct VSlotTable {
  int v[6][4][4];
};
constexpr VSlotTable make_vslot() {
  VSlotTable t{};
  for (int ty = 0; ty < 6; ++ty)
    for (int a = 0; a < 4; ++a)
      for (int c = 0; c < 4; ++c) t.v[ty][a][c] = vslot(ty, a, c);
  return t;
}
constexpr VSlotTable kVS = make_vslot();

// linear index within a macro lattice of size N -> (i, j, k)
__device__ inline void decode(int r, int N, int &i, int &j, int &k) {
  const int rem = c3(N) - r;  // >= 1: points in planes at or above the one holding r
  int M = static_cast<int>(cbrtf(6.0f * static_cast<float>(rem))) - 2;
  M = M < 0 ? 0 : (M > N ? N : M);
  while (M < N && c3(M) < rem) ++M;
  while (M > 0 && c3(M - 1) >= rem) --M;
  k = N - M;
  const int q = r - (c3(N) - c3(M));
  const float B = 2.0f * M + 3.0f;
  int jj = static_cast<int>(0.5f * (B - sqrtf(fmaxf(B * B - 8.0f * q, 0.0f))));
  jj = jj < 0 ? 0 : (jj > M ? M : jj);
  while (jj < M && ((jj + 1) * (2 * M + 3 - (jj + 1))) / 2 <= q) ++jj;
  while (jj > 0 && (jj * (2 * M + 3 - jj)) / 2 > q) --jj;
  j = jj;
  i = q - (jj * (2 * M + 3 - jj)) / 2;
}

__device__ inline bool is_bnd(uint32_t bnd, int i, int j, int k, int N) {
  return (bnd >> zero_pattern(i, j, k, N)) & 1u;
}

// load v at the 15-point neighbourhood; missing points read 0, and with MASK
// Dirichlet-boundary points read 0 as well
template <typename T, bool CHECK>
__device__ inline void load15(const T *__restrict__ v, int i, int j, int k, int N, bool mask,
                              uint32_t bnd, T out[15]) {
#pragma unroll
  for (int s = 0; s < 15; ++s) {
    const int ii = i + kNb[s][0], jj = j + kNb[s][1], kk = k + kNb[s][2];
    bool ok = true;
    if (CHECK) {
      ok = ii >= 0 && jj >= 0 && kk >= 0 && ii + jj + kk <= N;
      if (ok && mask) ok = !is_bnd(bnd, ii, jj, kk, N);
    }
    T val = T(0);
    if (ok) val = v[row_base(jj, kk, N) + ii];
    out[s] = val;
  }
}

template <bool CHECK>
__device__ inline bool tet_exists(int t, int a, int i, int j, int k, int N) {
  if (!CHECK) return true;
  const int bx = i - kOff[t][a][0], by = j - kOff[t][a][1], bz = k - kOff[t][a][2];
  return bx >= 0 && by >= 0 && bz >= 0 && bx + by + bz <= N - kLim[t];
}

// row p of sum_T kbar_T Gp_T x_T over the micro-tets containing p
template <typename T, bool VARK, bool CHECK>
__device__ inline T p1_row(const TypeGeo<T> *__restrict__ g, const T xs[15], const T ks[15], int i,
                           int j, int k, int N) {
  T acc = T(0);
#pragma unroll
  for (int t = 0; t < 6; ++t) {
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      if (tet_exists<CHECK>(t, a, i, j, k, N)) {
        const T *G = g[t].Gp + 4 * a;
        T r = G[0] * xs[kVS.v[t][a][0]];
        r += G[1] * xs[kVS.v[t][a][1]];
        r += G[2] * xs[kVS.v[t][a][2]];
        r += G[3] * xs[kVS.v[t][a][3]];
        if (VARK) {
          const T kb = (ks[kVS.v[t][a][0]] + ks[kVS.v[t][a][1]] + ks[kVS.v[t][a][2]] +
                        ks[kVS.v[t][a][3]]) * T(0.25);
          acc += kb * r;
        } else {
          acc += r;
        }
      }
    }
  }
  return acc;
}

template <typename T, int KIND>
__global__ __launch_bounds__(256) void k_p1_apply(P1Args<T> a) {
  constexpr bool VARK = KIND == P1_DIVKGRAD;
  const LatticeArgs<T> &L = a.lat;
  const int m = blockIdx.y;
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= L.L) return;
  const int N = L.N;
  int i, j, k;
  decode(r, N, i, j, k);
  const int64_t base = static_cast<int64_t>(m) * L.L;
  const uint32_t bnd = L.bnd[m];
  if (L.dirichlet && is_bnd(bnd, i, j, k, N)) {
    a.y[base + r] = T(0);
    return;
  }
  const T *x = a.x + base;
  const T *kc = VARK ? a.k + base : nullptr;
  const TypeGeo<T> *g = L.geo + 6 * m;
  const int d = L.dirichlet ? 2 : 1;
  const int s = i + j + k;
  T xs[15], ks[15];
  T acc;
  if (i >= d && j >= d && k >= d && s <= N - d) {
    load15<T, false>(x, i, j, k, N, false, bnd, xs);
    if (VARK) {
      load15<T, false>(kc, i, j, k, N, false, bnd, ks);
      acc = p1_row<T, true, false>(g, xs, ks, i, j, k, N);
    } else {
      const T *w = a.w15 + 15 * m;
      acc = T(0);
#pragma unroll
      for (int q = 0; q < 15; ++q) acc += w[q] * xs[q];
    }
  } else {
    load15<T, true>(x, i, j, k, N, L.dirichlet != 0, bnd, xs);
    if (VARK) load15<T, true>(kc, i, j, k, N, false, bnd, ks);
    acc = p1_row<T, VARK, true>(g, xs, ks, i, j, k, N);
  }
  a.y[base + r] = acc;
}

// Fused reverse mode of y = A(k) x for the P1 div(k grad) operator:
//   gx_p = (A(k) gy)_p
//   gk_p = sum_{T containing p} 1/4 (D gy)_T . Gp_T (D x)_T
// (A_T = kbar_T Gp_T with kbar_T the mean of the four nodal k of T).
template <typename T, bool CHECK>
__device__ inline T p1_kgrad(const TypeGeo<T> *__restrict__ g, const T rs[15], const T xs[15], int i,
                             int j, int k, int N) {
  T acc = T(0);
#pragma unroll
  for (int t = 0; t < 6; ++t) {
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      if (tet_exists<CHECK>(t, a, i, j, k, N)) {
        const T *G = g[t].Gp;
        T bil = T(0);
#pragma unroll
        for (int c1 = 0; c1 < 4; ++c1) {
          T row = G[4 * c1 + 0] * xs[kVS.v[t][a][0]];
          row += G[4 * c1 + 1] * xs[kVS.v[t][a][1]];
          row += G[4 * c1 + 2] * xs[kVS.v[t][a][2]];
          row += G[4 * c1 + 3] * xs[kVS.v[t][a][3]];
          bil += rs[kVS.v[t][a][c1]] * row;
        }
        acc += bil;
      }
    }
  }
  return acc * T(0.25);
}

template <typename T>
__global__ __launch_bounds__(256) void k_p1_adjoint(P1AdjArgs<T> a) {
  const LatticeArgs<T> &L = a.lat;
  const int m = blockIdx.y;
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= L.L) return;
  const int N = L.N;
  int i, j, k;
  decode(r, N, i, j, k);
  const int64_t base = static_cast<int64_t>(m) * L.L;
  const uint32_t bnd = L.bnd[m];
  const TypeGeo<T> *g = L.geo + 6 * m;
  const bool self_bnd = L.dirichlet && is_bnd(bnd, i, j, k, N);
  const int d = L.dirichlet ? 2 : 1;
  const int s = i + j + k;
  T rs[15], xs[15], ks[15];
  T gx, gk;
  if (i >= d && j >= d && k >= d && s <= N - d) {
    load15<T, false>(a.gy + base, i, j, k, N, false, bnd, rs);
    load15<T, false>(a.x + base, i, j, k, N, false, bnd, xs);
    load15<T, false>(a.k + base, i, j, k, N, false, bnd, ks);
    gx = p1_row<T, true, false>(g, rs, ks, i, j, k, N);
    gk = p1_kgrad<T, false>(g, rs, xs, i, j, k, N);
  } else {
    const bool mask = L.dirichlet != 0;
    load15<T, true>(a.gy + base, i, j, k, N, mask, bnd, rs);
    load15<T, true>(a.x + base, i, j, k, N, mask, bnd, xs);
    load15<T, true>(a.k + base, i, j, k, N, false, bnd, ks);
    gx = self_bnd ? T(0) : p1_row<T, true, true>(g, rs, ks, i, j, k, N);
    gk = p1_kgrad<T, true>(g, rs, xs, i, j, k, N);
  }
  a.gx[base + r] = gx;
  if (a.gk) a.gk[base + r] = gk;
}

}  // namespace

template <typename T>
hipError_t launch_p1_apply(const P1Args<T> &a, int kind, hipStream_t s) {
  dim3 grid((a.lat.L + 255) / 256, a.lat.nt);
  if (kind == P1_LAPLACE)
    hipLaunchKernelGGL((k_p1_apply<T, P1_LAPLACE>), grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_p1_apply<T, P1_DIVKGRAD>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_p1_adjoint(const P1AdjArgs<T> &a, hipStream_t s) {
  dim3 grid((a.lat.L + 255) / 256, a.lat.nt);
  hipLaunchKernelGGL((k_p1_adjoint<T>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

template hipError_t launch_p1_apply<double>(const P1Args<double> &, int, hipStream_t);
template hipError_t launch_p1_apply<float>(const P1Args<float> &, int, hipStream_t);
template hipError_t launch_p1_adjoint<double>(const P1AdjArgs<double> &, hipStream_t);
template hipError_t launch_p1_adjoint<float>(const P1AdjArgs<float> &, hipStream_t);

}  // namespace tmf
