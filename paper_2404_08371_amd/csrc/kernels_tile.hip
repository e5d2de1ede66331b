// P2 and vector-P2 operators: element-centric kernels over LDS-staged tiles.
//
// A workgroup owns a box of TX x TY x TZ micro-cubes of one macro (the
// spatial blocking of section "Cubes Loop Strategy": all micro-tets of a
// cube, and of neighbouring cubes, reuse DoFs already staged on chip).  It
//   1. stages the (2TX+1)(2TY+1)(2TZ+1) P2 lattice points of the box (x, the
//      coefficient, Dirichlet mask applied to x) from HBM into LDS,
//   2. applies the fused local operator to every micro-tet of the box -- a
//      lane per cube, each wavefront running a fixed subset of the six
//      micro-tet types -- and accumulates the 10 (or 30) local results into
//      an FP64 LDS copy of y,
//   3. writes y at the points that belong to this box alone, and its partial
//      sums at the points of box faces shared with neighbouring boxes to the
//      instance's partial buffer; a second kernel (k_seam) adds the partials
//      of each shared point in a fixed order.  Every entry of y is written
//      once: no global atomics and no zero fill of y.  Inside a box the six
//      wavefronts add into the LDS copy of y with LDS atomics, whose order
//      across wavefronts is not fixed, so two applies can differ in the last
//      bits of a sum (both within rounding of the exact one).
// The local operator is never formed (remark on fused local quadrature after
// algorithm "LocalApply"): for affine elements the gradient of a P2 field is
// a P1 field, grad u = sum_a lambda_a g_a, and every integral becomes a
// product with exact weights int k lambda_a lambda_e; see p2_elem.
#include "tmf_internal.h"

namespace tmf {

namespace {

__device__ inline bool is_bnd(uint32_t bnd, int i, int j, int k, int N) {
  return (bnd >> zero_pattern(i, j, k, N)) & 1u;
}

// Per-type geometry and quadrature tables are read-only for the whole launch
// and indexed by wave-uniform values (type, quadrature point).  Reading them
// through the constant address space turns the reads into scalar loads kept
// in SGPRs; through a generic pointer they would be per-lane flat loads whose
// completion every later LDS wait also has to cover.
template <typename T>
using CPtr = const __attribute__((address_space(4))) T *;
template <typename T>
__device__ __forceinline__ CPtr<T> cptr(const T *p) {
  return (CPtr<T>)p;
}
// A pointer read from a descriptor in memory has no known address space, so
// accesses through it compile to flat instructions, which count against both
// the vector-memory and the LDS wait counters: a later LDS wait then also
// waits for every flat load or store in flight, and loads that the code
// issues one after another complete one after another.  Per-lane accesses
// through such pointers are therefore cast to the global address space.
template <typename T>
using GPtr = __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ GPtr<T> gptr(T *p) {
  return (GPtr<T>)p;
}
// LDS view of a __shared__ array (a generic pointer to it would again be flat)
template <typename T>
using LPtr = const __attribute__((address_space(3))) T *;

// Exact weights W_ce = (1/|T|) int_T k lambda_c lambda_e for k nodal P2.
// k in Bernstein form: k = sum_b kappa_b B_b, B_aa = lambda_a^2,
// B_ab = 2 lambda_a lambda_b, kappa_aa = k_a, kappa_ab = 2 k_ab - (k_a + k_b)/2.
// With int lambda^g = 6|T| g!/(|g|+3)!:  W_ce = (kappa_ce + S1_c + S1_e + S0)/420
// (c != e), W_cc = (S2_c + 3 S1_c + 2 S0)/420, S0 = sum kappa, S1_c = sum_b
// kappa_b b_c, S2_c = sum_b kappa_b b_c^2.
template <typename T>
__device__ inline void weights_p2(const T kv[10], T W[4][4]) {
  T kap[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a) kap[a][a] = kv[a];
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    const int a = kEdge[e][0], b = kEdge[e][1];
    const T v = T(2) * kv[4 + e] - T(0.5) * (kv[a] + kv[b]);
    kap[a][b] = v;
    kap[b][a] = v;
  }
  T S0 = T(0), S1[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    T off = T(0);
#pragma unroll
    for (int b = 0; b < 4; ++b)
      if (b != c) off += kap[c][b];
    S1[c] = T(2) * kap[c][c] + off;
    S0 += kap[c][c];
  }
#pragma unroll
  for (int e = 0; e < 6; ++e) S0 += kap[kEdge[e][0]][kEdge[e][1]];
  const T s = T(1) / T(420);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    W[c][c] = (S1[c] + T(2) * kap[c][c] + T(3) * S1[c] + T(2) * S0) * s;
#pragma unroll
    for (int e = c + 1; e < 4; ++e) {
      const T v = (kap[c][e] + S1[c] + S1[e] + S0) * s;
      W[c][e] = v;
      W[e][c] = v;
    }
  }
}

// The same weights scaled by 840, with the Bernstein sums collected in the
// nodal values: with V = sum of the vertex values k_c, E_c = sum of the edge
// values at vertex c and h = sum_c E_c - 3 V / 2,
//   840 W_ce = 4 k_ce + b_c + b_e  (c != e),   840 W_cc = 4 (b_c + 2 k_c),
//   b_c = k_c + 4 E_c + h
// (43 operations instead of 71 for the form above).
template <typename T>
__device__ inline void weights_p2_840(const T kv[10], T W[4][4]) {
  T E[4];
  E[0] = kv[4] + kv[5] + kv[6];
  E[1] = kv[4] + kv[7] + kv[8];
  E[2] = kv[5] + kv[7] + kv[9];
  E[3] = kv[6] + kv[8] + kv[9];
  const T V = (kv[0] + kv[1]) + (kv[2] + kv[3]);
  const T h = T(-1.5) * V + ((E[0] + E[1]) + (E[2] + E[3]));
  T b[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    b[c] = T(4) * E[c] + (kv[c] + h);
    W[c][c] = T(4) * (T(2) * kv[c] + b[c]);
  }
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    const int c = kEdge[e][0], d = kEdge[e][1];
    const T v = T(4) * kv[4 + e] + (b[c] + b[d]);
    W[c][d] = v;
    W[d][c] = v;
  }
}

// Gradient coefficients of a P2 field on an affine tet in the barycentric
// gradient basis: grad u = sum_c lambda_c g_c with g_c = sum_a s[c][a] grad(lambda_a),
// s[c][c] = 3 u_c, s[c][a] = 4 u_ca - u_a.  Returned shifted by s[c][0]
// (sum_a grad(lambda_a) = 0), as sp[c][a-1] for a = 1..3.
template <typename T>
__device__ inline void grad_coeffs(const T u[10], T sp[4][3]) {
  T s[4][4];
#pragma unroll
  for (int c = 0; c < 4; ++c) s[c][c] = T(3) * u[c];
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    const int a = kEdge[e][0], b = kEdge[e][1];
    s[a][b] = T(4) * u[4 + e] - u[b];
    s[b][a] = T(4) * u[4 + e] - u[a];
  }
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int a = 1; a < 4; ++a) sp[c][a - 1] = s[c][a] - s[c][0];
}

// Fused local apply of int k grad u . grad phi_j on one affine tet.
//   h[c][d] = g_c . |T| grad(lambda_d)          (16 values, Gp = |T| G)
//   sigma[e][d] = sum_c W_ce h[c][d]
//   y_vertex b = 4 sigma[b][b] - sum_e sigma[e][b]
//   y_edge bc  = 4 (sigma[c][b] + sigma[b][c])
// (from grad phi_b = (4 lambda_b - 1) grad lambda_b and
//  grad phi_bc = 4 (lambda_c grad lambda_b + lambda_b grad lambda_c)).
// The apply with given coefficient weights W (see p2_elem).
template <typename T>
__device__ inline void p2_elem_w(const T u[10], const T W[4][4], CPtr<T> Gp, T y[10]) {
  T sp[4][3];
  grad_coeffs(u, sp);
  T h[4][4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
#pragma unroll
    for (int d = 1; d < 4; ++d)
      h[c][d] = sp[c][0] * Gp[4 * 1 + d] + sp[c][1] * Gp[4 * 2 + d] + sp[c][2] * Gp[4 * 3 + d];
    h[c][0] = -(h[c][1] + h[c][2] + h[c][3]);
  }
  T sig[4][4];
#pragma unroll
  for (int e = 0; e < 4; ++e)
#pragma unroll
    for (int d = 0; d < 4; ++d)
      sig[e][d] = W[0][e] * h[0][d] + W[1][e] * h[1][d] + W[2][e] * h[2][d] + W[3][e] * h[3][d];
#pragma unroll
  for (int b = 0; b < 4; ++b)
    y[b] = T(4) * sig[b][b] - (sig[0][b] + sig[1][b] + sig[2][b] + sig[3][b]);
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    const int b = kEdge[e][0], c = kEdge[e][1];
    y[4 + e] = T(4) * (sig[c][b] + sig[b][c]);
  }
}

// Weights W_ce = (1/|T|) int k lambda_c lambda_e by a quadrature rule (the
// under-integration variant): 6 sum_q w_q k(q) lambda_c(q) lambda_e(q), with
// k(q) = sum_b k_b phi_b(q); table rows [w, lambda(4), phi(10), ...].
template <typename T>
__device__ inline void weights_quad(const T kv[10], CPtr<T> qtab, int nq, T W[4][4]) {
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int e = 0; e < 4; ++e) W[c][e] = T(0);
  for (int q = 0; q < nq; ++q) {
    CPtr<T> Q = qtab + q * kQStride;
    T kq = T(0);
#pragma unroll
    for (int b = 0; b < 10; ++b) kq += kv[b] * Q[5 + b];
    const T f = T(6) * Q[0] * kq;
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int e = c; e < 4; ++e) W[c][e] += f * Q[1 + c] * Q[1 + e];
  }
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int e = 0; e < c; ++e) W[c][e] = W[e][c];
}

template <typename T, bool HASK>
__device__ inline void p2_elem(const T u[10], const T kv[10], CPtr<T> Gp, CPtr<T> Gs, T y[10]) {
  T sp[4][3];
  grad_coeffs(u, sp);
  if (HASK) {
    // sig' = 4 sig = (W'^T sp) Gs with W' = 840 W and Gs = Gp / 210 (rows
    // 1..3; Gp has zero row sums, so the column of lambda_0 follows from the
    // other three): 4 x 3 then 4 x 3 products, and the edge outputs become
    // plain sums
    T W[4][4];
    weights_p2_840(kv, W);
    T sig[4][4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      T Q[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) Q[a] = W[0][e] * sp[0][a] + W[1][e] * sp[1][a] + W[2][e] * sp[2][a] + W[3][e] * sp[3][a];
#pragma unroll
      for (int d = 1; d < 4; ++d) sig[e][d] = Q[0] * Gs[d] + Q[1] * Gs[4 + d] + Q[2] * Gs[8 + d];
      sig[e][0] = -(sig[e][1] + sig[e][2] + sig[e][3]);
    }
#pragma unroll
    for (int b = 0; b < 4; ++b)
      y[b] = sig[b][b] - T(0.25) * (sig[0][b] + sig[1][b] + sig[2][b] + sig[3][b]);
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      const int b = kEdge[e][0], c = kEdge[e][1];
      y[4 + e] = sig[c][b] + sig[b][c];
    }
  } else {
    T h[4][4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
#pragma unroll
      for (int d = 1; d < 4; ++d)
        h[c][d] = sp[c][0] * Gp[4 * 1 + d] + sp[c][1] * Gp[4 * 2 + d] + sp[c][2] * Gp[4 * 3 + d];
      h[c][0] = -(h[c][1] + h[c][2] + h[c][3]);
    }
    // W = (1 + delta)/20
    T sig[4][4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const T H = h[0][d] + h[1][d] + h[2][d] + h[3][d];
#pragma unroll
      for (int e = 0; e < 4; ++e) sig[e][d] = (H + h[e][d]) * T(0.05);
    }
#pragma unroll
    for (int b = 0; b < 4; ++b)
      y[b] = T(4) * sig[b][b] - (sig[0][b] + sig[1][b] + sig[2][b] + sig[3][b]);
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      const int b = kEdge[e][0], c = kEdge[e][1];
      y[4 + e] = T(4) * (sig[c][b] + sig[b][c]);
    }
  }
}

// Diagonal of the local matrix: entry v is (A_T e_v)_v.  The unit vectors
// are compile-time constants, so the unrolled calls fold to the terms that
// touch node v (and the coefficient weights are formed once).
template <typename T, bool HASK>
__device__ inline void p2_diag(const T kv[10], CPtr<T> Gp, CPtr<T> Gs, T d[10]) {
#pragma unroll
  for (int v = 0; v < 10; ++v) {
    T u[10], y[10];
#pragma unroll
    for (int w = 0; w < 10; ++w) u[w] = w == v ? T(1) : T(0);
    p2_elem<T, HASK>(u, kv, Gp, Gs, y);
    d[v] = y[v];
  }
}

// Coefficient gradient of the local div(k grad) form: A_T(k) is linear in the
// 10 nodal values of k, so gk_b = gy . A_T(e_b) u.  Writing the apply as
// y = Y(sigma), sigma[e][d] = sum_c W[c][e] h[c][d] (see p2_elem), gives
// gy . y = sum_{c,e} W[c][e] M[c][e] with M[c][e] = sum_d h[c][d] Gam[e][d],
// where Gam collects the coefficients of gy . Y(sigma) in sigma; then
// gk_b = sum_{c,e} W(e_b)[c][e] M[c][e] with the constant weights W(e_b).
template <typename T>
__device__ inline void p2_gradk(const T u[10], const T g[10], CPtr<T> Gp, T gk[10]) {
  T sp[4][3];
  grad_coeffs(u, sp);
  T h[4][4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
#pragma unroll
    for (int d = 1; d < 4; ++d)
      h[c][d] = sp[c][0] * Gp[4 * 1 + d] + sp[c][1] * Gp[4 * 2 + d] + sp[c][2] * Gp[4 * 3 + d];
    h[c][0] = -(h[c][1] + h[c][2] + h[c][3]);
  }
  // gy . Y(sigma) = sum_b g_b (4 sigma[b][b] - sum_e sigma[e][b])
  //               + sum_edges (b,c) 4 g_bc (sigma[c][b] + sigma[b][c])
  T gam[4][4];
#pragma unroll
  for (int e = 0; e < 4; ++e)
#pragma unroll
    for (int b = 0; b < 4; ++b) gam[e][b] = -g[b] + (e == b ? T(4) * g[b] : T(0));
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    const int b = kEdge[e][0], c = kEdge[e][1];
    gam[c][b] += T(4) * g[4 + e];
    gam[b][c] += T(4) * g[4 + e];
  }
  T M[4][4];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int e = 0; e < 4; ++e)
      M[c][e] = h[c][0] * gam[e][0] + h[c][1] * gam[e][1] + h[c][2] * gam[e][2] + h[c][3] * gam[e][3];
  // With the collected weights of weights_p2_840, 840 sum W M =
  // sum_edges 4 k_ce P_ce + sum_c b_c Z_c + sum_c 8 k_c M_cc (P_ce = M_ce + M_ec,
  // Z_c = sum_{e != c} P_ce + 4 M_cc), whose derivatives are
  //   840 gk_c  = Z_c + 8 M_cc - 3/2 sum Z,
  //   840 gk_ce = 4 P_ce + 4 (Z_c + Z_e) + 2 sum Z.
  T P[6];
#pragma unroll
  for (int e = 0; e < 6; ++e) P[e] = M[kEdge[e][0]][kEdge[e][1]] + M[kEdge[e][1]][kEdge[e][0]];
  T Z[4];
  Z[0] = (P[0] + P[1]) + (P[2] + T(4) * M[0][0]);
  Z[1] = (P[0] + P[3]) + (P[4] + T(4) * M[1][1]);
  Z[2] = (P[1] + P[3]) + (P[5] + T(4) * M[2][2]);
  Z[3] = (P[2] + P[4]) + (P[5] + T(4) * M[3][3]);
  const T zs = (Z[0] + Z[1]) + (Z[2] + Z[3]);
  const T s = T(1) / T(840);
#pragma unroll
  for (int c = 0; c < 4; ++c) gk[c] = (Z[c] + T(8) * M[c][c] - T(1.5) * zs) * s;
#pragma unroll
  for (int e = 0; e < 6; ++e)
    gk[4 + e] = (T(4) * (P[e] + Z[kEdge[e][0]] + Z[kEdge[e][1]]) + T(2) * zs) * s;
}

// Fused local apply of int 2 mu eps(u):eps(v) on one affine tet.
//   component gradients: grad u_c = sum_a lambda_a g^c_a
//   strain at vertex a: E_a = sym(G_a), row c of G_a = g^c_a
//   sigma_e = sum_a W_ae E_a   (W from mu as above)
//   y_vertex b = 2|T| (4 sigma_b - sum_e sigma_e) grad lambda_b
//   y_edge bc  = 8|T| (sigma_c grad lambda_b + sigma_b grad lambda_c)
template <typename T>
__device__ inline void eps_elem(const T u[3][10], const T mu[10], CPtr<T> grad, T vol, T y[3][10]) {
  // g[c][a][r]
  T E[4][6];  // symmetric strain per vertex: xx, yy, zz, xy, xz, yz
  {
    T g[3][4][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T sp[4][3];
      grad_coeffs(u[c], sp);
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int r = 0; r < 3; ++r)
          g[c][a][r] = sp[a][0] * grad[3 * 1 + r] + sp[a][1] * grad[3 * 2 + r] + sp[a][2] * grad[3 * 3 + r];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      E[a][0] = g[0][a][0];
      E[a][1] = g[1][a][1];
      E[a][2] = g[2][a][2];
      E[a][3] = T(0.5) * (g[0][a][1] + g[1][a][0]);
      E[a][4] = T(0.5) * (g[0][a][2] + g[2][a][0]);
      E[a][5] = T(0.5) * (g[1][a][2] + g[2][a][1]);
    }
  }
  T W[4][4];
  weights_p2(mu, W);
  T sig[4][6], tot[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) tot[q] = T(0);
#pragma unroll
  for (int e = 0; e < 4; ++e)
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      sig[e][q] = W[0][e] * E[0][q] + W[1][e] * E[1][q] + W[2][e] * E[2][q] + W[3][e] * E[3][q];
      tot[q] += sig[e][q];
    }
  auto matvec = [](const T S[6], CPtr<T> v, T out[3]) {
    out[0] = S[0] * v[0] + S[3] * v[1] + S[4] * v[2];
    out[1] = S[3] * v[0] + S[1] * v[1] + S[5] * v[2];
    out[2] = S[4] * v[0] + S[5] * v[1] + S[2] * v[2];
  };
  const T fv = T(2) * vol, fe = T(8) * vol;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    T S[6], o[3];
#pragma unroll
    for (int q = 0; q < 6; ++q) S[q] = fv * (T(4) * sig[b][q] - tot[q]);
    matvec(S, grad + 3 * b, o);
#pragma unroll
    for (int c = 0; c < 3; ++c) y[c][b] = o[c];
  }
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    const int b = kEdge[e][0], c2 = kEdge[e][1];
    T o1[3], o2[3];
    matvec(sig[c2], grad + 3 * b, o1);
    matvec(sig[b], grad + 3 * c2, o2);
#pragma unroll
    for (int c = 0; c < 3; ++c) y[c][4 + e] = fe * (o1[c] + o2[c]);
  }
}

// Epsilon operator on a curved element of the radially blended map
// x = Phi(xi) = xi (s.xi)/|xi|, integrated with the given rule:
//   xi_q = P0 + JT xhat_q, J = DPhi(xi_q) JT,
//   grad u_c = (ref-grad u_c) J^-1,  sigma = 2 mu_q w_q |det J| sym(grad u),
//   y_(i,d) += sum_r (sigma J^-T)_(d r) ref-grad_r phi_i(xhat_q).
// DPhi = a0 I + xi v^T with a0 = rho/|xi|, rho = s.xi > 0 and
// v = s/|xi| - rho xi/|xi|^3.  Since v.xi = 0, DPhi^-1 = (I - xi v^T/a0)/a0
// and det DPhi = a0^3; J^-1 = JT^-1 DPhi^-1, whose first factor is the
// micro-tet's (constant) barycentric gradients.
// 1 / sqrt(v) and 1 / v (v > 0) from the hardware estimates refined by
// Newton's iteration (reciprocal square root: y <- y (3 - v y^2) / 2;
// reciprocal: y <- y + y (1 - v y)); each step doubles the correct bits, two
// steps reach double precision to a few ulp, one step single precision
template <typename T>
__device__ __forceinline__ T rsqrt_nr(T v) {
  if constexpr (sizeof(T) == 8) {
    T y = __builtin_amdgcn_rsq(v);
#pragma unroll
    for (int i = 0; i < 2; ++i) y = y * (T(1.5) - T(0.5) * v * y * y);
    return y;
  } else {
    const T y = __builtin_amdgcn_rsqf(v);
    return y * (T(1.5) - T(0.5) * v * y * y);
  }
}
template <typename T>
__device__ __forceinline__ T rcp_nr(T v) {
  if constexpr (sizeof(T) == 8) {
    T y = __builtin_amdgcn_rcp(v);
#pragma unroll
    for (int i = 0; i < 2; ++i) y = y + y * (T(1) - v * y);
    return y;
  } else {
    const T y = __builtin_amdgcn_rcpf(v);
    return y + y * (T(1) - v * y);
  }
}

template <typename T>
__device__ __forceinline__ T shell_map(const T P0[3], CPtr<T> JT, const T s[3], const T xh[3], T xi[3], T v[3]) {
#pragma unroll
  for (int d = 0; d < 3; ++d) xi[d] = P0[d] + JT[3 * d + 0] * xh[0] + JT[3 * d + 1] * xh[1] + JT[3 * d + 2] * xh[2];
  const T rho = s[0] * xi[0] + s[1] * xi[1] + s[2] * xi[2];
  const T n2 = xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2];
  const T inv = rsqrt_nr(n2);
  const T c3i = rho * inv * inv * inv;
#pragma unroll
  for (int d = 0; d < 3; ++d) v[d] = s[d] * inv - c3i * xi[d];
  return rho * inv;
}

// g = h (I - p q^T / a0) / a0 for a row vector h: with (p, q) = (xi, v) this
// is h DPhi^-1, with (p, q) = (v, xi) it is h DPhi^-T
template <typename T>
__device__ __forceinline__ void shell_pull(const T h[3], const T p[3], const T q[3], T ia0, T g[3]) {
  const T t = (h[0] * p[0] + h[1] * p[1] + h[2] * p[2]) * ia0;
#pragma unroll
  for (int d = 0; d < 3; ++d) g[d] = ia0 * (h[d] - t * q[d]);
}

// Gradient coefficients of a P2 field in xi coordinates (the affine part of
// the map): grad_xi u(q) = sum_a lambda_a(q) H[a], H[a] = sum_b s[a][b] grad lambda_b
template <typename T>
__device__ __forceinline__ void xi_grad_coeffs(const T u[10], CPtr<T> gl, T H[4][3]) {
  T sp[4][3];
  grad_coeffs(u, sp);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int d = 0; d < 3; ++d) H[a][d] = sp[a][0] * gl[3 + d] + sp[a][1] * gl[6 + d] + sp[a][2] * gl[9 + d];
}

template <typename T>
__device__ inline void eps_blended_elem(const T u[3][10], const T mu[10], const T P0[3], CPtr<T> JT, CPtr<T> gl,
                                        T vol, const T s[3], CPtr<T> qtab, int nq, T y[3][10]) {
  // Every gradient is linear in lambda on the affine part of the map: the
  // gradient of u_c in xi coordinates is sum_a lambda_a(q) H[c][a]; the
  // outputs need only Tx[d][a] = sum_q lambda_a(q) (sigma_q DPhi^-T)_d,
  // mapped after the loop by the P2 output rule of p2_elem with
  // sigma[a][b] = Tx[d][a] . grad lambda_b.
  T H[3][4][3];
#pragma unroll
  for (int c = 0; c < 3; ++c) xi_grad_coeffs(u[c], gl, H[c]);
  T Tx[3][4][3];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int r = 0; r < 3; ++r) Tx[d][a][r] = T(0);
  const T vol6 = T(6) * vol;
  for (int q = 0; q < nq; ++q) {
    CPtr<T> Q = qtab + q * kQStride;  // w, bary[4], phi[10]
    const T lam[4] = {Q[1], Q[2], Q[3], Q[4]};
    const T xh[3] = {Q[2], Q[3], Q[4]};
    T xi[3], v[3];
    const T a0 = shell_map(P0, JT, s, xh, xi, v);
    const T ia0 = rcp_nr(a0);
    T gu[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T h[3];
#pragma unroll
      for (int r = 0; r < 3; ++r)
        h[r] = lam[0] * H[c][0][r] + lam[1] * H[c][1][r] + lam[2] * H[c][2][r] + lam[3] * H[c][3][r];
      shell_pull(h, xi, v, ia0, gu[c]);
    }
    T muq = T(0);
#pragma unroll
    for (int i = 0; i < 10; ++i) muq += mu[i] * Q[5 + i];
    const T f = T(2) * muq * Q[0] * (a0 * a0 * a0 * vol6);
    T sg[3][3];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int e = 0; e < 3; ++e) sg[d][e] = f * T(0.5) * (gu[d][e] + gu[e][d]);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      T Sx[3];
      shell_pull(sg[d], v, xi, ia0, Sx);
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int r = 0; r < 3; ++r) Tx[d][a][r] += lam[a] * Sx[r];
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    T sig[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
      for (int b = 1; b < 4; ++b)
        sig[a][b] = Tx[d][a][0] * gl[3 * b + 0] + Tx[d][a][1] * gl[3 * b + 1] + Tx[d][a][2] * gl[3 * b + 2];
      sig[a][0] = -(sig[a][1] + sig[a][2] + sig[a][3]);
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) y[d][b] = T(4) * sig[b][b] - (sig[0][b] + sig[1][b] + sig[2][b] + sig[3][b]);
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      const int b = kEdge[e][0], c = kEdge[e][1];
      y[d][4 + e] = T(4) * (sig[c][b] + sig[b][c]);
    }
  }
}

// Coefficient gradient of the affine epsilon form (A_T linear in the nodal
// mu): with sigma_e = sum_a W_ae E_a as in eps_elem, gy . y = sum_e sigma_e :
// Gam_e where Gam collects the coefficients of gy . Y(sigma), so
// gy . y = sum_{a,e} W_ae (E_a : Gam_e) and gmu_b = sum_{a,e} W(e_b)_ae M_ae.
// Symmetric 3x3 tensors are stored as (xx, yy, zz, xy, xz, yz); S : P counts
// the off-diagonal entries twice.
template <typename T>
__device__ inline void eps_strains(const T u[3][10], CPtr<T> grad, T E[4][6]) {
  T g[3][4][3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    T sp[4][3];
    grad_coeffs(u[c], sp);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int r = 0; r < 3; ++r)
        g[c][a][r] = sp[a][0] * grad[3 * 1 + r] + sp[a][1] * grad[3 * 2 + r] + sp[a][2] * grad[3 * 3 + r];
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    E[a][0] = g[0][a][0];
    E[a][1] = g[1][a][1];
    E[a][2] = g[2][a][2];
    E[a][3] = T(0.5) * (g[0][a][1] + g[1][a][0]);
    E[a][4] = T(0.5) * (g[0][a][2] + g[2][a][0]);
    E[a][5] = T(0.5) * (g[1][a][2] + g[2][a][1]);
  }
}

template <typename T>
__device__ inline void eps_gradmu(const T u[3][10], const T gy[3][10], CPtr<T> grad, T vol, T gmu[10]) {
  T E[4][6];
  eps_strains(u, grad, E);
  // sym(v w^T) of a nodal vector v of gy and a barycentric gradient w, scaled by f, added to G
  auto addsym = [](T G[6], T f, T v0, T v1, T v2, CPtr<T> w) {
    G[0] += f * v0 * w[0];
    G[1] += f * v1 * w[1];
    G[2] += f * v2 * w[2];
    G[3] += f * T(0.5) * (v0 * w[1] + v1 * w[0]);
    G[4] += f * T(0.5) * (v0 * w[2] + v2 * w[0]);
    G[5] += f * T(0.5) * (v1 * w[2] + v2 * w[1]);
  };
  const T fv = T(2) * vol, fe = T(8) * vol;
  T gam[4][6], vt[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    vt[q] = T(0);
#pragma unroll
    for (int e = 0; e < 4; ++e) gam[e][q] = T(0);
  }
  // vertices: gy_b . (fv (4 sigma_b - sum_e sigma_e) grad lambda_b)
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    addsym(gam[b], T(4) * fv, gy[0][b], gy[1][b], gy[2][b], grad + 3 * b);
    addsym(vt, fv, gy[0][b], gy[1][b], gy[2][b], grad + 3 * b);
  }
#pragma unroll
  for (int e = 0; e < 4; ++e)
#pragma unroll
    for (int q = 0; q < 6; ++q) gam[e][q] -= vt[q];
  // edges (b, c): gy_bc . (fe (sigma_c grad lambda_b + sigma_b grad lambda_c))
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    const int b = kEdge[e][0], c = kEdge[e][1];
    addsym(gam[c], fe, gy[0][4 + e], gy[1][4 + e], gy[2][4 + e], grad + 3 * b);
    addsym(gam[b], fe, gy[0][4 + e], gy[1][4 + e], gy[2][4 + e], grad + 3 * c);
  }
  T M[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int e = 0; e < 4; ++e)
      M[a][e] = E[a][0] * gam[e][0] + E[a][1] * gam[e][1] + E[a][2] * gam[e][2] +
                T(2) * (E[a][3] * gam[e][3] + E[a][4] * gam[e][4] + E[a][5] * gam[e][5]);
#pragma unroll
  for (int b = 0; b < 10; ++b) {
    T kb[10], Wb[4][4];
#pragma unroll
    for (int w = 0; w < 10; ++w) kb[w] = w == b ? T(1) : T(0);
    weights_p2(kb, Wb);
    T acc = T(0);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc += Wb[a][e] * M[a][e];
    gmu[b] = acc;
  }
}

// Coefficient gradient of the blended epsilon form: mu_q = sum_b mu_b phi_b(q)
// enters as 2 mu_q w_q |det J| eps(u):eps(v), so
// gmu_b = sum_q phi_b(q) 2 w_q |det J| eps(u_q) : eps(gy_q).
template <typename T>
__device__ inline void eps_blended_gradmu(const T u[3][10], const T gy[3][10], const T P0[3], CPtr<T> JT,
                                          CPtr<T> gl, T vol, const T s[3], CPtr<T> qtab, int nq, T gmu[10]) {
  // eps(u) : eps(gy) = sym(grad u) : grad gy = sum_c (sym(grad u)_c DPhi^-T) . hg_c
  // with hg_c the gradient of gy_c in xi coordinates: only the gradient of u
  // goes through DPhi^-1 (map and coefficients as in eps_blended_elem)
  T Hu[3][4][3], Hg[3][4][3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    xi_grad_coeffs(u[c], gl, Hu[c]);
    xi_grad_coeffs(gy[c], gl, Hg[c]);
  }
#pragma unroll
  for (int i = 0; i < 10; ++i) gmu[i] = T(0);
  const T vol6 = T(6) * vol;
  for (int q = 0; q < nq; ++q) {
    CPtr<T> Q = qtab + q * kQStride;  // w, bary[4], phi[10]
    const T lam[4] = {Q[1], Q[2], Q[3], Q[4]};
    const T xh[3] = {Q[2], Q[3], Q[4]};
    T xi[3], v[3];
    const T a0 = shell_map(P0, JT, s, xh, xi, v);
    const T ia0 = rcp_nr(a0);
    T gu[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T h[3];
#pragma unroll
      for (int r = 0; r < 3; ++r)
        h[r] = lam[0] * Hu[c][0][r] + lam[1] * Hu[c][1][r] + lam[2] * Hu[c][2][r] + lam[3] * Hu[c][3][r];
      shell_pull(h, xi, v, ia0, gu[c]);
    }
    T ee = T(0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T sc[3], px[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) sc[d] = T(0.5) * (gu[c][d] + gu[d][c]);
      shell_pull(sc, v, xi, ia0, px);
#pragma unroll
      for (int r = 0; r < 3; ++r)
        ee += px[r] * (lam[0] * Hg[c][0][r] + lam[1] * Hg[c][1][r] + lam[2] * Hg[c][2][r] + lam[3] * Hg[c][3][r]);
    }
    const T f = T(2) * Q[0] * (a0 * a0 * a0 * vol6) * ee;
#pragma unroll
    for (int i = 0; i < 10; ++i) gmu[i] += f * Q[5 + i];
  }
}

// N1 curl-curl + mass on one affine tet (equation N1), lowest-order
// first-kind Nedelec basis phi_ab = lambda_a g_b - lambda_b g_a (g = grad
// lambda, edges a < b oriented a -> b), alpha and beta nodal P1:
//   curl u = C = sum_e u_e c_e, c_e = 2 g_a x g_b (constant), so the curl
//   part is y_e = |T| mean(alpha) c_e . C;
//   u = sum_p lambda_p U_p with U_a += u_e g_b, U_b -= u_e g_a, and with
//   B_pq = int beta lambda_p lambda_q = |T| (sum beta + beta_p + beta_q) / 120
//   (p != q), |T| (sum beta + 2 beta_p) / 60 (p = q), V_q = sum_p B_pq U_p,
//   the mass part is y_ab = g_b . V_a - g_a . V_b.
template <typename T>
__device__ inline void n1_elem(const T u[6], const T al[4], const T be[4], CPtr<T> g, T vol, T y[6]) {
  T c[6][3], C[3] = {T(0), T(0), T(0)};
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    const int a = kEdge[e][0], b = kEdge[e][1];
    c[e][0] = T(2) * (g[3 * a + 1] * g[3 * b + 2] - g[3 * a + 2] * g[3 * b + 1]);
    c[e][1] = T(2) * (g[3 * a + 2] * g[3 * b + 0] - g[3 * a + 0] * g[3 * b + 2]);
    c[e][2] = T(2) * (g[3 * a + 0] * g[3 * b + 1] - g[3 * a + 1] * g[3 * b + 0]);
#pragma unroll
    for (int d = 0; d < 3; ++d) C[d] += u[e] * c[e][d];
  }
  const T am = T(0.25) * (al[0] + al[1] + al[2] + al[3]) * vol;
#pragma unroll
  for (int e = 0; e < 6; ++e) y[e] = am * (c[e][0] * C[0] + c[e][1] * C[1] + c[e][2] * C[2]);
  T U[4][3];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int d = 0; d < 3; ++d) U[p][d] = T(0);
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    const int a = kEdge[e][0], b = kEdge[e][1];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      U[a][d] += u[e] * g[3 * b + d];
      U[b][d] -= u[e] * g[3 * a + d];
    }
  }
  const T sb = be[0] + be[1] + be[2] + be[3];
  T B[4][4];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q)
      B[p][q] = p == q ? vol * (sb + T(2) * be[p]) * T(1.0 / 60.0) : vol * (sb + be[p] + be[q]) * T(1.0 / 120.0);
  T V[4][3];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int d = 0; d < 3; ++d) V[q][d] = B[0][q] * U[0][d] + B[1][q] * U[1][d] + B[2][q] * U[2][d] + B[3][q] * U[3][d];
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    const int a = kEdge[e][0], b = kEdge[e][1];
    y[e] += g[3 * b + 0] * V[a][0] + g[3 * b + 1] * V[a][1] + g[3 * b + 2] * V[a][2] -
            (g[3 * a + 0] * V[b][0] + g[3 * a + 1] * V[b][1] + g[3 * a + 2] * V[b][2]);
  }
}

// +1 if local edge e (a -> b) of type t runs along its lattice direction (the
// micro-edge direction with first nonzero component positive), else -1
constexpr int n1_edge_sign(int t, int e) {
  int d[3] = {0, 0, 0};
  for (int c = 0; c < 3; ++c) d[c] = kOff[t][kEdge[e][1]][c] - kOff[t][kEdge[e][0]][c];
  return d[0] != 0 ? (d[0] > 0 ? 1 : -1) : d[1] != 0 ? (d[1] > 0 ? 1 : -1) : (d[2] > 0 ? 1 : -1);
}

// LDS barrier without a wait on global memory (buffer-to-LDS loads and
// global stores stay in flight): the fences order LDS accesses only
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}
// wait for this wavefront's vector memory operations (vmcnt(0); LDS counter untouched)
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Buffer loads and stores over one macro block (or one partial-sum block):
// the hardware range check turns an offset past the block into a load of 0
// or a dropped store.
constexpr int kFarOff = 0x7fffff00;  // byte offset past any block (blocks are < 2^31 bytes)
typedef unsigned int U32x2 __attribute__((ext_vector_type(2)));
template <typename T>
__device__ __forceinline__ T buf_ld(__amdgpu_buffer_rsrc_t r, int off) {
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <typename T, int AUX>
__device__ __forceinline__ void buf_st(T v, __amdgpu_buffer_rsrc_t r, int off) {
  if constexpr (sizeof(T) == 8)
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U32x2, v), r, off, 0, AUX);
  else
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, 0, AUX);
}

template <typename T, int KIND, int MAP, int TX, int TY, int TZ>
struct TileCfg {
  static constexpr int RX = 2 * TX + 1, RY = 2 * TY + 1, RZ = 2 * TZ + 1;
  static constexpr int R = RX * RY * RZ;  // lattice points of the box
  // LDS layout of a box row: the TX + 1 even-x points first, the TX odd-x
  // points from slot OO, row pitch RXP.  Lane l of a wavefront works on cube
  // x = l mod TX, so a given local node is read by consecutive lanes from
  // consecutive 8-byte slots (the natural layout would stride by 2 and use
  // half the banks), and the pitch puts the 16 / TX cube rows of a 16-lane
  // group 8 TX bytes apart modulo 128: 2 RXP = TX (mod 16).
  static constexpr int OO = TX + 1;
  static constexpr int RXP = TX == 8 ? 20 : 10;
  static constexpr int RP = RXP * RY * RZ;  // LDS slots per array
  static_assert(TX == 4 || TX == 8, "row pitch chosen for TX = 4 or 8");
  static_assert(RXP >= OO + TX && (2 * RXP - TX) % 16 == 0, "row pitch");
  static constexpr int C = TX * TY * TZ;
  static constexpr bool EPS = KIND == P2V_EPSILON || KIND == P2V_EPSILON_GRADMU || KIND == P2V_EPSILON_DIAG;
  static constexpr int NC = (KIND == P2V_EPSILON || KIND == P2V_EPSILON_DIAG) ? 3 : 1;  // output components
  // diagonal modes: no x is staged, each micro-tet adds its local diagonal
  static constexpr bool DIAG = KIND == P2_LAPLACE_DIAG || KIND == P2_DIVKGRAD_DIAG || KIND == P2V_EPSILON_DIAG;
  // coefficient-gradient modes: x and gy staged (both masked), no coefficient;
  // the output gk is not zeroed on Dirichlet DoFs (boundary values of k act
  // on interior rows)
  static constexpr bool GRADK = KIND == P2_DIVKGRAD_GRADK, GRADMU = KIND == P2V_EPSILON_GRADMU;
  static constexpr bool GRAD = GRADK || GRADMU;
  static constexpr int NCX = GRADMU ? 3 : GRADK ? 1 : NC;   // components of x
  static constexpr int NCI = DIAG ? 1 : GRAD ? 2 * NCX : NC;  // staged input vectors (x, then gy; diagonal: none used)
  static constexpr bool HASK = KIND != P2_LAPLACE && KIND != P2_LAPLACE_DIAG && !GRAD && KIND != P2_STORED_APPLY;
  // N1: edge DoFs with a per-slot orientation sign; two coefficients (alpha,
  // beta) read at the vertex points
  static constexpr bool N1 = KIND == N1_CURLCURL;
  static constexpr int NK = N1 ? 2 : 1;
  // stored-matrix modes: STORE builds the local matrices from k (no x, no
  // output), SAPPLY applies them (x only)
  static constexpr bool STORE = KIND == P2_DIVKGRAD_STORE, SAPPLY = KIND == P2_STORED_APPLY;
  static constexpr bool STORED = STORE || SAPPLY;
  // Scalar kinds: WPG wavefronts per workgroup, wavefront w applying the
  // micro-tet types t = w (mod WPG) to every cube of the box, so the type is
  // a compile-time constant inside each loop (LDS node offsets become
  // instruction immediates, the type's geometry is loaded once into scalar
  // registers).  64-cube boxes use 3 wavefronts (two types each): more
  // workgroups then fit per CU (LDS, not wave slots, becomes the limit),
  // which overlaps more staging round trips -- 12% faster than 6 on the FP64
  // div(k grad) kernel; 128-cube boxes keep 6.
  // (the epsilon element needs 124-235 VGPRs: there 4-wavefront groups, two
  // per CU, beat one 6-wavefront group; wavefronts then take (type, cube)
  // slots with a wave-uniform type)
  static constexpr int WPG = C == 64 ? 3 : 6;
  static constexpr int NTH = EPS ? 256 : 64 * WPG;
  static_assert(C % 64 == 0, "every lane of a wavefront needs a cube: 64 | cubes per tile");
};

// one micro-tet whose 10 local nodes sit at LDS points li[]
// The stored element matrices of one (tile, type): entry e of cube c at
// element e * C + c.  A buffer resource over the block keeps the 55 entry
// offsets as scalar offsets of one per-lane offset, instead of 55 64-bit
// addresses held in vector registers.
struct MatRef {
  __amdgpu_buffer_rsrc_t r;
  int off;  // byte offset of this lane's cube
};
template <typename T>
__device__ __forceinline__ T mat_load(const MatRef &m, int e) {
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(m.r, m.off, e * 8, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(m.r, m.off, e * 4, 0));
}
template <typename T>
__device__ __forceinline__ void mat_store(const MatRef &m, int e, T v) {
  typedef unsigned int U2 __attribute__((ext_vector_type(2)));
  if constexpr (sizeof(T) == 8)
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, v), m.r, m.off, e * 8, 0);
  else
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), m.r, m.off, e * 4, 0);
}

// one micro-tet whose 10 local nodes sit at LDS points li[]: its local
// results go to out[] (out[10 c + v] for component c at node v; N1 uses
// out[4 .. 9] for its edges), added into the accumulator later in a fixed
// order (cube_scatter)
template <typename T, int KIND, int MAP, int R, int t, int CS>
__device__ __forceinline__ void tile_elem(const TileArgs<T> &a, const InstDesc<T> *D, T (*sx)[R], const T *sk,
                                          T *out, const int li[10], int m, int bxc, int byc, int bzc,
                                          const MatRef &me) {
  const TypeGeo<T> *g = D->geo + 6 * m + t;
  if constexpr (KIND == P2V_EPSILON) {
    T u[3][10], mu[10], y[3][10];
#pragma unroll
    for (int v = 0; v < 10; ++v) {
      u[0][v] = sx[0][li[v]];
      u[1][v] = sx[1][li[v]];
      u[2][v] = sx[2][li[v]];
      mu[v] = sk[li[v]];
    }
    if constexpr (MAP == 0) {
      eps_elem(u, mu, cptr(g->grad), *cptr(&g->vol), y);
    } else {
      const __attribute__((address_space(4))) MacroGeo<T> &mg =
          *(const __attribute__((address_space(4))) MacroGeo<T> *)(D->mgeo + m);
      const T bc[3] = {T(bxc + kOff[t][0][0]), T(byc + kOff[t][0][1]), T(bzc + kOff[t][0][2])};
      const T inv_n = T(1) / T(D->n);
      T P0[3];
#pragma unroll
      for (int d = 0; d < 3; ++d)
        P0[d] = mg.v0[d] + (mg.JM[3 * d + 0] * bc[0] + mg.JM[3 * d + 1] * bc[1] + mg.JM[3 * d + 2] * bc[2]) * inv_n;
      const T sv[3] = {mg.s[0], mg.s[1], mg.s[2]};
      eps_blended_elem(u, mu, P0, cptr(g->JT), cptr(g->grad), *cptr(&g->vol), sv, cptr(a.qtab), a.nq, y);
    }
#pragma unroll
    for (int v = 0; v < 10; ++v)
#pragma unroll
      for (int c = 0; c < 3; ++c) out[10 * c + v] = y[c][v];
  } else if constexpr (KIND == P2V_EPSILON_DIAG) {
    // the 30 diagonal entries (A_T)_(v,c),(v,c): the element applied to each
    // unit vector in turn (a runtime loop, so the element code is emitted
    // once), entry (v, c) of the result kept
    T mu[10];
#pragma unroll
    for (int v = 0; v < 10; ++v) mu[v] = sk[li[v]];
#pragma unroll
    for (int e = 0; e < 30; ++e) out[e] = T(0);
    T P0[3] = {T(0), T(0), T(0)}, sv[3] = {T(0), T(0), T(0)};
    if constexpr (MAP != 0) {
      const __attribute__((address_space(4))) MacroGeo<T> &mg =
          *(const __attribute__((address_space(4))) MacroGeo<T> *)(D->mgeo + m);
      const T bc[3] = {T(bxc + kOff[t][0][0]), T(byc + kOff[t][0][1]), T(bzc + kOff[t][0][2])};
      const T inv_n = T(1) / T(D->n);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        P0[d] = mg.v0[d] + (mg.JM[3 * d + 0] * bc[0] + mg.JM[3 * d + 1] * bc[1] + mg.JM[3 * d + 2] * bc[2]) * inv_n;
        sv[d] = mg.s[d];
      }
    }
#pragma unroll 1
    for (int idx = 0; idx < 30; ++idx) {
      T u[3][10], y[3][10];
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int v = 0; v < 10; ++v) u[c][v] = (10 * c + v == idx) ? T(1) : T(0);
      if constexpr (MAP == 0) {
        eps_elem(u, mu, cptr(g->grad), *cptr(&g->vol), y);
      } else {
        eps_blended_elem(u, mu, P0, cptr(g->JT), cptr(g->grad), *cptr(&g->vol), sv, cptr(a.qtab), a.nq, y);
      }
      T dv = T(0);
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int v = 0; v < 10; ++v) dv += u[c][v] * y[c][v];
#pragma unroll
      for (int e = 0; e < 30; ++e) out[e] = e == idx ? dv : out[e];
    }
  } else if constexpr (KIND == P2_DIVKGRAD_Q) {
    T u[10], kv[10], y[10], W[4][4];
#pragma unroll
    for (int v = 0; v < 10; ++v) {
      u[v] = sx[0][li[v]];
      kv[v] = sk[li[v]];
    }
    weights_quad(kv, cptr(a.qtab), a.nq, W);
    p2_elem_w(u, W, cptr(g->Gp), y);
#pragma unroll
    for (int v = 0; v < 10; ++v) out[v] = y[v];
  } else if constexpr (KIND == P2_DIVKGRAD_STORE) {
    // columns A e_v of the local matrix; the upper triangle is stored
    T kv[10], A[10][10];
#pragma unroll
    for (int v = 0; v < 10; ++v) kv[v] = sk[li[v]];
#pragma unroll
    for (int v = 0; v < 10; ++v) {
      T u[10];
#pragma unroll
      for (int w = 0; w < 10; ++w) u[w] = w == v ? T(1) : T(0);
      p2_elem<T, true>(u, kv, cptr(g->Gp), cptr(g->Gs), A[v]);
    }
    int e = 0;
#pragma unroll
    for (int i = 0; i < 10; ++i)
#pragma unroll
      for (int j = i; j < 10; ++j) mat_store<T>(me, (e++) * CS, A[j][i]);
  } else if constexpr (KIND == P2_STORED_APPLY) {
    T u[10], y[10];
#pragma unroll
    for (int v = 0; v < 10; ++v) {
      u[v] = sx[0][li[v]];
      y[v] = T(0);
    }
    int e = 0;
#pragma unroll
    for (int i = 0; i < 10; ++i)
#pragma unroll
      for (int j = i; j < 10; ++j) {
        const T aij = mat_load<T>(me, (e++) * CS);
        y[i] += aij * u[j];
        if (j != i) y[j] += aij * u[i];
      }
#pragma unroll
    for (int v = 0; v < 10; ++v) out[v] = y[v];
  } else if constexpr (KIND == N1_CURLCURL) {
    T u[6], al[4], be[4], y6[6];
#pragma unroll
    for (int e = 0; e < 6; ++e) u[e] = T(n1_edge_sign(t, e)) * sx[0][li[4 + e]];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      al[v] = sk[li[v]];
      be[v] = sk[R + li[v]];
    }
    n1_elem(u, al, be, cptr(g->grad), *cptr(&g->vol), y6);
#pragma unroll
    for (int e = 0; e < 6; ++e) out[4 + e] = T(n1_edge_sign(t, e)) * y6[e];
  } else if constexpr (KIND == P2V_EPSILON_GRADMU) {
    T u[3][10], gv[3][10], gm[10];
#pragma unroll
    for (int v = 0; v < 10; ++v)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        u[c][v] = sx[c][li[v]];
        gv[c][v] = sx[3 + c][li[v]];
      }
    if constexpr (MAP == 0) {
      eps_gradmu(u, gv, cptr(g->grad), *cptr(&g->vol), gm);
    } else {
      const __attribute__((address_space(4))) MacroGeo<T> &mg =
          *(const __attribute__((address_space(4))) MacroGeo<T> *)(D->mgeo + m);
      const T bc[3] = {T(bxc + kOff[t][0][0]), T(byc + kOff[t][0][1]), T(bzc + kOff[t][0][2])};
      const T inv_n = T(1) / T(D->n);
      T P0[3];
#pragma unroll
      for (int d = 0; d < 3; ++d)
        P0[d] = mg.v0[d] + (mg.JM[3 * d + 0] * bc[0] + mg.JM[3 * d + 1] * bc[1] + mg.JM[3 * d + 2] * bc[2]) * inv_n;
      const T sv[3] = {mg.s[0], mg.s[1], mg.s[2]};
      eps_blended_gradmu(u, gv, P0, cptr(g->JT), cptr(g->grad), *cptr(&g->vol), sv, cptr(a.qtab), a.nq, gm);
    }
#pragma unroll
    for (int v = 0; v < 10; ++v) out[v] = gm[v];
  } else if constexpr (KIND == P2_DIVKGRAD_GRADK) {
    T u[10], gv[10], gk[10];
#pragma unroll
    for (int v = 0; v < 10; ++v) {
      u[v] = sx[0][li[v]];
      gv[v] = sx[1][li[v]];
    }
    p2_gradk<T>(u, gv, cptr(g->Gp), gk);
#pragma unroll
    for (int v = 0; v < 10; ++v) out[v] = gk[v];
  } else if constexpr (KIND == P2_LAPLACE_DIAG || KIND == P2_DIVKGRAD_DIAG) {
    constexpr bool HASK = KIND == P2_DIVKGRAD_DIAG;
    T kv[10], d[10];
#pragma unroll
    for (int v = 0; v < 10; ++v) kv[v] = HASK ? sk[li[v]] : T(1);
    p2_diag<T, HASK>(kv, cptr(g->Gp), cptr(g->Gs), d);
#pragma unroll
    for (int v = 0; v < 10; ++v) out[v] = d[v];
  } else {
    constexpr bool HASK = KIND != P2_LAPLACE;
    T u[10], kv[10], y[10];
#pragma unroll
    for (int v = 0; v < 10; ++v) {
      u[v] = sx[0][li[v]];
      kv[v] = HASK ? sk[li[v]] : T(1);
    }
    p2_elem<T, HASK>(u, kv, cptr(g->Gp), cptr(g->Gs), y);
#pragma unroll
    for (int v = 0; v < 10; ++v) out[v] = y[v];
  }
}

// LDS slot of box point (rx, ry, rz) (x-parity split rows, pitch RXP)
constexpr int lds_slot(int rx, int row, int OO, int RXP) { return ((rx & 1) ? OO + (rx >> 1) : (rx >> 1)) + RXP * row; }

// LDS offset of local node v of a type-t micro-tet from its cube's slot
// (P2 lattice: vertex p -> 2p, edge (p, q) -> p + q; the cube's base point
// has even coordinates, so x offset 0 / 2 stays in the even half, 1 maps to
// the odd half)
constexpr int node_off(int t, int v, int RY, int OO, int RXP) {
  int o[3] = {0, 0, 0};
  for (int d = 0; d < 3; ++d)
    o[d] = v < 4 ? 2 * kOff[t][v][d] : kOff[t][kEdge[v - 4][0]][d] + kOff[t][kEdge[v - 4][1]][d];
  return lds_slot(o[0], o[1] + RY * o[2], OO, RXP);
}

// micro-tet of type t in cube c of the box (x fastest): its local results
// into out[] and its cube's LDS slot into cbo; false if it does not exist
template <typename T, int KIND, int MAP, int TX, int TY, int TZ, int t, int R>
__device__ __forceinline__ bool cube_elem(const TileArgs<T> &a, const InstDesc<T> *D, T (*sx)[R], const T *sk,
                                          T *out, int &cbo, int m, int bx0, int by0, int bz0, int c, int tw) {
  using Cfg = TileCfg<T, KIND, MAP, TX, TY, TZ>;
  constexpr int RY = Cfg::RY, OO = Cfg::OO, RXP = Cfg::RXP;
  const int cx = c % TX, cy = (c / TX) % TY, cz = c / (TX * TY);
  const bool exists = c < Cfg::C && bx0 + by0 + bz0 + cx + cy + cz <= D->n - kLim[t];
  // scalar P2 applies compute every lane's micro-tet (its nodes lie in the
  // staged box either way, and a missing one is not added): no branch around
  // the element code and no defined results needed on a skipped path.  Their
  // cube index is always below C: the lane (64-cube boxes, three wavefronts)
  // or lane + 64 r (128-cube boxes, six wavefronts).
  constexpr bool ALWAYS = KIND == P2_LAPLACE || KIND == P2_DIVKGRAD;
  if (!ALWAYS && !exists) return false;
  const int cb = cx + RXP * (2 * cy + RY * 2 * cz);
  cbo = cb;
  int li[10];
#pragma unroll
  for (int v = 0; v < 10; ++v) li[v] = cb + node_off(t, v, RY, OO, RXP);
  // stored-matrix modes: the element's 55 entries at entry e * C, e = 0..54
  MatRef me{};
  if constexpr (Cfg::STORED) {
    me.r = __builtin_amdgcn_make_buffer_rsrc(a.mat + (static_cast<int64_t>(tw) * 6 + t) * kStoredEntries * Cfg::C, 0,
                                             kStoredEntries * Cfg::C * static_cast<int>(sizeof(T)), 0x00020000);
    me.off = c * static_cast<int>(sizeof(T));
  }
  tile_elem<T, KIND, MAP, R, t, Cfg::C>(a, D, sx, sk, out, li, m, bx0 + cx, by0 + cy, bz0 + cz, me);
  return exists;
}

// add a micro-tet's local results (cube_elem) into the LDS accumulator
template <typename T, int KIND, int MAP, int TX, int TY, int TZ, int t, int R>
__device__ __forceinline__ void cube_scatter(double (*sy)[R], int cb, const T *out) {
  using Cfg = TileCfg<T, KIND, MAP, TX, TY, TZ>;
  constexpr int RY = Cfg::RY, OO = Cfg::OO, RXP = Cfg::RXP;
  if constexpr (KIND == N1_CURLCURL) {
#pragma unroll
    for (int e = 0; e < 6; ++e) atomicAdd(&sy[0][cb + node_off(t, 4 + e, RY, OO, RXP)], double(out[4 + e]));
  } else {
    constexpr int NCO = (KIND == P2V_EPSILON || KIND == P2V_EPSILON_DIAG) ? 3 : 1;
#pragma unroll
    for (int c = 0; c < NCO; ++c)
#pragma unroll
      for (int v = 0; v < 10; ++v) atomicAdd(&sy[c][cb + node_off(t, v, RY, OO, RXP)], double(out[10 * c + v]));
  }
}

// one round of micro-tets of type t for wavefront w: the local results into
// registers, then NW barrier phases, this wavefront adding its results into
// the accumulator in phase w.  Each type's results stay inside its own branch
// (a merge after a switch over the types costs ~50 registers in the vector
// kinds).  Every wavefront passes NW barriers whatever its type.
template <typename T, int KIND, int MAP, int TX, int TY, int TZ, int t, int R>
__device__ __forceinline__ void cube_apply(const TileArgs<T> &a, const InstDesc<T> *D, T (*sx)[R], const T *sk,
                                           double (*sy)[R], int m, int bx0, int by0, int bz0, int c, int tw, int w,
                                           bool first) {
  using Cfg = TileCfg<T, KIND, MAP, TX, TY, TZ>;
  constexpr int NOUT = Cfg::NC == 3 ? 30 : 10, NW = Cfg::NTH / 64;
  T out[NOUT];
  int cb = 0;
  const bool valid = cube_elem<T, KIND, MAP, TX, TY, TZ, t, R>(a, D, sx, sk, out, cb, m, bx0, by0, bz0, c, tw);
  if constexpr (!Cfg::STORE) {
#pragma unroll
    for (int p = 0; p < NW; ++p) {
      // (the first round's first phase needs no barrier: the staging barrier
      // came before, and the other wavefronts' work reads only x and k)
      if (p > 0 || !first) lds_barrier();
      if (p == w && valid) cube_scatter<T, KIND, MAP, TX, TY, TZ, t, R>(sy, cb, out);
    }
  }
}

// One workgroup per tile.  Workgroup ids are dispatched round-robin over the
// 8 XCDs; the id -> tile map below is a bijection that gives every XCD a
// contiguous run of the (spatially ordered) tile list, so neighbouring boxes
// -- which share halo inputs and seam outputs -- meet in the same L2.
template <typename T, int KIND, int MAP, int TX, int TY, int TZ>
__global__ __launch_bounds__((TileCfg<T, KIND, MAP, TX, TY, TZ>::NTH)) void k_tile(TileArgs<T> a) {
  using Cfg = TileCfg<T, KIND, MAP, TX, TY, TZ>;
  constexpr int RX = Cfg::RX, RY = Cfg::RY, R = Cfg::R, NC = Cfg::NC, NCI = Cfg::NCI, NTH = Cfg::NTH;
  constexpr int OO = Cfg::OO, RXP = Cfg::RXP, RP = Cfg::RP;
  constexpr bool HASK = Cfg::HASK;
  __shared__ T sx[NCI][RP];
  // the element results are accumulated in FP64 in both precisions: FP64
  // LDS atomics run at full speed on gfx950 where FP32 ones stall the LDS
  // pipeline, and the partial sums of a point keep 53-bit mantissas
  __shared__ double sy[NC][RP];
  __shared__ T sk[HASK ? Cfg::NK * RP : 1];
  __shared__ int8_t ssg[Cfg::N1 ? RP : 1];  // N1: orientation sign of each box point

  const int tid = threadIdx.x;
  const int nxcd = 8;
  const int q = a.ntiles / nxcd, rem = a.ntiles % nxcd;
  const int x8 = blockIdx.x % nxcd;
  const int ti = x8 * q + (x8 < rem ? x8 : rem) + static_cast<int>(blockIdx.x) / nxcd;
  const int4 tl = a.tiles[ti];
  const InstDesc<T> *D = a.inst + tl.x;
  if (a.active != nullptr && a.active[tl.x] == 0) return;
  const int m = tl.y;
  const int bx0 = tl.z & 1023, by0 = (tl.z >> 10) & 1023, bz0 = (tl.z >> 20) & 1023;
  const int N = D->N;
  const int64_t nl = D->n_local;
  const uint32_t bnd = D->dirichlet ? *cptr(D->bnd + m) : 0u;
  const int64_t base = D->off + static_cast<int64_t>(m) * D->L;

  // 0. the box's lattice rows (qj, qk): {offset in the macro block of the
  // row's first box point (qi = 2 bx0), bits}: bits 0 .. RX-1 mark the box
  // points whose x is staged (inside the macro and not a Dirichlet DoF), bits
  // 17 .. 21 hold the number of the row's box points inside the macro (khi + 1;
  // 0 for a row outside it), bit 22 is set for a row outside the macro and bit
  // 23 for a row this box owns in y and z (write-back).  A point's Dirichlet
  // test by its face pattern is folded into the row: within a row only the two
  // end points can differ from the rest.
  static_assert(RX <= 17, "the row masks hold at most 17 points");
  // Points of the box per thread (staging and write-back).  For 9-point rows
  // (TX = 4) a wavefront takes 7 whole rows per step, lane l point l mod 9 of
  // row l / 9 (lane 63 idle): a thread's x offset and LDS slot are then fixed
  // and its row advances by a constant, so the per-point index arithmetic
  // becomes immediate offsets.  Otherwise thread t takes points t + NTH p.
  constexpr int NROWS = RY * Cfg::RZ;
  constexpr bool LANEMAP = RX == 9;
  constexpr int RPI = LANEMAP ? 7 * (NTH / 64) : 1;  // rows per step of the lane map
  constexpr int PF = LANEMAP ? (NROWS + RPI - 1) / RPI : (R + NTH - 1) / NTH;
  constexpr int NSROW = LANEMAP ? PF * RPI : NROWS;  // row table padded to whole steps
  const int lane63 = tid & 63, lq = lane63 < 63 ? lane63 / 9 : 0;
  const int lrow = LANEMAP ? (tid >> 6) * 7 + lq : 0;
  const int lx = LANEMAP ? (lane63 < 63 ? lane63 - 9 * lq : 16) : 0;  // 16: no point
  // point p of this thread: its row and x, and whether it is a box point
  auto point = [&](int p, int &row, int &rx) -> bool {
    if constexpr (LANEMAP) {
      row = lrow + RPI * p;
      rx = lx;
      return lx < RX && ((p + 1) * RPI <= NROWS || row < NROWS);
    } else {
      const int r = tid + p * NTH;
      const int rc = r < R ? r : 0;
      row = rc / RX;
      rx = rc - row * RX;
      return r < R;
    }
  };
  __shared__ int2 srow[NSROW];
  for (int row = tid; row < NSROW; row += NTH) {
    if (row >= NROWS) {
      srow[row] = make_int2(0, 1 << 22);  // padding: a row outside the macro
      continue;
    }
    const int ry = row % RY, rz = row / RY;
    const int qj = 2 * by0 + ry, qk = 2 * bz0 + rz;
    const int lim = N - qj - qk, L = lim - 2 * bx0;
    const bool empty = L < 0;
    const int khi = empty ? 0 : min(L, 2 * TX);
    const bool limin = !empty && L <= 2 * TX;
    const int rowzp = ((qj == 0) << 2) | ((qk == 0) << 3);
    uint32_t xmask = empty ? 0u : (2u << khi) - 1u;
    if (!empty) {
      if ((bnd >> rowzp) & 1u) xmask = 0u;
      if (bx0 == 0 && ((bnd >> (rowzp | 2 | (lim == 0 ? 1 : 0))) & 1u)) xmask &= ~1u;
      if (limin && ((bnd >> (rowzp | 1 | (lim == 0 ? 2 : 0))) & 1u)) xmask &= ~(1u << khi);
    }
    const bool ey = (ry & 1) || ((ry > 0 || by0 == 0) && ry < 2 * TY);
    const bool ez = (rz & 1) || ((rz > 0 || bz0 == 0) && rz < 2 * TZ);
    srow[row] = make_int2(empty ? 0 : row_base(qj, qk, N) + 2 * bx0,
                          static_cast<int>(xmask | (uint32_t(empty ? 0 : khi + 1) << 17) | (uint32_t(empty) << 22) |
                                           (uint32_t(ey && ez) << 23)));
  }
  __syncthreads();

  // 1. stage the box: x with Dirichlet DoFs zeroed, and the coefficient.
  // Buffer loads over the macro block: a point outside the macro (or a
  // Dirichlet DoF of x) gets an offset past the block and loads 0, so there
  // are no branches and all of a thread's loads are in flight together (one
  // memory latency per tile instead of one per point).
  const int nbytes = D->L * static_cast<int>(sizeof(T));
  __amdgpu_buffer_rsrc_t rsx[NCI], rsk[Cfg::NK];
#pragma unroll
  for (int c = 0; c < NCI; ++c)
    rsx[c] = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<T *>((c < Cfg::NCX ? a.x + c * nl : a.x2 + (c - Cfg::NCX) * nl) + base), 0, nbytes, 0x00020000);
#pragma unroll
  for (int c = 0; c < Cfg::NK; ++c)
    rsk[c] = __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(HASK ? a.k + c * nl + base : a.x + base), 0, nbytes,
                                               0x00020000);
  // N1: the per-slot orientation signs (bytes) over the same block
  const __amdgpu_buffer_rsrc_t rss = __builtin_amdgcn_make_buffer_rsrc(
      Cfg::N1 ? const_cast<int8_t *>(D->sign + base) : nullptr, 0, Cfg::N1 ? D->L : 0, 0x00020000);
  constexpr int NK = Cfg::NK;
  T xv[PF][NCI], kv[PF][NK];
  int sgv[PF];
#pragma unroll
  for (int p = 0; p < PF; ++p) {
    int row, rx;
    const bool in = point(p, row, rx);
    const int2 rw = srow[row];
    const uint32_t bits = static_cast<uint32_t>(rw.y);
    // (with the lane map, the padding rows and the idle lane 63, x = 16, fail
    // both tests by themselves: no point count or x bit reaches them)
    const bool kin = (LANEMAP || in) && rx < static_cast<int>((bits >> 17) & 31u);
    const bool xin = (LANEMAP || in) && ((bits >> rx) & 1u);
    const int off = rw.x + rx;
#pragma unroll
    for (int c = 0; c < NCI; ++c)
      xv[p][c] = (Cfg::DIAG || Cfg::STORE) ? T(0) : buf_ld<T>(rsx[c], xin ? off * static_cast<int>(sizeof(T)) : kFarOff);
    sgv[p] = 0;
    if constexpr (Cfg::N1) {
      // x in the lattice orientation; alpha and beta live at the vertex points
      sgv[p] = static_cast<int8_t>(__builtin_amdgcn_raw_buffer_load_b8(rss, kin ? off : kFarOff, 0, 0));
      xv[p][0] *= T(sgv[p]);
      const int ry = row % RY, rz = row / RY;
      const bool vert = kin && !(rx & 1) && !(ry & 1) && !(rz & 1);
#pragma unroll
      for (int c = 0; c < NK; ++c) kv[p][c] = buf_ld<T>(rsk[c], vert ? off * static_cast<int>(sizeof(T)) : kFarOff);
    } else {
#pragma unroll
      for (int c = 0; c < NK; ++c)
        kv[p][c] = HASK ? buf_ld<T>(rsk[c], kin ? off * static_cast<int>(sizeof(T)) : kFarOff) : T(0);
    }
  }
#pragma unroll
  for (int p = 0; p < PF; ++p) {
    int row, rx;
    if (point(p, row, rx)) {
      const int sl = lds_slot(rx, row, OO, RXP);
#pragma unroll
      for (int c = 0; c < NCI; ++c) sx[c][sl] = xv[p][c];
#pragma unroll
      for (int c = 0; c < NC; ++c) sy[c][sl] = 0.0;
      if (HASK) {
#pragma unroll
        for (int c = 0; c < NK; ++c) sk[c * RP + sl] = kv[p][c];
      }
      if constexpr (Cfg::N1) ssg[sl] = static_cast<int8_t>(sgv[p]);
    }
  }
  __syncthreads();

  // 2. micro-tets, in two rounds.  Scalar kinds: wavefront w applies type w
  // (6 wavefronts: to cubes lane and lane + 64) or types w and w + 3 (3
  // wavefronts), so the type is a compile-time constant inside each body (LDS
  // node offsets become instruction immediates, the type's geometry is loaded
  // once into scalar registers).  Epsilon: slot e = tid + NTH r -> (type e / C,
  // cube e % C), with 64 | C the type is wave-uniform.  Each round, every
  // wavefront first computes its micro-tets' results into registers; then
  // the wavefronts add them into the accumulator one after another, in
  // wavefront order, between barriers.  Every point therefore receives its
  // contributions in the same order on every run: results are reproducible
  // bit for bit (an LDS atomic of one wavefront touches distinct points in
  // its lanes, and one wavefront's atomics are applied in program order).
  {
    constexpr int NW = NTH / 64, C = Cfg::C;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      int t, c;
      if constexpr (Cfg::EPS) {
        const int e = tid + NTH * r;
        t = __builtin_amdgcn_readfirstlane(e / C);
        c = e - t * C;
      } else if constexpr (Cfg::WPG == 3) {
        t = w + 3 * r;
        c = lane;
      } else {
        t = w;
        c = lane + 64 * r;
      }
      switch (t) {
        case 0: cube_apply<T, KIND, MAP, TX, TY, TZ, 0, RP>(a, D, sx, sk, sy, m, bx0, by0, bz0, c, tl.w, w, r == 0); break;
        case 1: cube_apply<T, KIND, MAP, TX, TY, TZ, 1, RP>(a, D, sx, sk, sy, m, bx0, by0, bz0, c, tl.w, w, r == 0); break;
        case 2: cube_apply<T, KIND, MAP, TX, TY, TZ, 2, RP>(a, D, sx, sk, sy, m, bx0, by0, bz0, c, tl.w, w, r == 0); break;
        case 3: cube_apply<T, KIND, MAP, TX, TY, TZ, 3, RP>(a, D, sx, sk, sy, m, bx0, by0, bz0, c, tl.w, w, r == 0); break;
        case 4: cube_apply<T, KIND, MAP, TX, TY, TZ, 4, RP>(a, D, sx, sk, sy, m, bx0, by0, bz0, c, tl.w, w, r == 0); break;
        case 5: cube_apply<T, KIND, MAP, TX, TY, TZ, 5, RP>(a, D, sx, sk, sy, m, bx0, by0, bz0, c, tl.w, w, r == 0); break;
        default:  // no micro-tets this round (vector kinds, round 1): the phases only
          if constexpr (!Cfg::STORE) {
#pragma unroll
            for (int p = 0; p < NW; ++p)
              if (p > 0 || r != 0) lds_barrier();
          }
          break;
      }
    }
  }
  if constexpr (Cfg::STORE) return;  // the matrices are the output
  __syncthreads();

  // 3. write back: points of this box alone go to y (Dirichlet DoFs as 0),
  // points of shared box faces to this tile's partials
  // [component][box point], through buffer resources over the macro block
  // and the tile's partial block.
  {
    __amdgpu_buffer_rsrc_t rsy[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c)
      rsy[c] = __builtin_amdgcn_make_buffer_rsrc(a.y + base + c * nl, 0, nbytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t rsp = __builtin_amdgcn_make_buffer_rsrc(
        (a.partial ? a.partial : D->partial) + static_cast<int64_t>(tl.w) * NC * R, 0,
        NC * R * static_cast<int>(sizeof(T)), 0x00020000);
    // (unrolled only for the lane map, where it turns the row steps into immediate offsets)
    constexpr int WB_UNROLL = LANEMAP ? PF : 1;
#pragma unroll WB_UNROLL
    for (int p = 0; p < PF; ++p) {
      int row, rx;
      const bool in = point(p, row, rx);
      const int r = row * RX + rx;
      const int2 rw = srow[row];
      const uint32_t bits = static_cast<uint32_t>(rw.y);
      const bool valid = (LANEMAP || in) && rx < static_cast<int>((bits >> 17) & 31u);
      const bool excl = ((bits >> 23) & 1u) && ((rx & 1) || ((rx > 0 || bx0 == 0) && rx < 2 * TX));
      // a point inside the macro whose x bit is clear is a Dirichlet DoF
      const bool dir = !Cfg::GRAD && !((bits >> rx) & 1u);
      const int sl = lds_slot(rx, row, OO, RXP);
      // N1: back to the global orientation (partials too, so that the gather
      // adds values of one orientation)
      const T osg = Cfg::N1 ? T(ssg[sl]) : T(1);
      // plain stores for y too: with the non-temporal policy the kernel's
      // measured HBM writes were 43.4 instead of 31.9 MB per launch (FP64 cube
      // level 6), at the same kernel time
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const T v = osg * T(sy[c][sl]);
        if (valid && excl)
          buf_st<T, 0>(dir ? T(0) : v, rsy[c], (rw.x + rx) * static_cast<int>(sizeof(T)));
        else if (valid)
          buf_st<T, 0>(v, rsp, (c * R + r) * static_cast<int>(sizeof(T)));
      }
    }
  }
}

// Seam reduction.  A lattice point q lies on a face shared by two boxes in
// dimension d when q_d is a positive multiple of 2 T_d; then the boxes at
// q_d / 2 - T_d (q on its upper face) and q_d / 2 (lower face) both hold a
// partial for it, otherwise the one box at T_d floor(q_d / (2 T_d)).  Of the
// up to 8 candidate boxes those that exist (bx + by + bz <= n - 1) each wrote
// their partial; they are added in a fixed order (z, y, x; lower first).
template <int TX, int TY, int TZ>
__device__ __forceinline__ bool is_seam(int qx, int qy, int qz) {
  return (qx > 0 && qx % (2 * TX) == 0) || (qy > 0 && qy % (2 * TY) == 0) || (qz > 0 && qz % (2 * TZ) == 0);
}

// Macro m's partial sums form one block of tpm NC R values, below 10^9 bytes
// at the largest level, so a candidate is addressed by the block's 64-bit base
// (uniform over a seam work entry) and a 32-bit byte offset.
// macro-local slot of a packed lattice point qx | qy << 10 | qz << 20
__device__ __forceinline__ int seam_slot(int pk, int N) { return row_base((pk >> 10) & 1023, pk >> 20, N) + (pk & 1023); }

template <typename T, int NC, int TX, int TY, int TZ>
__device__ __forceinline__ GPtr<const char> partial_block(const SeamInst<T> &a, const T *ovr, int m) {
  constexpr int R = (2 * TX + 1) * (2 * TY + 1) * (2 * TZ + 1);
  return (GPtr<const char>)gptr((ovr ? ovr : a.partial) + static_cast<int64_t>(m) * a.tpm * NC * R);
}

template <typename T, int NC, int TX, int TY, int TZ, typename RS>
__device__ __forceinline__ void seam_sum(const SeamInst<T> &a, RS rs, GPtr<const char> pm, int qx, int qy, int qz,
                                         T acc[NC]) {
  constexpr int RX = 2 * TX + 1, RY = 2 * TY + 1, R = RX * RY * (2 * TZ + 1);
  auto lower = [](int q, int t) { return (q > 0 && q % (2 * t) == 0) ? q / 2 - t : t * (q / (2 * t)); };
  const int x0 = lower(qx, TX), y0 = lower(qy, TY), z0 = lower(qz, TZ);
  const bool fx = qx > 0 && qx % (2 * TX) == 0, fy = qy > 0 && qy % (2 * TY) == 0, fz = qz > 0 && qz % (2 * TZ) == 0;
  // a candidate's loads are issued only where it exists (a wavefront of face
  // points skips the candidates across the other two faces), and none of the
  // loads is used before all are issued, so they are in flight together; a
  // missing candidate adds +0, which leaves the sum (started at +0) unchanged.
  // Candidate e = (ix, iy, iz) is the box (x0 + ix TX, y0 + iy TY, z0 + iz TZ)
  // in tile row (iy, iz): the up to 4 row lookups come first (entry 0 for a
  // row without a candidate box), so they are in flight together; within a
  // row the tile id advances by ix, and the box-local point index falls by
  // 2 TX ix + 2 TY RX iy + 2 TZ RX RY iz.
  const int s0 = x0 + y0 + z0;
  const int rbase = (z0 / TZ) * a.nby + y0 / TY;
  const uint32_t r0 = static_cast<uint32_t>((qx - 2 * x0) + RX * ((qy - 2 * y0) + RY * (qz - 2 * z0)));
  int rowt[4];
  bool rowok[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int iy = j & 1, iz = j >> 1;
    rowok[j] = (!iy || fy) && (!iz || fz) && s0 + iy * TY + iz * TZ <= a.n - 1;
    rowt[j] = rs[rowok[j] ? rbase + iz * a.nby + iy : 0] + x0 / TX;
  }
  uint32_t boff[8];
  bool ok[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int ix = e & 1, iy = (e >> 1) & 1, iz = e >> 2;
    ok[e] = rowok[iy + 2 * iz] && (!ix || fx) && s0 + ix * TX + iy * TY + iz * TZ <= a.n - 1;
    const uint32_t tile = static_cast<uint32_t>(rowt[iy + 2 * iz] + ix);
    const uint32_t r = r0 - static_cast<uint32_t>(2 * TX * ix + 2 * TY * RX * iy + 2 * TZ * RX * RY * iz);
    boff[e] = (tile * (NC * R) + r) * static_cast<uint32_t>(sizeof(T));
  }
  T v[8][NC];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
#pragma unroll
    for (int c = 0; c < NC; ++c) v[e][c] = T(0);
    if (ok[e]) {
#pragma unroll
      for (int c = 0; c < NC; ++c)
        v[e][c] = *(GPtr<const T>)(pm + (boff[e] + static_cast<uint32_t>(c * R * sizeof(T))));
    }
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    T s = T(0);
#pragma unroll
    for (int e = 0; e < 8; ++e) s += v[e][c];
    acc[c] = s;
  }
}

// Work entries: (instance, macro, first seam point, 0) reduce up to 256 PPT
// seam points of one macro (PPT set by how the work list was chunked);
// (instance, first member, end member, 1) reduce whole interface groups, one
// thread per member (at most 256 members).  The tile-row
// starts of the instance are staged in dynamic LDS (`rows_lds` entries; a
// larger table is read from global memory).  At most 96 VGPRs (5 waves per
// SIMD): a launch of up to 1280 work entries is then resident at once.
template <typename T, int NC, int PPT, int TX, int TY, int TZ>
__global__ __launch_bounds__(256, 5) void k_seam(const SeamInst<T> *__restrict__ insts,
                                                 const int4 *__restrict__ work, T *__restrict__ y,
                                                 const uint8_t *__restrict__ active, int flags, int rows_lds,
                                                 const T *__restrict__ partial) {
  const bool local = flags & kSeamLocal;
  extern __shared__ int srs[];
  __shared__ T sv[NC][256];
  __shared__ uint8_t sd[256];
  const int4 w = work[blockIdx.x];
  if (active != nullptr && active[w.x] == 0) return;
  const SeamInst<T> &a = insts[w.x];
  const int t = threadIdx.x;
  const bool grp = w.w == 1;
  // this thread's first loads, issued before the row-table staging
  int pks[PPT];
  bool mine = false;
  int pl = 0, m = 0;  // threads past the entry's end keep point 0 of macro 0
  int64_t slot = 0;
  if (!grp) {
    m = w.y;
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
      const int p = w.z + t + 256 * u;
      pks[u] = p < a.npts ? gptr(a.pts)[p] : -1;
    }
  } else {
    const int q = w.y + t;
    mine = q < w.z;
    pks[0] = 0;
    if (mine) {
      const int64_t pos = gptr(a.gpos)[q];
      slot = gptr(a.gidx)[q];
      pl = gptr(a.gpl)[q];
      m = static_cast<int>(pos >> 32);
      pks[0] = static_cast<int>(pos & 0xffffffff);
    }
  }
  const int nrows = ((a.n + TZ - 1) / TZ) * a.nby;
  const bool in_lds = nrows <= rows_lds;
  if (in_lds)
    for (int e = t; e < nrows; e += 256) srs[e] = gptr(a.rowstart)[e];
  __syncthreads();
  T *yi = y + a.yoff;
  // the rest once with the row table in LDS, once reading it from global memory
  auto body = [&](auto rs) {
    if (!grp) {
      // seam points of macro m (PPT per thread, 256 apart); points with copies
      // in other macros are left to their interface group (unless a
      // macro-local result is asked for)
      // every point's loads first, then the stores (the compiler cannot move a
      // load of one point above the store of another: y and the partials may alias)
      const uint32_t bm = a.dirichlet && !(flags & kSeamKeepBoundary) ? *cptr(a.bnd + m) : 0u;
      const uint32_t sh = local ? 0u : *cptr(a.shared + m);
      const GPtr<const char> pmw = partial_block<T, NC, TX, TY, TZ>(a, partial, w.y);
      T acc[PPT][NC];
      bool wr[PPT], dz[PPT];
#pragma unroll
      for (int u = 0; u < PPT; ++u) {
        const int pk = pks[u] < 0 ? 0 : pks[u];
        const int qx = pk & 1023, qy = (pk >> 10) & 1023, qz = pk >> 20;
        const int z = zero_pattern(qx, qy, qz, a.N);
        wr[u] = pks[u] >= 0 && !((sh >> z) & 1u);
        dz[u] = (bm >> z) & 1u;
        seam_sum<T, NC, TX, TY, TZ>(a, rs, pmw, qx, qy, qz, acc[u]);
      }
#pragma unroll
      for (int u = 0; u < PPT; ++u)
        if (wr[u])
#pragma unroll
          for (int c = 0; c < NC; ++c)
            yi[static_cast<int64_t>(m) * a.L + seam_slot(pks[u], a.N) + c * a.n_local] = dz[u] ? T(0) : acc[u][c];
      return;
    }
    const int pk = pks[0];
    const int qx = pk & 1023, qy = (pk >> 10) & 1023, qz = pk >> 20;
    const int z = zero_pattern(qx, qy, qz, a.N);
    const bool dir = a.dirichlet && !(flags & kSeamKeepBoundary) && ((gptr(a.bnd)[m] >> z) & 1u);
    // interface groups: each member's macro-local value (seam sum or the tile
    // kernel's store) goes to LDS; every member then adds its group's values in
    // ascending member order, so all copies receive the same sum
    if (mine) {
      T v[NC];
      if (is_seam<TX, TY, TZ>(qx, qy, qz)) {
        seam_sum<T, NC, TX, TY, TZ>(a, rs, partial_block<T, NC, TX, TY, TZ>(a, partial, m), qx, qy, qz, v);
      } else {
#pragma unroll
        for (int c = 0; c < NC; ++c) v[c] = yi[slot + c * a.n_local];
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) sv[c][t] = v[c];
      sd[t] = dir;
    }
    __syncthreads();
    if (!mine) return;
    const int len = pl & 0xffff, h = t - (pl >> 16);
    T sum[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) sum[c] = T(0);
    bool gdir = false;
    for (int i = h; i < h + len; ++i) {
#pragma unroll
      for (int c = 0; c < NC; ++c) sum[c] += sv[c][i];
      gdir = gdir || sd[i];
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) yi[slot + c * a.n_local] = gdir ? T(0) : sum[c];
  };
  if (in_lds)
    body((LPtr<int>)srs);
  else
    body(gptr(a.rowstart));
}

// ---------------------------------------------------------------------------
// Marching element kernel for the scalar P2 applies (P2_LAPLACE, P2_DIVKGRAD).
//
// A tile here is a column segment of S sub-boxes of 4 x 4 x 4 micro-cubes
// stacked in z (the cubes loop of section "Cubes Loop Strategy", marched
// along z).  The launch is persistent: each workgroup walks its share of the
// segments sub-box by sub-box and
//   - stages the next sub-box's x (Dirichlet DoFs as 0) and coefficient
//     straight from HBM into a second LDS buffer with buffer-to-LDS loads
//     (no registers held) while it applies the current one, so the load
//     latency of one sub-box hides behind the element work of the previous;
//   - carries the partial sums of the face shared by two sub-boxes of a
//     segment in LDS: that face is written once, complete, by the upper
//     sub-box, never through HBM;
//   - writes the points of the segment's own faces shared with neighbouring
//     segments as partial sums, in the segment-box layout the seam reduction
//     reads (the seam reduction treats a segment as one tall box).
// Per sub-box: the loads of the next sub-box are issued, the micro-tets are
// applied (wavefront w: types w and w + 3, a lane per cube, LDS atomics into
// the accumulator), then the sub-box is written back, the accumulator is
// cleared (keeping the carried face), and the tables of the sub-box after
// next are built.  Three LDS barriers; the only wait on global memory follows
// the element work, for the loads issued before it (the write-back's stores
// drain during the next sub-box).

template <typename T, int KIND, int S>
struct MarchCfg {
  static constexpr int TX = 4, TY = 4, TZS = 4;     // sub-box, micro-cubes
  static constexpr int RX = 9, RY = 9, RZ = 9;      // sub-box lattice points
  static constexpr int OO = TX + 1, RXP = 10;       // LDS row: even points, odd points, pitch (as TileCfg)
  static constexpr int ROWS = RY * RZ;
  static constexpr int RP = RXP * ROWS;             // LDS slots of one staged array
  static constexpr int PLANE = RXP * RY;            // LDS slots of one lattice plane
  static constexpr int DW = sizeof(T) / 4;          // dwords per value
  // each staged array is padded to whole 64-dword loads, so that every
  // buffer-to-LDS load belongs to one array (its buffer descriptor is uniform)
  static constexpr int RPA = ((RP * DW + 63) / 64) * 64 / DW;
  static constexpr int IPA = RPA * DW / 64;         // loads per array per sub-box
  static constexpr bool HASK = KIND == P2_DIVKGRAD;
  static constexpr int NA = HASK ? 2 : 1;
  static constexpr int NINS = NA * IPA;
  static constexpr int WPG = 3, NTH = 64 * WPG;
  static constexpr int IPW = (NINS + WPG - 1) / WPG;  // loads per wavefront
  static constexpr int TZ = TZS * S;                 // segment height in cubes
  static constexpr int RSEG = RX * RY * (2 * TZ + 1);  // points of the segment box (partial layout)
};

// one sub-box of the march: segment (tile index), sub-box in the segment
struct MarchItem {
  int seg, sub;
};

// descriptors read through the constant address space (scalar loads)
template <typename T>
using CDesc = const __attribute__((address_space(4))) InstDesc<T>;
// tile record i of a list, read through the constant address space
__device__ __forceinline__ int4 tile_rec(const int4 *tiles, int i) {
  const CPtr<int> q = cptr(reinterpret_cast<const int *>(tiles)) + 4 * i;
  return make_int4(q[0], q[1], q[2], q[3]);
}
// row table entry (.x, .y) from LDS as one 64-bit read
__device__ __forceinline__ int2 row_rec(LPtr<uint64_t> t, int row) {
  const uint64_t v = t[row];
  return make_int2(static_cast<int>(static_cast<uint32_t>(v)), static_cast<int>(static_cast<uint32_t>(v >> 32)));
}

// Row table entry of a sub-box, one per lattice row (ry, rz):
//   .x = macro-block index of the row's point at rx = 0
//   .y = bits 0-8: rx whose x is staged (inside the macro, not a Dirichlet
//        DoF); bits 9-17: rx inside the macro (coefficient staged, point
//        written back); bit 18: the row's last macro point qi = lim lies in the
//        box; 19: qj = 0; 20: qk = 0; 21: the row's points belong to this
//        segment in y and z (write-back); bits 24-28: largest rx inside the macro
template <typename T, int KIND, int S>
__device__ __forceinline__ void march_row_table(CDesc<T> *D, int4 tl, int sub, int row, int2 *trow) {
  using C = MarchCfg<T, KIND, S>;
  const int m = tl.y;
  const int bx0 = tl.z & 1023, by0 = (tl.z >> 10) & 1023, bz0 = (tl.z >> 20) & 1023;
  const int N = D->N;
  const int ry = row % C::RY, rz = row / C::RY;
  const int qj = 2 * by0 + ry, qk = 2 * (bz0 + C::TZS * sub) + rz;
  const int lim = N - qj - qk, L = lim - 2 * bx0;
  const bool empty = L < 0;
  const int khi = empty ? 0 : min(L, 2 * C::TX);
  const bool limin = !empty && L <= 2 * C::TX;
  const int rowzp = ((qj == 0) << 2) | ((qk == 0) << 3);
  const uint32_t kmask = empty ? 0u : (2u << khi) - 1u;
  uint32_t xmask = kmask;
  if (D->dirichlet && !empty) {
    const uint32_t bnd = *cptr(D->bnd + m);
    if ((bnd >> rowzp) & 1u) xmask = 0u;
    if (bx0 == 0 && ((bnd >> (rowzp | 2 | (lim == 0 ? 1 : 0))) & 1u)) xmask &= ~1u;
    if (limin && ((bnd >> (rowzp | 1 | (lim == 0 ? 2 : 0))) & 1u)) xmask &= ~(1u << khi);
  }
  const int rzs = 2 * C::TZS * sub + rz;  // plane within the segment box
  const bool ey = (ry & 1) || ((ry > 0 || by0 == 0) && ry < 2 * C::TY);
  const bool ez = (rzs & 1) || ((rzs > 0 || bz0 == 0) && rzs < 2 * C::TZ);
  trow[row] = make_int2(empty ? 0 : row_base(qj, qk, N) + 2 * bx0,
                        static_cast<int>(xmask | (kmask << 9) | (uint32_t(limin) << 18) | (uint32_t(qj == 0) << 19) |
                                         (uint32_t(qk == 0) << 20) | (uint32_t(ey && ez) << 21) |
                                         (uint32_t(khi) << 24)));
}

// issue this wavefront's buffer-to-LDS loads of one sub-box (x, then the
// coefficient) into `dst`.  geo[i] of a lane: row | bit << 8 | byte << 16
// (bit: position of its rx in the row's staged mask, 31 for padding slots;
// byte: rx * sizeof(T) + 4 * dword half).  A lane whose bit is clear (outside
// the macro, a Dirichlet DoF of x, padding) gets an out-of-range offset,
// which loads 0.
template <typename T, int KIND, int S>
__device__ __forceinline__ void march_stage(const TileArgs<T> &a, CDesc<T> *D, int4 tl, const int *geo,
                                            LPtr<uint64_t> trow, __attribute__((address_space(3))) T *dst, int w) {
  using C = MarchCfg<T, KIND, S>;
  const int64_t base = D->off + static_cast<int64_t>(tl.y) * D->L;
  const int nbytes = D->L * static_cast<int>(sizeof(T));
  const __amdgpu_buffer_rsrc_t rx_ =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(a.x + base), 0, nbytes, 0x00020000);
  const __amdgpu_buffer_rsrc_t rk_ =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(C::HASK ? a.k + base : a.x + base), 0, nbytes, 0x00020000);
#pragma unroll
  for (int i = 0; i < C::IPW; ++i) {
    const int j = w + C::WPG * i;
    if (j < C::NINS) {
      const int gv = geo[i];
      const int2 e = row_rec(trow, gv & 127);
      const uint32_t bit = (static_cast<uint32_t>(e.y) >> ((gv >> 8) & 31)) & 1u;
      const uint32_t voff = bit ? static_cast<uint32_t>(e.x) * static_cast<uint32_t>(sizeof(T)) + (gv >> 16) : 0xffffffffu;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(j < C::IPA ? rx_ : rk_,
                                               (__attribute__((address_space(3))) void *)(dst + (j * 64) / C::DW),
                                               4, voff, 0, 0, 0);
    }
  }
}

// y[addr + OFF] += v in LDS (FP64, no return), written as an instruction
// the compiler does not track: after a buffer-to-LDS load it would otherwise
// wait for that load before every LDS atomic, although the atomics never
// touch the buffer being loaded.  Its completion is waited for explicitly
// (lgkmcnt) before the barrier that ends the element work.
template <int OFF>
__device__ __forceinline__ void lds_add_f64(uint32_t addr, double v) {
  asm volatile("ds_add_f64 %0, %1 offset:%2" ::"v"(addr), "v"(v), "i"(OFF) : "memory");
}

// the micro-tet of type t in the lane's cube of the current sub-box: local
// results into y[], the cube's LDS slot into cbo; false if it does not exist
template <typename T, int KIND, int S, int t>
__device__ __forceinline__ bool march_elem(CDesc<T> *D, int m, int bsum, LPtr<T> sx, LPtr<T> sk, int lane, double *y,
                                           int &cbo) {
  using C = MarchCfg<T, KIND, S>;
  const int cx = lane % C::TX, cy = (lane / C::TX) % C::TY, cz = lane / (C::TX * C::TY);
  if (bsum + cx + cy + cz > D->n - kLim[t]) return false;
  const int cb = cx + C::RXP * (2 * cy + C::RY * 2 * cz);
  cbo = cb;
  const TypeGeo<T> *g = D->geo + 6 * m + t;
  T u[10], kv[10], yt[10];
#pragma unroll
  for (int v = 0; v < 10; ++v) {
    const int li = cb + node_off(t, v, C::RY, C::OO, C::RXP);
    u[v] = sx[li];
    kv[v] = C::HASK ? sk[li] : T(1);
  }
  p2_elem<T, C::HASK>(u, kv, cptr(g->Gp), cptr(g->Gs), yt);
#pragma unroll
  for (int v = 0; v < 10; ++v) y[v] = double(yt[v]);
  return true;
}

// add a micro-tet's results into the accumulator at LDS byte address sy
template <typename T, int KIND, int S, int t>
__device__ __forceinline__ void march_scatter(uint32_t sy, int cb, const double *y) {
  using C = MarchCfg<T, KIND, S>;
  const uint32_t ab = sy + 8u * static_cast<uint32_t>(cb);
  lds_add_f64<8 * node_off(t, 0, C::RY, C::OO, C::RXP)>(ab, y[0]);
  lds_add_f64<8 * node_off(t, 1, C::RY, C::OO, C::RXP)>(ab, y[1]);
  lds_add_f64<8 * node_off(t, 2, C::RY, C::OO, C::RXP)>(ab, y[2]);
  lds_add_f64<8 * node_off(t, 3, C::RY, C::OO, C::RXP)>(ab, y[3]);
  lds_add_f64<8 * node_off(t, 4, C::RY, C::OO, C::RXP)>(ab, y[4]);
  lds_add_f64<8 * node_off(t, 5, C::RY, C::OO, C::RXP)>(ab, y[5]);
  lds_add_f64<8 * node_off(t, 6, C::RY, C::OO, C::RXP)>(ab, y[6]);
  lds_add_f64<8 * node_off(t, 7, C::RY, C::OO, C::RXP)>(ab, y[7]);
  lds_add_f64<8 * node_off(t, 8, C::RY, C::OO, C::RXP)>(ab, y[8]);
  lds_add_f64<8 * node_off(t, 9, C::RY, C::OO, C::RXP)>(ab, y[9]);
}

template <typename T, int KIND, int S>
__global__ __launch_bounds__(192) void k_march(TileArgs<T> a) {
  using C = MarchCfg<T, KIND, S>;
  constexpr int RX = C::RX, RY = C::RY, RXP = C::RXP, OO = C::OO, ROWS = C::ROWS, RP = C::RP, PLANE = C::PLANE;
  __shared__ T sbuf[2][C::NA * C::RPA];
  __shared__ double sy[RP];
  __shared__ int2 trow[2][ROWS];
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;

  // this workgroup's segments: XCD x (workgroups are dispatched round-robin
  // over the 8 XCDs) owns a contiguous run of the spatially ordered segment
  // list, and its workgroups take that run's segments in turn
  const int G = gridDim.x, x8 = blockIdx.x % 8, jw = blockIdx.x / 8;
  const int gx = G / 8 + (x8 < G % 8 ? 1 : 0);
  const int q = a.ntiles / 8, rem = a.ntiles % 8;
  const int s_begin = x8 * q + min(x8, rem), s_end = s_begin + q + (x8 < rem ? 1 : 0);

  // active flag of segment s's instance, read as a scalar (the aligned word holding its byte)
  auto active = [&](int s) {
    if (a.active == nullptr) return true;
    const uintptr_t p = reinterpret_cast<uintptr_t>(a.active + tile_rec(a.tiles, s).x);
    const uint32_t wv = *cptr(reinterpret_cast<const uint32_t *>(p & ~uintptr_t(3)));
    return ((wv >> (8 * (p & 3))) & 255u) != 0u;
  };
  auto first_from = [&](int s) {
    while (s < s_end && !active(s)) s += gx;
    return s;
  };
  // the sub-box after `it`: the next one of its segment if it exists, else
  // the first of this workgroup's next active segment (seg >= s_end: none)
  auto advance = [&](MarchItem it) {
    const int4 tl = tile_rec(a.tiles, it.seg);
    CDesc<T> *D = (CDesc<T> *)(a.inst + tl.x);
    const int bs = (tl.z & 1023) + ((tl.z >> 10) & 1023) + ((tl.z >> 20) & 1023);
    if (it.sub + 1 < S && bs + C::TZS * (it.sub + 1) <= D->n - 1) return MarchItem{it.seg, it.sub + 1};
    return MarchItem{first_from(it.seg + gx), 0};
  };

  // per-lane geometry of this wavefront's loads (see march_stage)
  int geo[C::IPW];
#pragma unroll
  for (int i = 0; i < C::IPW; ++i) {
    const int j = w + C::WPG * i;
    const int arr = j / C::IPA;
    const int d = (j % C::IPA) * 64 + lane;  // dword within the array
    const int slot = d / C::DW, half = d % C::DW;
    const int row = slot / RXP, xs = slot - row * RXP;
    const int rx = xs < OO ? 2 * xs : (xs < OO + C::TX ? 2 * (xs - OO) + 1 : -1);
    const bool ok = j < C::NINS && row < ROWS && rx >= 0;
    geo[i] = ok ? (row | ((rx + 9 * arr) << 8) | ((rx * static_cast<int>(sizeof(T)) + 4 * half) << 16)) : (31 << 8);
  }

  MarchItem cur{first_from(s_begin + jw), 0};
  if (cur.seg >= s_end) return;
  MarchItem nxt = advance(cur);
  int cb = 0;
  // prologue: tables and loads of the first sub-box, tables of the second, clear the accumulator
  if (tid < ROWS) {
    const int4 tl = tile_rec(a.tiles, cur.seg);
    march_row_table<T, KIND, S>((CDesc<T> *)(a.inst + tl.x), tl, cur.sub, tid, trow[0]);
  }
  lds_barrier();
  {
    const int4 tl = tile_rec(a.tiles, cur.seg);
    march_stage<T, KIND, S>(a, (CDesc<T> *)(a.inst + tl.x), tl, geo, (LPtr<uint64_t>)trow[0],
                            (__attribute__((address_space(3))) T *)sbuf[0], w);
  }
  if (nxt.seg < s_end && tid < ROWS) {
    const int4 tl = tile_rec(a.tiles, nxt.seg);
    march_row_table<T, KIND, S>((CDesc<T> *)(a.inst + tl.x), tl, nxt.sub, tid, trow[1]);
  }
  for (int s = tid; s < RP; s += C::NTH) sy[s] = 0.0;
  wait_vmem();
  lds_barrier();

  while (true) {
    const int nb = cb ^ 1;
    const int4 tl = tile_rec(a.tiles, cur.seg);
    CDesc<T> *D = (CDesc<T> *)(a.inst + tl.x);
    const int m = tl.y;
    const int bx0 = tl.z & 1023, by0 = (tl.z >> 10) & 1023, bz0 = (tl.z >> 20) & 1023;
    const bool more = nxt.seg < s_end;
    // A. loads of the next sub-box
    if (more) {
      const int4 tn = tile_rec(a.tiles, nxt.seg);
      march_stage<T, KIND, S>(a, (CDesc<T> *)(a.inst + tn.x), tn, geo, (LPtr<uint64_t>)trow[nb],
                              (__attribute__((address_space(3))) T *)sbuf[nb], w);
    }
    // B. micro-tets of the current sub-box
    {
      const LPtr<T> sx = (LPtr<T>)sbuf[cb];
      const LPtr<T> sk = (LPtr<T>)(sbuf[cb] + (C::HASK ? C::RPA : 0));
      const uint32_t syb = static_cast<uint32_t>(reinterpret_cast<uintptr_t>((__attribute__((address_space(3))) double *)sy));
      const int bsum = bx0 + by0 + bz0 + C::TZS * cur.sub;
      // wavefront w: types w (round 0) and w + 3 (round 1); each round the
      // wavefronts add their results in wavefront order (reproducible sums,
      // as in k_tile); the untracked LDS atomics are waited for explicitly
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int t = w + 3 * r;
        double y[10];
        int cbe = 0;
        bool valid = false;
        switch (t) {
          case 0: valid = march_elem<T, KIND, S, 0>(D, m, bsum, sx, sk, lane, y, cbe); break;
          case 1: valid = march_elem<T, KIND, S, 1>(D, m, bsum, sx, sk, lane, y, cbe); break;
          case 2: valid = march_elem<T, KIND, S, 2>(D, m, bsum, sx, sk, lane, y, cbe); break;
          case 3: valid = march_elem<T, KIND, S, 3>(D, m, bsum, sx, sk, lane, y, cbe); break;
          case 4: valid = march_elem<T, KIND, S, 4>(D, m, bsum, sx, sk, lane, y, cbe); break;
          default: valid = march_elem<T, KIND, S, 5>(D, m, bsum, sx, sk, lane, y, cbe); break;
        }
#pragma unroll
        for (int p = 0; p < C::WPG; ++p) {
          __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
          lds_barrier();
          if (p == w && valid) {
            switch (t) {
              case 0: march_scatter<T, KIND, S, 0>(syb, cbe, y); break;
              case 1: march_scatter<T, KIND, S, 1>(syb, cbe, y); break;
              case 2: march_scatter<T, KIND, S, 2>(syb, cbe, y); break;
              case 3: march_scatter<T, KIND, S, 3>(syb, cbe, y); break;
              case 4: march_scatter<T, KIND, S, 4>(syb, cbe, y); break;
              default: march_scatter<T, KIND, S, 5>(syb, cbe, y); break;
            }
          }
        }
      }
    }
    // the element work's LDS atomics, the next sub-box's loads and the
    // previous write-back's stores are complete here (s_waitcnt 0: all
    // counters); the next iteration reads the loaded buffer after two more barriers
    __builtin_amdgcn_s_waitcnt(0);
    lds_barrier();
    // C. write-back: planes 0 .. 7 of the sub-box, and plane 8 if it ends its segment
    const bool carry = more && nxt.seg == cur.seg;
    {
      const int64_t base = D->off + static_cast<int64_t>(m) * D->L;
      GPtr<T> yb = gptr(a.y + base);
      GPtr<T> pt = gptr(a.partial ? a.partial : D->partial) + static_cast<int64_t>(tl.w) * C::RSEG;
      const uint32_t bnd = D->dirichlet ? *cptr(D->bnd + m) : 0u;
      const int npts = RX * RY * (carry ? C::RZ - 1 : C::RZ);
      const LPtr<uint64_t> tr = (LPtr<uint64_t>)trow[cb];
      for (int r = tid; r < npts; r += C::NTH) {
        const int row = r / RX, rx = r - row * RX;
        const int2 e = row_rec(tr, row);
        const uint32_t inf = static_cast<uint32_t>(e.y);
        if (!((inf >> (9 + rx)) & 1u)) continue;
        const T v = T(sy[lds_slot(rx, row, OO, RXP)]);
        const bool ex = (rx & 1) || ((rx > 0 || bx0 == 0) && rx < 2 * C::TX);
        if (((inf >> 21) & 1u) && ex) {
          const int zp = (((inf >> 18) & 1u) && rx == static_cast<int>((inf >> 24) & 31u)) |
                         ((bx0 == 0 && rx == 0) << 1) | (((inf >> 19) & 1u) << 2) | (((inf >> 20) & 1u) << 3);
          __builtin_nontemporal_store(((bnd >> zp) & 1u) ? T(0) : v, &yb[e.x + rx]);
        } else {
          const int ry = row % RY, rz = row / RY;
          pt[rx + RX * (ry + RY * (2 * C::TZS * cur.sub + rz))] = v;
        }
      }
    }
    lds_barrier();
    // D. clear the accumulator (the carried face moves to plane 0) and build
    // the tables of the sub-box after next
    MarchItem nn{s_end, 0};
    if (more) nn = advance(nxt);
    for (int s = tid; s < PLANE; s += C::NTH) {
      const double c = carry ? sy[s + (C::RZ - 1) * PLANE] : 0.0;
      sy[s] = c;
#pragma unroll
      for (int p = 1; p < C::RZ; ++p) sy[s + p * PLANE] = 0.0;
    }
    if (nn.seg < s_end && tid < ROWS) {
      const int4 t2 = tile_rec(a.tiles, nn.seg);
      march_row_table<T, KIND, S>((CDesc<T> *)(a.inst + t2.x), t2, nn.sub, tid, trow[cb]);
    }
    if (!more) break;
    lds_barrier();
    cur = nxt;
    nxt = nn;
    cb = nb;
  }
}

// LDS per CU that concurrently resident workgroups can actually hold on
// gfx950 (measured: three 40 KB workgroups fit, four do not)
constexpr int kUsableLdsPerCU = 120 * 1024;

template <typename T, int KIND, int S>
hipError_t launch_march(const TileArgs<T> &a, hipStream_t s) {
  if (a.ntiles == 0) return hipSuccess;
  // persistent: as many workgroups as are resident at once (at most one per
  // segment); the occupancy query overstates how many fit in LDS, so the
  // count is also capped by the usable LDS
  static int resident = 0;
  if (resident == 0) {
    int dev = 0, ncu = 0, per = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_march<T, KIND, S>, MarchCfg<T, KIND, S>::NTH, 0);
    hipFuncAttributes fa;
    if (e == hipSuccess) e = hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(k_march<T, KIND, S>));
    if (e != hipSuccess) return e;
    const int by_lds = fa.sharedSizeBytes > 0 ? kUsableLdsPerCU / static_cast<int>(fa.sharedSizeBytes) : per;
    resident = ncu * max(1, min(per, by_lds));
  }
  const int grid = a.ntiles < resident ? a.ntiles : resident;
  hipLaunchKernelGGL((k_march<T, KIND, S>), dim3(grid), dim3(MarchCfg<T, KIND, S>::NTH), 0, s, a);
  return hipGetLastError();
}

template <typename T, int KIND, int MAP, int TX, int TY, int TZ>
hipError_t launch_cfg(const TileArgs<T> &a, hipStream_t s) {
  using Cfg = TileCfg<T, KIND, MAP, TX, TY, TZ>;
  if (a.ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL((k_tile<T, KIND, MAP, TX, TY, TZ>), dim3(a.ntiles), dim3(Cfg::NTH), 0, s, a);
  return hipGetLastError();
}

template <typename T, int KIND, int MAP>
hipError_t launch_kind(const TileArgs<T> &a, int cfg, hipStream_t s) {
  switch (cfg) {
    case 0: return launch_cfg<T, KIND, MAP, 4, 4, 4>(a, s);
    case 1: return launch_cfg<T, KIND, MAP, 8, 4, 2>(a, s);
    case 2: return launch_cfg<T, KIND, MAP, 8, 4, 4>(a, s);
    case 3: return launch_cfg<T, KIND, MAP, 4, 4, 8>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

template <typename T, int KIND>
hipError_t launch_march_cfg(const TileArgs<T> &a, int cfg, hipStream_t s) {
  switch (kTileMarch[cfg]) {
    case 2: return launch_march<T, KIND, 2>(a, s);
    case 4: return launch_march<T, KIND, 4>(a, s);
    case 8: return launch_march<T, KIND, 8>(a, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_tile_apply(const TileArgs<T> &a, int kind, int map, int cfg, hipStream_t s) {
  if (cfg < 0 || cfg >= kNumTileCfg) return hipErrorInvalidValue;
  if (kTileMarch[cfg] != 0) {
    // marching tiles: the scalar P2 applies
    if (map != 0) return hipErrorInvalidValue;
    if (kind == P2_LAPLACE) return launch_march_cfg<T, P2_LAPLACE>(a, cfg, s);
    if (kind == P2_DIVKGRAD) return launch_march_cfg<T, P2_DIVKGRAD>(a, cfg, s);
    return hipErrorInvalidValue;
  }
  switch (kind) {
    case P2_LAPLACE: return launch_kind<T, P2_LAPLACE, 0>(a, cfg, s);
    case P2_DIVKGRAD: return launch_kind<T, P2_DIVKGRAD, 0>(a, cfg, s);
    case N1_CURLCURL: return launch_kind<T, N1_CURLCURL, 0>(a, cfg, s);
    case P2_DIVKGRAD_STORE: return launch_kind<T, P2_DIVKGRAD_STORE, 0>(a, cfg, s);
    case P2_DIVKGRAD_Q: return launch_kind<T, P2_DIVKGRAD_Q, 0>(a, cfg, s);
    case P2_STORED_APPLY: return launch_kind<T, P2_STORED_APPLY, 0>(a, cfg, s);
    case P2_LAPLACE_DIAG: return launch_kind<T, P2_LAPLACE_DIAG, 0>(a, cfg, s);
    case P2_DIVKGRAD_DIAG: return launch_kind<T, P2_DIVKGRAD_DIAG, 0>(a, cfg, s);
    case P2_DIVKGRAD_GRADK: return launch_kind<T, P2_DIVKGRAD_GRADK, 0>(a, cfg, s);
    case P2V_EPSILON_GRADMU:
      if (cfg == 0)
        return map == 0 ? launch_cfg<T, P2V_EPSILON_GRADMU, 0, 4, 4, 4>(a, s)
                        : launch_cfg<T, P2V_EPSILON_GRADMU, 1, 4, 4, 4>(a, s);
      if (cfg == 1)
        return map == 0 ? launch_cfg<T, P2V_EPSILON_GRADMU, 0, 8, 4, 2>(a, s)
                        : launch_cfg<T, P2V_EPSILON_GRADMU, 1, 8, 4, 2>(a, s);
      return hipErrorInvalidValue;
    case P2V_EPSILON_DIAG:
      if (cfg == 0)
        return map == 0 ? launch_cfg<T, P2V_EPSILON_DIAG, 0, 4, 4, 4>(a, s)
                        : launch_cfg<T, P2V_EPSILON_DIAG, 1, 4, 4, 4>(a, s);
      if (cfg == 1)
        return map == 0 ? launch_cfg<T, P2V_EPSILON_DIAG, 0, 8, 4, 2>(a, s)
                        : launch_cfg<T, P2V_EPSILON_DIAG, 1, 8, 4, 2>(a, s);
      return hipErrorInvalidValue;
    case P2V_EPSILON:
      // the epsilon tiles stage 3 components: only the 64-cube boxes (4 x 4 x 4
      // and 8 x 4 x 2, 45 and 50 KB of LDS in FP64) fit twice per CU
      if (cfg == 0)
        return map == 0 ? launch_cfg<T, P2V_EPSILON, 0, 4, 4, 4>(a, s) : launch_cfg<T, P2V_EPSILON, 1, 4, 4, 4>(a, s);
      if (cfg == 1)
        return map == 0 ? launch_cfg<T, P2V_EPSILON, 0, 8, 4, 2>(a, s) : launch_cfg<T, P2V_EPSILON, 1, 8, 4, 2>(a, s);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_tile_apply<double>(const TileArgs<double> &, int, int, int, hipStream_t);
template hipError_t launch_tile_apply<float>(const TileArgs<float> &, int, int, int, hipStream_t);

template <typename T>
hipError_t launch_seam_gather(const SeamInst<T> *inst, const int4 *work, int nwork, T *y, const uint8_t *active,
                              int flags, int ncomp, int ppt, int cfg, int rows_lds, hipStream_t s,
                              const T *partial) {
  if (nwork == 0) return hipSuccess;
  const dim3 grid(nwork);
  const size_t sh = static_cast<size_t>(rows_lds) * sizeof(int);
#define TMF_SEAM(NC_, PPT_, TX_, TY_, TZ_)                                                                   \
  hipLaunchKernelGGL((k_seam<T, NC_, PPT_, TX_, TY_, TZ_>), grid, dim3(256), sh, s, inst, work, y, active, flags, \
                     rows_lds, partial)
  if (ncomp == 3 || ppt == 1) {
    // vector fields and the scalar gradient of a vector operator: cfg 0 or 1, one point per thread
    if (cfg > 1 || ppt != 1) return hipErrorInvalidValue;
    if (cfg == 0) {
      if (ncomp == 3) TMF_SEAM(3, 1, 4, 4, 4);
      else TMF_SEAM(1, 1, 4, 4, 4);
    } else {
      if (ncomp == 3) TMF_SEAM(3, 1, 8, 4, 2);
      else TMF_SEAM(1, 1, 8, 4, 2);
    }
    return hipGetLastError();
  }
  if (ppt != kSeamPointsPerThread) return hipErrorInvalidValue;
  switch (cfg) {
    case 0: TMF_SEAM(1, kSeamPointsPerThread, 4, 4, 4); break;
    case 1: TMF_SEAM(1, kSeamPointsPerThread, 8, 4, 2); break;
    case 2: TMF_SEAM(1, kSeamPointsPerThread, 8, 4, 4); break;
    case 3:
    case 4: TMF_SEAM(1, kSeamPointsPerThread, 4, 4, 8); break;
    case 5: TMF_SEAM(1, kSeamPointsPerThread, 4, 4, 16); break;
    case 6: TMF_SEAM(1, kSeamPointsPerThread, 4, 4, 32); break;
    default: return hipErrorInvalidValue;
  }
#undef TMF_SEAM
  return hipGetLastError();
}

template hipError_t launch_seam_gather<double>(const SeamInst<double> *, const int4 *, int, double *,
                                               const uint8_t *, int, int, int, int, int, hipStream_t, const double *);
template hipError_t launch_seam_gather<float>(const SeamInst<float> *, const int4 *, int, float *, const uint8_t *,
                                              int, int, int, int, int, hipStream_t, const float *);

}  // namespace tmf
