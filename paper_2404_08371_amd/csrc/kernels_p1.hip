// P1 operators: vertex-centric ("owner computes") matrix-free kernels.
//
// Each thread owns one lattice point p = (i, j, k) of one macro and forms row
// p of A x: y_p = sum over the (up to 24) micro-tets T containing p of
// (A_T x_T)_p (equation (4.1) restricted to one row).  Every row is written
// exactly once: no write conflicts, no atomics, fixed summation order.  A
// wavefront owns a chunk of up to 64 consecutive points of one lattice row
// (a host-built table lists the chunks, so no thread decodes a packed index),
// the row bases of the 7 lattice rows its 15-point neighbourhoods touch are
// computed once per wavefront, and all 15 neighbour loads of a point are
// issued together (neighbouring lanes read neighbouring words).  Chunks at
// distance >= 2 from every macro face (the bulk) take an unguarded path;
// the others check each neighbour and zero Dirichlet DoFs of x (x_b ignored).
//
// The local matrices are the per-(macro, type) constants
// Gp = |T| grad(lambda_a).grad(lambda_b) (affine macros: every micro-tet of
// a type shares its Jacobian -- the loop-invariant hoisting of section
// "Automatic Identification of Loop Invariants", done once on the host).
// For the constant-coefficient operator they are pre-summed into 15-point
// stencils, one per boundary class: which of the four macro faces (i = 0,
// j = 0, k = 0, i + j + k = N) the point lies on decides which of its 24
// micro-tets exist, so 16 stencils cover every point of a macro.
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

// 15-point neighbour q -> (plane: 0 = k-1, 1 = k, 2 = k+1; in-plane slot)
constexpr int kNbPlane[15] = {1, 1, 1, 1, 1, 2, 0, 1, 1, 0, 2, 0, 2, 2, 0};
constexpr int kNbSlot[15] = {0, 1, 2, 3, 4, 0, 0, 5, 6, 1, 2, 3, 4, 5, 6};

static_assert(kNb[5][2] == 1 && kNb[6][2] == -1 && kNb[13][0] == 1 && kNb[14][2] == -1, "neighbour table");

// micro-tet (t, slot a) containing p exists, given p's zero pattern z
// (bit 0: i+j+k = N, bit 1: i = 0, bit 2: j = 0, bit 3: k = 0)
template <int t, int a>
__device__ __forceinline__ bool tet_exists(int z) {
  constexpr int ox = kOff[t][a][0], oy = kOff[t][a][1], oz = kOff[t][a][2];
  constexpr bool diag = ox + oy + oz < kLim[t];
  constexpr int bad = (diag ? 1 : 0) | (ox ? 2 : 0) | (oy ? 4 : 0) | (oz ? 8 : 0);
  return (z & bad) == 0;
}

template <typename T>
__device__ __forceinline__ T nbval(const T P[3][7], int q) {
  return P[kNbPlane[q]][kNbSlot[q]];
}

// row p of sum_T kbar_T Gp_T x_T over the existing micro-tets containing p
template <typename T, int t, int a>
__device__ __forceinline__ void p1k_tet(const TypeGeo<T> *__restrict__ g, const T X[3][7], const T K[3][7], int z,
                                        T &acc) {
  const T *G = g[t].Gp + 4 * a;
  const int q0 = kVS.v[t][a][0], q1 = kVS.v[t][a][1], q2 = kVS.v[t][a][2], q3 = kVS.v[t][a][3];
  const T r = G[0] * nbval(X, q0) + G[1] * nbval(X, q1) + G[2] * nbval(X, q2) + G[3] * nbval(X, q3);
  const T kb = (nbval(K, q0) + nbval(K, q1) + nbval(K, q2) + nbval(K, q3)) * T(0.25);
  const T c = kb * r;
  acc += tet_exists<t, a>(z) ? c : T(0);
}

template <typename T>
__device__ __forceinline__ T p1k_row(const TypeGeo<T> *g, const T X[3][7], const T K[3][7], int z) {
  T acc = T(0);
  p1k_tet<T, 0, 0>(g, X, K, z, acc); p1k_tet<T, 0, 1>(g, X, K, z, acc);
  p1k_tet<T, 0, 2>(g, X, K, z, acc); p1k_tet<T, 0, 3>(g, X, K, z, acc);
  p1k_tet<T, 1, 0>(g, X, K, z, acc); p1k_tet<T, 1, 1>(g, X, K, z, acc);
  p1k_tet<T, 1, 2>(g, X, K, z, acc); p1k_tet<T, 1, 3>(g, X, K, z, acc);
  p1k_tet<T, 2, 0>(g, X, K, z, acc); p1k_tet<T, 2, 1>(g, X, K, z, acc);
  p1k_tet<T, 2, 2>(g, X, K, z, acc); p1k_tet<T, 2, 3>(g, X, K, z, acc);
  p1k_tet<T, 3, 0>(g, X, K, z, acc); p1k_tet<T, 3, 1>(g, X, K, z, acc);
  p1k_tet<T, 3, 2>(g, X, K, z, acc); p1k_tet<T, 3, 3>(g, X, K, z, acc);
  p1k_tet<T, 4, 0>(g, X, K, z, acc); p1k_tet<T, 4, 1>(g, X, K, z, acc);
  p1k_tet<T, 4, 2>(g, X, K, z, acc); p1k_tet<T, 4, 3>(g, X, K, z, acc);
  p1k_tet<T, 5, 0>(g, X, K, z, acc); p1k_tet<T, 5, 1>(g, X, K, z, acc);
  p1k_tet<T, 5, 2>(g, X, K, z, acc); p1k_tet<T, 5, 3>(g, X, K, z, acc);
  return acc;
}

// 1/4 (D gy)_T . Gp_T (D x)_T summed over the existing micro-tets containing p
template <typename T, int t, int a>
__device__ __forceinline__ void kgrad_tet(const TypeGeo<T> *__restrict__ g, const T R[3][7], const T X[3][7], int z,
                                          T &acc) {
  const T *G = g[t].Gp;
  T bil = T(0);
#pragma unroll
  for (int c1 = 0; c1 < 4; ++c1) {
    const T row = G[4 * c1 + 0] * nbval(X, kVS.v[t][a][0]) + G[4 * c1 + 1] * nbval(X, kVS.v[t][a][1]) +
                  G[4 * c1 + 2] * nbval(X, kVS.v[t][a][2]) + G[4 * c1 + 3] * nbval(X, kVS.v[t][a][3]);
    bil += nbval(R, kVS.v[t][a][c1]) * row;
  }
  acc += tet_exists<t, a>(z) ? bil : T(0);
}

template <typename T>
__device__ __forceinline__ T kgrad_row(const TypeGeo<T> *g, const T R[3][7], const T X[3][7], int z) {
  T acc = T(0);
  kgrad_tet<T, 0, 0>(g, R, X, z, acc); kgrad_tet<T, 0, 1>(g, R, X, z, acc);
  kgrad_tet<T, 0, 2>(g, R, X, z, acc); kgrad_tet<T, 0, 3>(g, R, X, z, acc);
  kgrad_tet<T, 1, 0>(g, R, X, z, acc); kgrad_tet<T, 1, 1>(g, R, X, z, acc);
  kgrad_tet<T, 1, 2>(g, R, X, z, acc); kgrad_tet<T, 1, 3>(g, R, X, z, acc);
  kgrad_tet<T, 2, 0>(g, R, X, z, acc); kgrad_tet<T, 2, 1>(g, R, X, z, acc);
  kgrad_tet<T, 2, 2>(g, R, X, z, acc); kgrad_tet<T, 2, 3>(g, R, X, z, acc);
  kgrad_tet<T, 3, 0>(g, R, X, z, acc); kgrad_tet<T, 3, 1>(g, R, X, z, acc);
  kgrad_tet<T, 3, 2>(g, R, X, z, acc); kgrad_tet<T, 3, 3>(g, R, X, z, acc);
  kgrad_tet<T, 4, 0>(g, R, X, z, acc); kgrad_tet<T, 4, 1>(g, R, X, z, acc);
  kgrad_tet<T, 4, 2>(g, R, X, z, acc); kgrad_tet<T, 4, 3>(g, R, X, z, acc);
  kgrad_tet<T, 5, 0>(g, R, X, z, acc); kgrad_tet<T, 5, 1>(g, R, X, z, acc);
  kgrad_tet<T, 5, 2>(g, R, X, z, acc); kgrad_tet<T, 5, 3>(g, R, X, z, acc);
  return acc * T(0.25);
}

// The 15-point neighbourhood of the points of one row chunk: row bases (in
// the macro's block) of the 7 rows (j, k), (j+-1, k), (j, k+-1), (j+1, k-1),
// (j-1, k+1); slot q of point (i, j, k) is at rb[row of q] + i + di(q).
struct Rows {
  int rb[3][3];  // [plane k-1, k, k+1][row j-1, j, j+1]
};

__device__ __forceinline__ Rows chunk_rows(int j, int k, int N) {
  Rows R;
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const int kk = k + p - 1, jj = j + r - 1;
      const int M = N - kk;
      R.rb[p][r] = c3(N) - c3(M) + (jj * (2 * M + 3 - jj)) / 2;
    }
  return R;
}

// values of v at the neighbourhood of (i, j, k).  CHECK: points outside the
// lattice read 0, and with MASK Dirichlet DoFs read 0 too.
template <typename T, bool CHECK, bool MASK>
__device__ __forceinline__ void gather15(const T *__restrict__ v, const Rows &R, int i, int j, int k, int N,
                                         uint32_t bnd, T P[3][7]) {
#pragma unroll
  for (int q = 0; q < 15; ++q) {
    const int di = kNb[q][0], dj = kNb[q][1], dk = kNb[q][2];
    const int ii = i + di, jj = j + dj, kk = k + dk;
    bool ok = true;
    if (CHECK) {
      ok = ii >= 0 && jj >= 0 && kk >= 0 && ii + jj + kk <= N;
      if (MASK) ok = ok && !((bnd >> zero_pattern(ii, jj, kk, N)) & 1u);
    }
    T val = T(0);
    if (ok) val = v[R.rb[dk + 1][dj + 1] + ii];
    P[kNbPlane[q]][kNbSlot[q]] = val;
  }
}

// Workgroups are dealt round-robin to the 8 XCDs (each with its own L2).
// Renumber them so that XCD x runs one contiguous run of the (macro, chunk
// block) sequence, in order: neighbouring rows and planes -- the 15-point
// neighbourhoods -- are then read through the same L2.
__device__ __forceinline__ void xcd_block(int nchunks, int *m, int *cb) {
  const int per_macro = (nchunks + 3) / 4;
  const int nb = gridDim.x, b = blockIdx.x;
  const int x8 = b & 7, q = nb >> 3, rem = nb & 7;
  const int t = x8 * q + min(x8, rem) + (b >> 3);
  *m = t / per_macro;
  *cb = t - *m * per_macro;
}

// One wavefront per row chunk (up to 64 consecutive points of one lattice
// row); a 1-D grid of ceil(chunks / 4) * macros workgroups of 4 wavefronts.
template <typename T, int KIND>
__global__ __launch_bounds__(256) void k_p1_apply(P1Args<T> a, const int4 *__restrict__ chunks, int nchunks) {
  constexpr bool VARK = KIND == P1_DIVKGRAD;
  const LatticeArgs<T> &L = a.lat;
  const int N = L.N;
  int m, cb;
  xcd_block(nchunks, &m, &cb);
  const int ch = cb * 4 + (threadIdx.x >> 6);
  if (ch >= nchunks) return;
  const int4 c = chunks[ch];  // j, k, i0, length
  const int j = c.x, k = c.y, i = c.z + (threadIdx.x & 63);
  if (i >= c.z + c.w) return;
  const int64_t base = static_cast<int64_t>(m) * L.L;
  const uint32_t bnd = L.bnd[m];
  const Rows R = chunk_rows(j, k, N);
  const T *x = a.x + base;
  const T *kc = VARK ? a.k + base : nullptr;
  const TypeGeo<T> *g = L.geo + 6 * m;
  const int d = L.dirichlet ? 2 : 1;
  // every point of the chunk at distance >= d from each macro face: all 24
  // micro-tets exist and no neighbour is a Dirichlet DoF
  const bool inner = j >= d && k >= d && c.z >= d && c.z + c.w - 1 + j + k <= N - d;
  T X[3][7], K[3][7];
  T acc = T(0);
  if (inner) {
    gather15<T, false, false>(x, R, i, j, k, N, bnd, X);
    if (VARK) {
      gather15<T, false, false>(kc, R, i, j, k, N, bnd, K);
      acc = p1k_row(g, X, K, 0);
    } else {
      const T *w = a.w15 + 16 * 15 * m;  // class 0: the interior stencil
#pragma unroll
      for (int q = 0; q < 15; ++q) acc += w[q] * nbval(X, q);
    }
  } else {
    const int z = zero_pattern(i, j, k, N);
    if (!(L.dirichlet && ((bnd >> z) & 1u))) {
      if (L.dirichlet)
        gather15<T, true, true>(x, R, i, j, k, N, bnd, X);
      else
        gather15<T, true, false>(x, R, i, j, k, N, bnd, X);
      if (VARK) {
        gather15<T, true, false>(kc, R, i, j, k, N, bnd, K);
        acc = p1k_row(g, X, K, z);
      } else {
        const T *w = a.w15 + (16 * m + z) * 15;
#pragma unroll
        for (int q = 0; q < 15; ++q) acc += w[q] * nbval(X, q);
      }
    }
  }
  a.y[base + R.rb[1][1] + i] = acc;
}

// Fused reverse mode of the macro-local P1 div(k grad) apply:
//   gx_p = (L(k) gy)_p,  gk_p = sum_{T containing p} 1/4 (D gy)_T . Gp_T (D x)_T
template <typename T>
__global__ __launch_bounds__(256) void k_p1_adjoint(P1AdjArgs<T> a, const int4 *__restrict__ chunks, int nchunks) {
  const LatticeArgs<T> &L = a.lat;
  const int N = L.N;
  int m, cb;
  xcd_block(nchunks, &m, &cb);
  const int ch = cb * 4 + (threadIdx.x >> 6);
  if (ch >= nchunks) return;
  const int4 c = chunks[ch];
  const int j = c.x, k = c.y, i = c.z + (threadIdx.x & 63);
  if (i >= c.z + c.w) return;
  const int64_t base = static_cast<int64_t>(m) * L.L;
  const uint32_t bnd = L.bnd[m];
  const Rows R = chunk_rows(j, k, N);
  const TypeGeo<T> *g = L.geo + 6 * m;
  const int d = L.dirichlet ? 2 : 1;
  const bool inner = j >= d && k >= d && c.z >= d && c.z + c.w - 1 + j + k <= N - d;
  T G[3][7], X[3][7], K[3][7];
  int z = 0;
  if (inner) {
    gather15<T, false, false>(a.gy + base, R, i, j, k, N, bnd, G);
    gather15<T, false, false>(a.x + base, R, i, j, k, N, bnd, X);
    gather15<T, false, false>(a.k + base, R, i, j, k, N, bnd, K);
  } else {
    z = zero_pattern(i, j, k, N);
    if (L.dirichlet) {
      gather15<T, true, true>(a.gy + base, R, i, j, k, N, bnd, G);
      gather15<T, true, true>(a.x + base, R, i, j, k, N, bnd, X);
    } else {
      gather15<T, true, false>(a.gy + base, R, i, j, k, N, bnd, G);
      gather15<T, true, false>(a.x + base, R, i, j, k, N, bnd, X);
    }
    gather15<T, true, false>(a.k + base, R, i, j, k, N, bnd, K);
  }
  const bool self_bnd = L.dirichlet && ((bnd >> z) & 1u);
  const int64_t slot = base + R.rb[1][1] + i;
  a.gx[slot] = self_bnd ? T(0) : p1k_row(g, G, K, z);
  if (a.gk) a.gk[slot] = kgrad_row(g, G, X, z);
}

}  // namespace

template <typename T>
hipError_t launch_p1_apply(const P1Args<T> &a, int kind, const int4 *chunks, int nchunks, hipStream_t s) {
  const dim3 grid(((nchunks + 3) / 4) * a.lat.nt);
  if (kind == P1_LAPLACE)
    hipLaunchKernelGGL((k_p1_apply<T, P1_LAPLACE>), grid, dim3(256), 0, s, a, chunks, nchunks);
  else
    hipLaunchKernelGGL((k_p1_apply<T, P1_DIVKGRAD>), grid, dim3(256), 0, s, a, chunks, nchunks);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_p1_adjoint(const P1AdjArgs<T> &a, const int4 *chunks, int nchunks, hipStream_t s) {
  const dim3 grid(((nchunks + 3) / 4) * a.lat.nt);
  hipLaunchKernelGGL((k_p1_adjoint<T>), grid, dim3(256), 0, s, a, chunks, nchunks);
  return hipGetLastError();
}

template hipError_t launch_p1_apply<double>(const P1Args<double> &, int, const int4 *, int, hipStream_t);
template hipError_t launch_p1_apply<float>(const P1Args<float> &, int, const int4 *, int, hipStream_t);
template hipError_t launch_p1_adjoint<double>(const P1AdjArgs<double> &, const int4 *, int, hipStream_t);
template hipError_t launch_p1_adjoint<float>(const P1AdjArgs<float> &, const int4 *, int, hipStream_t);

}  // namespace tmf
