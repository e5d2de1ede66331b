// P1 operators: vertex-centric ("owner computes") matrix-free kernels.
//
// Each lane owns one lattice point p = (i, j, k) of one macro and forms row p
// of A x: y_p = sum over the (up to 24) micro-tets T containing p of
// (A_T x_T)_p (equation (4.1) restricted to one row).  Every row is written
// exactly once: no write conflicts, no atomics, fixed summation order.
//
// Data movement.  The 15-point neighbourhood of p spans 7 lattice rows: rows
// j-1, j, j+1 of plane k, rows j, j+1 of plane k-1 and rows j-1, j of plane
// k+1.  A wavefront owns 62 consecutive points of a row (lanes 1..62; lanes 0
// and 63 hold the i-1 / i+1 neighbours of the ends) and marches along j
// through a segment of rows of one plane, keeping a sliding window of rows
// in registers: each step loads only the 3 rows that enter the window (one
// per plane), issued one step ahead, and the i +- 1 neighbours come from the
// adjacent lanes.  This takes the vector-memory request rate -- which bounds
// a gather of 15 separate neighbour loads per point -- down to about 3.5 row
// loads per point.  Rows are loaded with out-of-lattice points as 0 and, for
// Dirichlet conditions, with boundary DoFs as 0 (x_b ignored), so every later
// use of a row sees the masked values.
//
// The local matrices are the per-(macro, type) constants
// Gp = |T| grad(lambda_a).grad(lambda_b) (affine macros: every micro-tet of
// a type shares its Jacobian -- the loop-invariant hoisting of section
// "Automatic Identification of Loop Invariants", done once on the host).
// For the constant-coefficient operator, points inside the macro (all 24
// micro-tets present) use their sum, a 15-point stencil; points on a macro
// face (i = 0, j = 0, k = 0 or i + j + k = N) sum the micro-tets that exist.
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

// per-type geometry: read-only, wave-uniform -> scalar loads via the constant address space
template <typename T>
using GeoPtr = const __attribute__((address_space(4))) TypeGeo<T> *;

// Gp_T is symmetric with zero row sums (sum_b grad(lambda_b) = 0), so its six
// off-diagonal entries determine it; the element code reads only those (upper
// triangle: 36 values per macro, which stay in scalar registers) and works
// with differences to the centre point p:
//   (Gp x)_a = sum_{c != a} Gp_ac (x_c - x_a)
//   r^T Gp x = -sum_{a < c} Gp_ac (r_a - r_c)(x_a - x_c)
template <typename T>
__device__ __forceinline__ T goff(GeoPtr<T> g, int t, int a, int c) {
  return a < c ? g[t].Gp[4 * a + c] : g[t].Gp[4 * c + a];
}

// neighbour values minus the centre value (slot 0 is p itself)
template <typename T>
__device__ __forceinline__ void centred(const T P[3][7], T D[3][7]) {
  const T c = P[1][0];
#pragma unroll
  for (int pl = 0; pl < 3; ++pl)
#pragma unroll
    for (int sl = 0; sl < 7; ++sl) D[pl][sl] = P[pl][sl] - c;
}

// row p of sum_T kbar_T Gp_T x_T over the existing micro-tets containing p
// (p is local vertex a of the type-t micro-tet; DX = centred x).  ALL: every
// micro-tet around p exists (a wavefront of interior points), no per-tet
// test.  The factor 1/4 of the vertex mean kbar is applied once to the sum
// (a power of two: the same result as per term).
template <typename T, int t, int a, bool ALL>
__device__ __forceinline__ void p1k_tet(GeoPtr<T> g, const T DX[3][7], const T K[3][7], int z, T &acc) {
  T r = T(0);
#pragma unroll
  for (int c = 0; c < 4; ++c)
    if (c != a) r += goff(g, t, a, c) * nbval(DX, kVS.v[t][a][c]);
  const int q0 = kVS.v[t][a][0], q1 = kVS.v[t][a][1], q2 = kVS.v[t][a][2], q3 = kVS.v[t][a][3];
  const T ks = (nbval(K, q0) + nbval(K, q1)) + (nbval(K, q2) + nbval(K, q3));
  if constexpr (ALL)
    acc += ks * r;
  else
    acc += tet_exists<t, a>(z) ? ks * r : T(0);
}

template <typename T, bool ALL>
__device__ __forceinline__ T p1k_row(GeoPtr<T> g, const T X[3][7], const T K[3][7], int z) {
  T DX[3][7];
  centred(X, DX);
  T acc = T(0);
  p1k_tet<T, 0, 0, ALL>(g, DX, K, z, acc); p1k_tet<T, 0, 1, ALL>(g, DX, K, z, acc);
  p1k_tet<T, 0, 2, ALL>(g, DX, K, z, acc); p1k_tet<T, 0, 3, ALL>(g, DX, K, z, acc);
  p1k_tet<T, 1, 0, ALL>(g, DX, K, z, acc); p1k_tet<T, 1, 1, ALL>(g, DX, K, z, acc);
  p1k_tet<T, 1, 2, ALL>(g, DX, K, z, acc); p1k_tet<T, 1, 3, ALL>(g, DX, K, z, acc);
  p1k_tet<T, 2, 0, ALL>(g, DX, K, z, acc); p1k_tet<T, 2, 1, ALL>(g, DX, K, z, acc);
  p1k_tet<T, 2, 2, ALL>(g, DX, K, z, acc); p1k_tet<T, 2, 3, ALL>(g, DX, K, z, acc);
  p1k_tet<T, 3, 0, ALL>(g, DX, K, z, acc); p1k_tet<T, 3, 1, ALL>(g, DX, K, z, acc);
  p1k_tet<T, 3, 2, ALL>(g, DX, K, z, acc); p1k_tet<T, 3, 3, ALL>(g, DX, K, z, acc);
  p1k_tet<T, 4, 0, ALL>(g, DX, K, z, acc); p1k_tet<T, 4, 1, ALL>(g, DX, K, z, acc);
  p1k_tet<T, 4, 2, ALL>(g, DX, K, z, acc); p1k_tet<T, 4, 3, ALL>(g, DX, K, z, acc);
  p1k_tet<T, 5, 0, ALL>(g, DX, K, z, acc); p1k_tet<T, 5, 1, ALL>(g, DX, K, z, acc);
  p1k_tet<T, 5, 2, ALL>(g, DX, K, z, acc); p1k_tet<T, 5, 3, ALL>(g, DX, K, z, acc);
  return acc * T(0.25);
}

// diagonal entry of row p: sum over the existing micro-tets containing p of
// kbar_T (Gp_T)_aa, with (Gp_T)_aa = -sum_{c != a} (Gp_T)_ac (zero row sums)
template <typename T, int t, int a>
__device__ __forceinline__ void p1k_diag_tet(GeoPtr<T> g, const T K[3][7], int z, T &acc) {
  T gaa = T(0);
#pragma unroll
  for (int c = 0; c < 4; ++c)
    if (c != a) gaa -= goff(g, t, a, c);
  const int q0 = kVS.v[t][a][0], q1 = kVS.v[t][a][1], q2 = kVS.v[t][a][2], q3 = kVS.v[t][a][3];
  const T kb = (nbval(K, q0) + nbval(K, q1) + nbval(K, q2) + nbval(K, q3)) * T(0.25);
  acc += tet_exists<t, a>(z) ? kb * gaa : T(0);
}

template <typename T>
__device__ __forceinline__ T p1k_diag(GeoPtr<T> g, const T K[3][7], int z) {
  T acc = T(0);
  p1k_diag_tet<T, 0, 0>(g, K, z, acc); p1k_diag_tet<T, 0, 1>(g, K, z, acc);
  p1k_diag_tet<T, 0, 2>(g, K, z, acc); p1k_diag_tet<T, 0, 3>(g, K, z, acc);
  p1k_diag_tet<T, 1, 0>(g, K, z, acc); p1k_diag_tet<T, 1, 1>(g, K, z, acc);
  p1k_diag_tet<T, 1, 2>(g, K, z, acc); p1k_diag_tet<T, 1, 3>(g, K, z, acc);
  p1k_diag_tet<T, 2, 0>(g, K, z, acc); p1k_diag_tet<T, 2, 1>(g, K, z, acc);
  p1k_diag_tet<T, 2, 2>(g, K, z, acc); p1k_diag_tet<T, 2, 3>(g, K, z, acc);
  p1k_diag_tet<T, 3, 0>(g, K, z, acc); p1k_diag_tet<T, 3, 1>(g, K, z, acc);
  p1k_diag_tet<T, 3, 2>(g, K, z, acc); p1k_diag_tet<T, 3, 3>(g, K, z, acc);
  p1k_diag_tet<T, 4, 0>(g, K, z, acc); p1k_diag_tet<T, 4, 1>(g, K, z, acc);
  p1k_diag_tet<T, 4, 2>(g, K, z, acc); p1k_diag_tet<T, 4, 3>(g, K, z, acc);
  p1k_diag_tet<T, 5, 0>(g, K, z, acc); p1k_diag_tet<T, 5, 1>(g, K, z, acc);
  p1k_diag_tet<T, 5, 2>(g, K, z, acc); p1k_diag_tet<T, 5, 3>(g, K, z, acc);
  return acc;
}

// 1/4 (D gy)_T . Gp_T (D x)_T summed over the existing micro-tets containing p
// (DR, DX centred gy and x; ALL as in p1k_tet)
template <typename T, int t, int a, bool ALL>
__device__ __forceinline__ void kgrad_tet(GeoPtr<T> g, const T DR[3][7], const T DX[3][7], int z, T &acc) {
  T bil = T(0);
#pragma unroll
  for (int c1 = 0; c1 < 4; ++c1)
#pragma unroll
    for (int c2 = c1 + 1; c2 < 4; ++c2) {
      const int q1 = kVS.v[t][a][c1], q2 = kVS.v[t][a][c2];
      bil -= goff(g, t, c1, c2) * (nbval(DR, q1) - nbval(DR, q2)) * (nbval(DX, q1) - nbval(DX, q2));
    }
  if constexpr (ALL)
    acc += bil;
  else
    acc += tet_exists<t, a>(z) ? bil : T(0);
}

template <typename T, bool ALL>
__device__ __forceinline__ T kgrad_row(GeoPtr<T> g, const T R[3][7], const T X[3][7], int z) {
  T DR[3][7], DX[3][7];
  centred(R, DR);
  centred(X, DX);
  T acc = T(0);
  kgrad_tet<T, 0, 0, ALL>(g, DR, DX, z, acc); kgrad_tet<T, 0, 1, ALL>(g, DR, DX, z, acc);
  kgrad_tet<T, 0, 2, ALL>(g, DR, DX, z, acc); kgrad_tet<T, 0, 3, ALL>(g, DR, DX, z, acc);
  kgrad_tet<T, 1, 0, ALL>(g, DR, DX, z, acc); kgrad_tet<T, 1, 1, ALL>(g, DR, DX, z, acc);
  kgrad_tet<T, 1, 2, ALL>(g, DR, DX, z, acc); kgrad_tet<T, 1, 3, ALL>(g, DR, DX, z, acc);
  kgrad_tet<T, 2, 0, ALL>(g, DR, DX, z, acc); kgrad_tet<T, 2, 1, ALL>(g, DR, DX, z, acc);
  kgrad_tet<T, 2, 2, ALL>(g, DR, DX, z, acc); kgrad_tet<T, 2, 3, ALL>(g, DR, DX, z, acc);
  kgrad_tet<T, 3, 0, ALL>(g, DR, DX, z, acc); kgrad_tet<T, 3, 1, ALL>(g, DR, DX, z, acc);
  kgrad_tet<T, 3, 2, ALL>(g, DR, DX, z, acc); kgrad_tet<T, 3, 3, ALL>(g, DR, DX, z, acc);
  kgrad_tet<T, 4, 0, ALL>(g, DR, DX, z, acc); kgrad_tet<T, 4, 1, ALL>(g, DR, DX, z, acc);
  kgrad_tet<T, 4, 2, ALL>(g, DR, DX, z, acc); kgrad_tet<T, 4, 3, ALL>(g, DR, DX, z, acc);
  kgrad_tet<T, 5, 0, ALL>(g, DR, DX, z, acc); kgrad_tet<T, 5, 1, ALL>(g, DR, DX, z, acc);
  kgrad_tet<T, 5, 2, ALL>(g, DR, DX, z, acc); kgrad_tet<T, 5, 3, ALL>(g, DR, DX, z, acc);
  return acc * T(0.25);
}

// Row march.  Window of one field at step j (values at i = i0 - 1 + lane):
//   c[0] = row (j-1, k), c[1] = (j, k), c[2] = (j+1, k)
//   u[0] = row (j-1, k+1), u[1] = (j, k+1)
//   d[0] = row (j, k-1), d[1] = (j+1, k-1)
// Entering rows at step j+1: (j+2, k), (j+1, k+1), (j+2, k-1).
template <typename T>
struct Window {
  T c[3], u[2], d[2];
};

// Whole-wavefront shifts by one lane as DPP moves (wave_shl:1 / wave_shr:1,
// GFX9 data-parallel controls): a VALU move per dword, where a generic shuffle
// goes through the LDS crossbar (ds_bpermute) and waits on it.  The lane that
// has no source (63 for the left shift, 0 for the right) receives 0; those
// two lanes are halo lanes and produce no output.
typedef unsigned int U32x2 __attribute__((ext_vector_type(2)));
constexpr int kDppWaveShl1 = 0x130, kDppWaveShr1 = 0x138;
template <int CTRL>
__device__ __forceinline__ double wave_shift(double v) {
  const U32x2 p = __builtin_bit_cast(U32x2, v);
  U32x2 r;
  r.x = static_cast<unsigned>(__builtin_amdgcn_update_dpp(0, static_cast<int>(p.x), CTRL, 0xF, 0xF, true));
  r.y = static_cast<unsigned>(__builtin_amdgcn_update_dpp(0, static_cast<int>(p.y), CTRL, 0xF, 0xF, true));
  return __builtin_bit_cast(double, r);
}
template <int CTRL>
__device__ __forceinline__ float wave_shift(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
// value of lane + 1 / lane - 1
template <typename T>
__device__ __forceinline__ T from_next(T v) { return wave_shift<kDppWaveShl1>(v); }
template <typename T>
__device__ __forceinline__ T from_prev(T v) { return wave_shift<kDppWaveShr1>(v); }

// the 15-point neighbourhood of each lane's point, in the slot layout of
// kNbPlane / kNbSlot (in-plane offsets (0,0) (1,0) (-1,0) (0,1) (0,-1) (1,-1)
// (-1,1)); i + 1 comes from lane + 1, i - 1 from lane - 1
template <typename T>
__device__ __forceinline__ void neighbourhood(const Window<T> &w, T P[3][7]) {
  P[1][0] = w.c[1];
  P[1][1] = from_next(w.c[1]);
  P[1][2] = from_prev(w.c[1]);
  P[1][3] = w.c[2];
  P[1][6] = from_prev(w.c[2]);
  P[1][4] = w.c[0];
  P[1][5] = from_next(w.c[0]);
  P[2][0] = w.u[1];
  P[2][2] = from_prev(w.u[1]);
  P[2][4] = w.u[0];
  P[2][5] = from_next(w.u[0]);
  P[0][0] = w.d[0];
  P[0][1] = from_next(w.d[0]);
  P[0][3] = w.d[1];
  P[0][6] = from_prev(w.d[1]);
  // slots no 15-point neighbour uses
  P[2][1] = P[2][3] = P[2][6] = T(0);
  P[0][2] = P[0][4] = P[0][5] = T(0);
}

// Buffer resources over one macro block.  The hardware range check of buffer
// instructions turns an access at an offset past the block into a load of 0
// or a dropped store, so out-of-lattice lanes need no branch: every step issues
// the same loads and stores, and the wait for rows prefetched two steps earlier
// can leave the newer loads in flight.
using Rsrc = __amdgpu_buffer_rsrc_t;
constexpr int kFar = 0x7fffff00;  // byte offset past any block (blocks are < 2^31 bytes)
template <typename T>
__device__ __forceinline__ Rsrc block_rsrc(const T *p, int points) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(p), 0, points * static_cast<int>(sizeof(T)), 0x00020000);
}
__device__ __forceinline__ double buf_load(double, Rsrc r, int off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ float buf_load(float, Rsrc r, int off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
// outputs are written once and not read again by the kernel: non-temporal
// stores (cache policy bit NT) keep them from evicting input rows from L2
constexpr int kStoreNT = 2;
__device__ __forceinline__ void buf_store(double v, Rsrc r, int off) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U32x2, v), r, off, 0, kStoreNT);
}
__device__ __forceinline__ void buf_store(float v, Rsrc r, int off) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, 0, kStoreNT);
}
// byte offset of point (i, j, k) of the block, or kFar if `ok` is false
template <typename T>
__device__ __forceinline__ int point_off(bool ok, int i, int j, int k, int N) {
  return ok ? (row_base(j, k, N) + i) * static_cast<int>(sizeof(T)) : kFar;
}

// Loads of one lattice row (j, k) of one macro at i = i0 - 1 + lane: 0 outside
// the lattice and, with MASK, at Dirichlet DoFs.  j and k are wave-uniform.
template <typename T, bool MASK>
__device__ __forceinline__ T row_load(Rsrc v, int i, int j, int k, int N, uint32_t dmask) {
  const bool row_ok = j >= 0 && k >= 0 && j + k <= N;
  const int lim = N - j - k;
  bool ok = row_ok && i >= 0 && i <= lim;
  if (MASK) ok = ok && !((dmask >> ((i == lim) | ((i == 0) << 1) | ((j == 0) << 2) | ((k == 0) << 3))) & 1u);
  return buf_load(T(0), v, point_off<T>(ok, i, j, k, N));
}

template <typename T, bool MASK>
__device__ __forceinline__ void window_init(Window<T> &w, Rsrc v, int i, int j, int k, int N, uint32_t dm) {
  w.c[0] = row_load<T, MASK>(v, i, j - 1, k, N, dm);
  w.c[1] = row_load<T, MASK>(v, i, j, k, N, dm);
  w.u[0] = row_load<T, MASK>(v, i, j - 1, k + 1, N, dm);
  w.d[0] = row_load<T, MASK>(v, i, j, k - 1, N, dm);
}
// the three rows entering at step j
template <typename T, bool MASK>
__device__ __forceinline__ void window_next(T nx[3], Rsrc v, int i, int j, int k, int N, uint32_t dm) {
  nx[0] = row_load<T, MASK>(v, i, j + 1, k, N, dm);
  nx[1] = row_load<T, MASK>(v, i, j, k + 1, N, dm);
  nx[2] = row_load<T, MASK>(v, i, j + 1, k - 1, N, dm);
}
template <typename T>
__device__ __forceinline__ void window_enter(Window<T> &w, const T nx[3]) {
  w.c[2] = nx[0];
  w.u[1] = nx[1];
  w.d[1] = nx[2];
}
template <typename T>
__device__ __forceinline__ void window_slide(Window<T> &w) {
  w.c[0] = w.c[1];
  w.c[1] = w.c[2];
  w.u[0] = w.u[1];
  w.d[0] = w.d[1];
}

// Work unit (k, i0, j0, j1): rows j0 .. j1-1 of plane k, points i0 .. i0+61.
// Workgroups are dealt round-robin to the 8 XCDs (each with its own L2);
// renumbered so that XCD x runs one contiguous run of the (macro, unit block)
// sequence in order, neighbouring rows and planes meet in the same L2.
struct Unit {
  int m, k, i0, j0, j1;
  bool valid;
};
__device__ __forceinline__ Unit unit_of(const int4 *__restrict__ units, int nunits) {
  const int per_macro = (nunits + 3) / 4;
  const int nb = gridDim.x, b = blockIdx.x;
  const int x8 = b & 7, q = nb >> 3, rem = nb & 7;
  const int t = x8 * q + min(x8, rem) + (b >> 3);
  Unit u;
  u.m = t / per_macro;
  const int id = __builtin_amdgcn_readfirstlane((t - u.m * per_macro) * 4 + (threadIdx.x >> 6));
  u.valid = id < nunits;
  const int4 w = units[u.valid ? id : 0];
  u.k = __builtin_amdgcn_readfirstlane(w.x);
  u.i0 = __builtin_amdgcn_readfirstlane(w.y);
  u.j0 = __builtin_amdgcn_readfirstlane(w.z);
  u.j1 = __builtin_amdgcn_readfirstlane(w.w);
  return u;
}
constexpr int kUnitPoints = 62;  // output points per wavefront row

// KIND P1_DIVKGRAD: y = A(k) x; P1_DIVKGRAD_DIAG: y = diag(A(k)) (no x read)
template <typename T, int KIND>
__global__ __launch_bounds__(256) void k_p1_apply(P1Args<T> a, const int4 *__restrict__ units, int nunits) {
  constexpr bool VARK = KIND == P1_DIVKGRAD || KIND == P1_DIVKGRAD_DIAG;
  constexpr bool DIAG = KIND == P1_DIVKGRAD_DIAG;
  const LatticeArgs<T> &L = a.lat;
  const Unit U = unit_of(units, nunits);
  // the macro's 16 boundary-class stencils (all units of a workgroup share
  // the macro); staged before any wavefront can leave
  __shared__ T sw[VARK ? 1 : 16 * 15];
  if (!VARK) {
    for (int e = threadIdx.x; e < 16 * 15; e += 256) sw[e] = a.w15[16 * 15 * U.m + e];
    __syncthreads();
  }
  if (!U.valid) return;
  const int N = L.N, k = U.k, lane = threadIdx.x & 63, i = U.i0 - 1 + lane;
  const int64_t base = static_cast<int64_t>(U.m) * L.L;
  const uint32_t bnd = L.bnd[U.m];
  const uint32_t dm = L.dirichlet ? bnd : 0u;
  const Rsrc x = block_rsrc(a.x + base, L.L);
  const Rsrc kc = block_rsrc(VARK ? a.k + base : a.x + base, VARK ? L.L : 0);
  const Rsrc y = block_rsrc(a.y + base, L.L);
  const GeoPtr<T> g = (GeoPtr<T>)(L.geo + 6 * U.m);
  const bool out_lane = lane >= 1 && lane <= kUnitPoints;
  // class-0 stencil (all 24 micro-tets present)
  const auto *w0 = (const __attribute__((address_space(4))) T *)(a.w15 + 16 * 15 * U.m);

  // rows entering at step j were loaded at step j - PD.  With PD = 2 the two
  // prefetch buffers alternate between even and odd steps (loads are always
  // issued; past the segment end they read masked zeros), so the wait for one
  // buffer leaves the other's loads in flight.  The variable-coefficient form
  // keeps PD = 1: its second field and element code need the registers.
  constexpr int PD = VARK ? 1 : 2;
  Window<T> X, K;
  T nx[PD][3], nk[PD][3];
  if (!DIAG) window_init<T, true>(X, x, i, U.j0, k, N, dm);
  if (VARK) window_init<T, false>(K, kc, i, U.j0, k, N, 0u);
#pragma unroll
  for (int b = 0; b < PD; ++b) {
    if (!DIAG) window_next<T, true>(nx[b], x, i, U.j0 + b, k, N, dm);
    if (VARK) window_next<T, false>(nk[b], kc, i, U.j0 + b, k, N, 0u);
  }
  auto step = [&](int j, T(&nxb)[3], T(&nkb)[3]) {
    if (!DIAG) window_enter(X, nxb);
    if (VARK) window_enter(K, nkb);
    if (!DIAG) window_next<T, true>(nxb, x, i, j + PD, k, N, dm);
    if (VARK) window_next<T, false>(nkb, kc, i, j + PD, k, N, 0u);
    T PX[3][7];
    if (!DIAG) neighbourhood(X, PX);
    const int z = zero_pattern(i, j, k, N);
    const bool out = out_lane && i <= N - j - k;
    T acc = T(0);
    if (DIAG) {
      T PK[3][7];
      neighbourhood(K, PK);
      acc = p1k_diag(g, PK, z);
    } else if (VARK) {
      T PK[3][7];
      neighbourhood(K, PK);
      // wavefront-uniform: all output points interior -> no per-tet tests
      acc = __ballot(out && z != 0) == 0 ? p1k_row<T, true>(g, PX, PK, z) : p1k_row<T, false>(g, PX, PK, z);
    } else if (__ballot(out && z != 0) == 0) {
      // every output point of the row segment lies inside the macro
#pragma unroll
      for (int q = 0; q < 15; ++q) acc += w0[q] * nbval(PX, q);
    } else {
      const T *w = sw + 15 * z;
#pragma unroll
      for (int q = 0; q < 15; ++q) acc += w[q] * nbval(PX, q);
    }
    if ((dm >> z) & 1u) acc = T(0);
    buf_store(acc, y, point_off<T>(out, i, j, k, N));
    if (!DIAG) window_slide(X);
    if (VARK) window_slide(K);
  };
  for (int j = U.j0; j < U.j1; j += PD) {
    step(j, nx[0], nk[0]);
    if (PD == 2 && j + 1 < U.j1) step(j + 1, nx[PD - 1], nk[PD - 1]);
  }
}

// Constant-coefficient stencil, 2.5-D blocking: a wavefront owns a tile of
// KJ rows x 62 points (rows j0 .. j0+KJ-1, points i0 .. i0+61) and marches
// through planes k0 .. k1-1 (4 planes: short marches keep many wavefronts,
// and so many loads, in flight).  It holds plane k's rows j0-1 .. j0+KJ, plane
// k-1's rows j0 .. j0+KJ and plane k+1's rows j0-1 .. j0+KJ-1; a step to
// plane k+1 loads KJ + 2 rows (plane k+2's KJ + 1, plane k+1's row j0+KJ)
// for KJ output rows, issued one step ahead.
constexpr int KJ = kStencilRows;
template <typename T>
__global__ __launch_bounds__(256) void k_p1_stencil(P1Args<T> a, const int4 *__restrict__ units, int nunits) {
  const LatticeArgs<T> &L = a.lat;
  const Unit U0 = unit_of(units, nunits);
  __shared__ T sw[16 * 15];
  for (int e = threadIdx.x; e < 16 * 15; e += 256) sw[e] = a.w15[16 * 15 * U0.m + e];
  __syncthreads();
  if (!U0.valid) return;
  // unit fields: (j0, i0, k0, k1)
  const int j0 = U0.k, i0 = U0.i0, k0 = U0.j0, k1 = U0.j1;
  const int N = L.N, lane = threadIdx.x & 63, i = i0 - 1 + lane;
  const int64_t base = static_cast<int64_t>(U0.m) * L.L;
  const uint32_t dm = L.dirichlet ? L.bnd[U0.m] : 0u;
  const Rsrc x = block_rsrc(a.x + base, L.L);
  const Rsrc y = block_rsrc(a.y + base, L.L);
  const bool out_lane = lane >= 1 && lane <= kUnitPoints;
  const auto *w0 = (const __attribute__((address_space(4))) T *)(a.w15 + 16 * 15 * U0.m);

  T A[KJ + 2], B[KJ + 1], C[KJ + 1];  // plane k rows j0-1.., plane k-1 rows j0.., plane k+1 rows j0-1..
  T nC[KJ + 1], nA;                   // next step: plane k+2 rows j0-1.., plane k+1 row j0+KJ
#pragma unroll
  for (int r = 0; r < KJ + 2; ++r) A[r] = row_load<T, true>(x, i, j0 - 1 + r, k0, N, dm);
#pragma unroll
  for (int r = 0; r < KJ + 1; ++r) {
    B[r] = row_load<T, true>(x, i, j0 + r, k0 - 1, N, dm);
    C[r] = row_load<T, true>(x, i, j0 - 1 + r, k0 + 1, N, dm);
  }
  for (int k = k0; k < k1; ++k) {
    // plane k+1's missing row and plane k+2, in flight during this step
    nA = row_load<T, true>(x, i, j0 + KJ, k + 1, N, dm);
#pragma unroll
    for (int r = 0; r < KJ + 1; ++r) nC[r] = row_load<T, true>(x, i, j0 - 1 + r, k + 2, N, dm);
#pragma unroll
    for (int r = 0; r < KJ; ++r) {
      const int j = j0 + r;
      Window<T> w;
      w.c[0] = A[r];
      w.c[1] = A[r + 1];
      w.c[2] = A[r + 2];
      w.d[0] = B[r];
      w.d[1] = B[r + 1];
      w.u[0] = C[r];
      w.u[1] = C[r + 1];
      T P[3][7];
      neighbourhood(w, P);
      const int z = zero_pattern(i, j, k, N);
      const bool out = out_lane && i <= N - j - k;
      T acc = T(0);
      if (__ballot(out && z != 0) == 0) {
#pragma unroll
        for (int q = 0; q < 15; ++q) acc += w0[q] * nbval(P, q);
      } else {
        const T *wz = sw + 15 * z;
#pragma unroll
        for (int q = 0; q < 15; ++q) acc += wz[q] * nbval(P, q);
      }
      if ((dm >> z) & 1u) acc = T(0);
      buf_store(acc, y, point_off<T>(out, i, j, k, N));
    }
    // slide to plane k+1
#pragma unroll
    for (int r = 0; r < KJ + 1; ++r) B[r] = A[r + 1];
#pragma unroll
    for (int r = 0; r < KJ + 1; ++r) A[r] = C[r];
    A[KJ + 1] = nA;
#pragma unroll
    for (int r = 0; r < KJ + 1; ++r) C[r] = nC[r];
  }
}

// Diagonal of the constant-coefficient operator: the centre weight of the
// point's boundary-class stencil (0 on Dirichlet rows), over the stencil
// tiles of k_p1_stencil
template <typename T>
__global__ __launch_bounds__(256) void k_p1_stencil_diag(P1Args<T> a, const int4 *__restrict__ units, int nunits) {
  const LatticeArgs<T> &L = a.lat;
  const Unit U0 = unit_of(units, nunits);
  if (!U0.valid) return;
  const int j0 = U0.k, i0 = U0.i0, k0 = U0.j0, k1 = U0.j1;
  const int N = L.N, lane = threadIdx.x & 63, i = i0 - 1 + lane;
  const int64_t base = static_cast<int64_t>(U0.m) * L.L;
  const uint32_t dm = L.dirichlet ? L.bnd[U0.m] : 0u;
  const Rsrc y = block_rsrc(a.y + base, L.L);
  const bool out_lane = lane >= 1 && lane <= kUnitPoints;
  const auto *w = (const __attribute__((address_space(4))) T *)(a.w15 + 16 * 15 * U0.m);
  for (int k = k0; k < k1; ++k)
#pragma unroll
    for (int r = 0; r < KJ; ++r) {
      const int j = j0 + r;
      const bool out = out_lane && i >= 0 && j + k <= N && i <= N - j - k;
      const int z = out ? zero_pattern(i, j, k, N) : 0;
      const T d = ((dm >> z) & 1u) ? T(0) : w[15 * z];
      buf_store(d, y, point_off<T>(out, i, j, k, N));
    }
}

// Fused reverse mode of the macro-local P1 div(k grad) apply:
//   gx_p = (L(k) gy)_p,  gk_p = sum_{T containing p} 1/4 (D gy)_T . Gp_T (D x)_T
template <typename T>
__global__ __launch_bounds__(256) void k_p1_adjoint(P1AdjArgs<T> a, const int4 *__restrict__ units, int nunits) {
  const LatticeArgs<T> &L = a.lat;
  const Unit U = unit_of(units, nunits);
  if (!U.valid) return;
  const int N = L.N, k = U.k, lane = threadIdx.x & 63, i = U.i0 - 1 + lane;
  const int64_t base = static_cast<int64_t>(U.m) * L.L;
  const uint32_t bnd = L.bnd[U.m];
  const uint32_t dm = L.dirichlet ? bnd : 0u;
  const Rsrc gy = block_rsrc(a.gy + base, L.L), x = block_rsrc(a.x + base, L.L), kc = block_rsrc(a.k + base, L.L);
  const Rsrc gxr = block_rsrc(a.gx + base, L.L);
  const Rsrc gkr = block_rsrc(a.gk ? a.gk + base : a.gx + base, a.gk ? L.L : 0);  // no gk: every store dropped
  const GeoPtr<T> g = (GeoPtr<T>)(L.geo + 6 * U.m);
  const bool out_lane = lane >= 1 && lane <= kUnitPoints;

  // three fields: rows entering at step j are loaded at step j - 1
  Window<T> G, X, K;
  T ng[3], nx[3], nk[3];
  window_init<T, true>(G, gy, i, U.j0, k, N, dm);
  window_init<T, true>(X, x, i, U.j0, k, N, dm);
  window_init<T, false>(K, kc, i, U.j0, k, N, 0u);
  window_next<T, true>(ng, gy, i, U.j0, k, N, dm);
  window_next<T, true>(nx, x, i, U.j0, k, N, dm);
  window_next<T, false>(nk, kc, i, U.j0, k, N, 0u);
  for (int j = U.j0; j < U.j1; ++j) {
    window_enter(G, ng);
    window_enter(X, nx);
    window_enter(K, nk);
    window_next<T, true>(ng, gy, i, j + 1, k, N, dm);
    window_next<T, true>(nx, x, i, j + 1, k, N, dm);
    window_next<T, false>(nk, kc, i, j + 1, k, N, 0u);
    T PG[3][7], PX[3][7], PK[3][7];
    neighbourhood(G, PG);
    neighbourhood(X, PX);
    neighbourhood(K, PK);
    const int z = zero_pattern(i, j, k, N);
    const bool out = out_lane && i <= N - j - k;
    // (one body for all points: an interior-only copy beside it raised the
    // kernel from 241 to 384 VGPRs)
    const T gx = ((dm >> z) & 1u) ? T(0) : p1k_row<T, false>(g, PG, PK, z);
    const T gk = kgrad_row<T, false>(g, PG, PX, z);
    const int off = point_off<T>(out, i, j, k, N);
    buf_store(gx, gxr, off);
    buf_store(gk, gkr, off);
    window_slide(G);
    window_slide(X);
    window_slide(K);
  }
}

}  // namespace

template <typename T>
hipError_t launch_p1_apply(const P1Args<T> &a, int kind, const int4 *units, int nunits, hipStream_t s) {
  const dim3 grid(((nunits + 3) / 4) * a.lat.nt);
  switch (kind) {
    case P1_LAPLACE: hipLaunchKernelGGL((k_p1_stencil<T>), grid, dim3(256), 0, s, a, units, nunits); break;
    case P1_DIVKGRAD: hipLaunchKernelGGL((k_p1_apply<T, P1_DIVKGRAD>), grid, dim3(256), 0, s, a, units, nunits); break;
    case P1_LAPLACE_DIAG: hipLaunchKernelGGL((k_p1_stencil_diag<T>), grid, dim3(256), 0, s, a, units, nunits); break;
    case P1_DIVKGRAD_DIAG:
      hipLaunchKernelGGL((k_p1_apply<T, P1_DIVKGRAD_DIAG>), grid, dim3(256), 0, s, a, units, nunits);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_p1_adjoint(const P1AdjArgs<T> &a, const int4 *units, int nunits, hipStream_t s) {
  const dim3 grid(((nunits + 3) / 4) * a.lat.nt);
  hipLaunchKernelGGL((k_p1_adjoint<T>), grid, dim3(256), 0, s, a, units, nunits);
  return hipGetLastError();
}

template hipError_t launch_p1_apply<double>(const P1Args<double> &, int, const int4 *, int, hipStream_t);
template hipError_t launch_p1_apply<float>(const P1Args<float> &, int, const int4 *, int, hipStream_t);
template hipError_t launch_p1_adjoint<double>(const P1AdjArgs<double> &, const int4 *, int, hipStream_t);
template hipError_t launch_p1_adjoint<float>(const P1AdjArgs<float> &, const int4 *, int, hipStream_t);

}  // namespace tmf
