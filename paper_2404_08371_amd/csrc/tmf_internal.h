// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tmf {

// ---------------------------------------------------------------------------
// The six micro-tetrahedron types of a uniformly refined macro-tetrahedron
// (section "Hybrid Tetrahedral Grids": every micro-tet is a translate of one
// of six reference shapes).  In the index space of the macro, a micro-cube
// with base b holds up to six tets with these vertex offsets; type t exists
// iff b >= 0 and b.x + b.y + b.z <= n - kLim[t].  The exclusive loop bounds of
// the sawtooth strategy give the same counts: C(n+2,3) white-up, C(n+1,3)
// for each of the four middle types, C(n,3) white-down.
// Order: white-up, four octahedron types, white-down.
constexpr int kOff[6][4][3] = {
    {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}},
    {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 0, 1}},
    {{1, 0, 0}, {0, 1, 0}, {1, 1, 0}, {1, 0, 1}},
    {{0, 1, 0}, {0, 0, 1}, {1, 0, 1}, {0, 1, 1}},
    {{0, 1, 0}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}},
    {{1, 1, 0}, {1, 0, 1}, {0, 1, 1}, {1, 1, 1}},
};
constexpr int kLim[6] = {1, 2, 2, 2, 2, 3};
// local edge order of the P2 edge DoFs of a tet
constexpr int kEdge[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

// The 15-point neighbourhood of a lattice vertex (itself + 14 neighbours).
constexpr int kNb[15][3] = {
    {0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1}, {1, -1, 0},
    {-1, 1, 0}, {1, 0, -1}, {-1, 0, 1}, {0, 1, -1}, {0, -1, 1}, {1, -1, 1}, {-1, 1, -1},
};

constexpr int nb_slot(int dx, int dy, int dz) {
  for (int s = 0; s < 15; ++s)
    if (kNb[s][0] == dx && kNb[s][1] == dy && kNb[s][2] == dz) return s;
  return -1;
}

// slot of vertex c of type t seen from vertex a of the same tet
constexpr int vslot(int t, int a, int c) {
  return nb_slot(kOff[t][c][0] - kOff[t][a][0], kOff[t][c][1] - kOff[t][a][1],
                 kOff[t][c][2] - kOff[t][a][2]);
}

// Per (macro, type) constants, computed in FP64 on the host.
//   Gp[a][b] = |T| grad(lambda_a) . grad(lambda_b)   (P1 local matrix)
//   grad[a][d] = grad(lambda_a), vol = |T|
//   JT = parametric Jacobian of the micro-tet (columns: edge vectors from vertex 0)
//   Gs = rows 1..3 of Gp / 210 (the P2 div(k grad) element forms its weights
//        scaled by 840 and its sigma scaled by 4, so 4 / 840 is folded in here)
template <typename T>
struct TypeGeo {
  T Gp[16];
  T grad[12];
  T vol;
  T JT[9];
  T Gs[12];
  T pad[2];
};

// Per macro constants for curved maps: parametric origin and Jacobian of the
// macro, octant sign vector.
template <typename T>
struct MacroGeo {
  T v0[3];
  T JM[9];
  T s[3];
  T pad;
};

// Packed tetrahedral lattice of size N: C3(M) = (M+1)(M+2)(M+3)/6 points.
__host__ __device__ inline int c3(int M) { return (M + 1) * (M + 2) * (M + 3) / 6; }
// storage index of the first point of row (j, k)
__host__ __device__ inline int row_base(int j, int k, int N) {
  const int M = N - k;
  return c3(N) - c3(M) + (j * (2 * M + 3 - j)) / 2;
}
// zero pattern of the barycentric coordinates (N-i-j-k, i, j, k): bit f set iff coordinate f is 0
__host__ __device__ inline int zero_pattern(int i, int j, int k, int N) {
  return (N - i - j - k == 0) | ((i == 0) << 1) | ((j == 0) << 2) | ((k == 0) << 3);
}

enum Kind { P1_LAPLACE = 0, P1_DIVKGRAD = 1, P2_LAPLACE = 2, P2_DIVKGRAD = 3, P2V_EPSILON = 4, N1_CURLCURL = 5 };
// element-kernel modes besides the applies: diag(A) of a scalar P2 kind, and
// the coefficient gradients gk_b = gy . (dA/dk_b) x of P2 div(k grad) and of
// the epsilon operator (k = mu)
enum KernelMode {
  P2_LAPLACE_DIAG = 16,
  P2_DIVKGRAD_DIAG = 17,
  P2_DIVKGRAD_GRADK = 18,
  P2V_EPSILON_GRADMU = 19,
  // stored local matrices (the precomputed-matrix comparison): build them
  // from k, or apply them
  P2_DIVKGRAD_STORE = 20,
  P2_STORED_APPLY = 21,
  // P2 div(k grad) with the weights from a quadrature rule (under-integration)
  P2_DIVKGRAD_Q = 22,
  // diag(A) of the P1 kinds and of the epsilon operator
  P1_LAPLACE_DIAG = 23,
  P1_DIVKGRAD_DIAG = 24,
  P2V_EPSILON_DIAG = 25
};
// entries of a stored symmetric 10 x 10 local matrix (upper triangle, row-major)
constexpr int kStoredEntries = 55;

template <typename T>
struct LatticeArgs {
  int n;          // micro-cubes per macro edge, 2^level
  int N;          // lattice size of the DoF space (n or 2n)
  int nt;         // number of macros
  int L;          // lattice points per macro, C3(N)
  int dirichlet;  // 1: zero boundary rows and columns
  const uint32_t *bnd;         // per macro: bit z set if points of zero pattern z are boundary DoFs
  const TypeGeo<T> *geo;       // per macro x 6 types
};

template <typename T>
struct P1Args {
  LatticeArgs<T> lat;
  const T *w15;  // per macro, per boundary class (16): 15-point stencil of the constant-coefficient operator
  const T *k;
  const T *x;
  T *y;
};

template <typename T>
struct P1AdjArgs {
  LatticeArgs<T> lat;
  const T *k;
  const T *x;
  const T *gy;
  T *gx;
  T *gk;
};

// One operator instance as seen by the element kernels (a batch holds many).
template <typename T>
struct InstDesc {
  int n, N, L, dirichlet;       // cubes per macro edge, P2 lattice size, points per macro, BC
  int64_t off;                  // offset of the instance in the concatenated vectors
  int64_t n_local;              // component stride of the instance's vector fields
  const uint32_t *bnd;          // per macro boundary table
  const int8_t *sign;           // N1: per slot, global / lattice orientation of its edge (NULL otherwise)
  const TypeGeo<T> *geo;        // per macro x 6 types
  const MacroGeo<T> *mgeo;      // per macro (curved maps)
  T *partial;                   // tile partial sums of seam points: [tile][component][box point]
};

// tile = (instance, macro, bx0 | by0 << 10 | bz0 << 20, tile id within the instance) in micro-cube units
__host__ __device__ inline int pack_base(int bx, int by, int bz) { return bx | (by << 10) | (bz << 20); }

template <typename T>
struct TileArgs {
  const InstDesc<T> *inst;
  const int4 *tiles;
  int ntiles;
  const uint8_t *active;  // per instance, NULL = all active; tiles of inactive instances are skipped
  const T *qtab;          // quadrature rule: per point [w, bary(4), phi(10)]
  int nq;
  const T *k;
  const T *x;
  const T *x2 = nullptr;  // second staged input (gy of the coefficient-gradient mode)
  T *mat = nullptr;       // stored local matrices [tile][type][entry][cube]
  T *y;
  T *partial = nullptr;   // if set, the tile partial sums go here instead of the instance's own buffer
};

struct GroupArgs {
  const int64_t *ptr;  // CSR of duplicate groups
  const int64_t *idx;  // member slots, ascending
  int64_t ngroups;
  int64_t n_local;
  int ncomp;
};

constexpr int kQStride = 15;  // values per quadrature point in qtab

// Seam and interface reduction, one launch for a whole batch.  y at every
// seam point (a lattice point on a face shared by tile boxes) = the
// fixed-order sum of the partials of the tiles containing it; every copy of a
// DoF shared by several macros = the sum, in ascending slot order, of its
// copies' macro-local values (each from the partials if it is a seam point,
// else the value the element kernel stored).  Work entries: (instance, macro,
// first seam point, 0) per 256 seam points and (instance, first group, 0, 1)
// per 256 interface groups.
template <typename T>
struct SeamInst {
  const int *pts;       // seam points of one macro lattice: qx | qy << 10 | qz << 20
  int npts;
  const int *rowstart;  // first tile id of box row (bz / TZ, by / TY) within a macro
  int nby;              // row stride of rowstart
  int tpm;              // tiles per macro
  int n, N, L, dirichlet;
  int64_t n_local;      // component stride
  int64_t yoff;         // offset of the instance in the concatenated vectors
  const uint32_t *bnd;
  const T *partial;
  // copies of DoFs shared with other macros (interface groups, members ascending)
  const uint32_t *shared;  // per macro: bit z set if points of zero pattern z have copies elsewhere
  const int64_t *gidx;     // per member: macro-local slot
  const int64_t *gpos;     // per member: macro << 32 | qx | qy << 10 | qz << 20
  const int *gpl;          // per member: position in its group << 16 | group size
};

// largest tile-row table staged in LDS by the seam reduction (entries)
constexpr int kSeamRowsLds = 8192;
// seam points per thread of the seam reduction for scalar fields (vector
// fields: 1); a seam work entry covers 256 times this many points
constexpr int kSeamPointsPerThread = 2;

// launchers (kernels.hip); return the HIP error of the launch
template <typename T>
hipError_t launch_p1_apply(const P1Args<T> &a, int kind, const int4 *chunks, int nchunks, hipStream_t s);
template <typename T>
hipError_t launch_p1_adjoint(const P1AdjArgs<T> &a, const int4 *chunks, int nchunks, hipStream_t s);
template <typename T>
hipError_t launch_tile_apply(const TileArgs<T> &a, int kind, int map, int tile_cfg, hipStream_t s);
// flags: kSeamLocal (macro-local result: no interface sums, shared points
// reduced within their macro), kSeamKeepBoundary (Dirichlet DoFs keep their
// sums instead of 0)
constexpr int kSeamLocal = 1, kSeamKeepBoundary = 2;
template <typename T>
// ncomp: components of y; ppt: seam points per thread, as the work list was
// chunked (256 ppt points per seam entry); partial: if set, the tile partial
// sums are read from it instead of each instance's own buffer (one instance)
hipError_t launch_seam_gather(const SeamInst<T> *inst, const int4 *work, int nwork, T *y, const uint8_t *active,
                              int flags, int ncomp, int ppt, int tile_cfg, int rows_lds, hipStream_t s,
                              const T *partial = nullptr);
template <typename T>
hipError_t launch_interface_sum(const GroupArgs &g, T *y, hipStream_t s);
template <typename T>
hipError_t launch_fill(T *p, int64_t n, T v, hipStream_t s);

// rows per wavefront of the constant-coefficient P1 stencil (2.5-D blocking)
constexpr int kStencilRows = 4;

// tile shapes available to the element-centric kernels (micro-cubes per
// tile).  The first kNumClassicTileCfg are boxes staged whole by one
// workgroup; the others are column segments of kTileMarch[cfg] sub-boxes of
// 4 x 4 x 4 cubes walked in z by the persistent marching kernel (scalar P2
// applies only; the other modes of those operators use a box shape).
constexpr int kNumTileCfg = 7;
constexpr int kNumClassicTileCfg = 4;
constexpr int kTileCfg[kNumTileCfg][3] = {{4, 4, 4}, {8, 4, 2}, {8, 4, 4}, {4, 4, 8}, {4, 4, 8}, {4, 4, 16}, {4, 4, 32}};
constexpr int kTileMarch[kNumTileCfg] = {0, 0, 0, 0, 2, 4, 8};

}  // namespace tmf
