// Host-side declarations shared by the runtime sources (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tetmf.h"
#include "tmf_internal.h"

namespace tmf {

tmf_status fail(tmf_status code, const char *fmt, ...);
tmf_status hip_fail(hipError_t e, const char *what);

template <typename T>
struct DevBuf {
  T *p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  tmf_status alloc(size_t count) {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = count;
    if (count == 0) return TMF_OK;
    if (hipMalloc(reinterpret_cast<void **>(&p), count * sizeof(T)) != hipSuccess) {
      p = nullptr;
      return fail(TMF_ENOMEM, "device allocation of %zu bytes failed", count * sizeof(T));
    }
    return TMF_OK;
  }
  tmf_status upload(const void *src, size_t count) {
    tmf_status st = alloc(count);
    if (st != TMF_OK || count == 0) return st;
    hipError_t e = hipMemcpy(p, src, count * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
    return TMF_OK;
  }
};

}  // namespace tmf

using namespace tmf;

struct SpaceLayout {
  bool built = false;
  int N = 0;
  int64_t L = 0, n_local = 0, n_unique = 0;
  std::vector<int64_t> gptr, gidx;  // duplicate groups (size >= 2), members ascending
  std::vector<uint8_t> owner;
};

struct tmf_mesh {
  int level = 0, n = 1, map = 0;
  int64_t nv = 0, nt = 0;
  std::vector<double> V;
  std::vector<int64_t> T;
  std::vector<uint32_t> bnd;  // per macro: boundary bit per zero pattern
  std::vector<double> sgn;    // per macro octant signs (shell map)
  SpaceLayout sp[3];
};


void tmf_build_layout(tmf_mesh *m, int space);

struct tmf_op {
  const tmf_mesh *mesh = nullptr;
  int kind = 0, prec = 0, bc = 0, space = 1, ncomp = 1, N = 1, nq = 0;
  int64_t L = 0, n_local = 0, n_unique = 0;
  int tile_cfg = 0;
  DevBuf<uint8_t> geo, w15, mgeo, qtab;
  DevBuf<uint32_t> bnd;
  DevBuf<int4> tiles[kNumTileCfg];
  int ntiles[kNumTileCfg] = {0};
  DevBuf<int64_t> gptr, gidx;
  int64_t ngroups = 0;
  DevBuf<uint8_t> owner;
  DevBuf<uint8_t> desc;  // one InstDesc of the op's precision
  DevBuf<int4> chunks;   // P1: row-march work units (k, i0, j0, j1) of one macro lattice
  int nchunks = 0;
};

// device descriptor of an op, for the element kernels
template <typename T>
InstDesc<T> make_desc(const tmf_op *op, int64_t off) {
  InstDesc<T> d;
  d.n = op->mesh->n;
  d.N = op->N;
  d.L = static_cast<int>(op->L);
  d.dirichlet = op->bc == TMF_BC_DIRICHLET_ZERO;
  d.off = off;
  d.n_local = op->n_local;
  d.bnd = op->bnd.p;
  d.geo = reinterpret_cast<const TypeGeo<T> *>(op->geo.p);
  d.mgeo = reinterpret_cast<const MacroGeo<T> *>(op->mgeo.p);
  return d;
}


namespace tmf {
inline bool has_coeff(int kind) {
  return kind == TMF_P1_DIVKGRAD || kind == TMF_P2_DIVKGRAD || kind == TMF_P2V_EPSILON;
}
}  // namespace tmf
