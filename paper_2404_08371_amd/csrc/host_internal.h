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
  int classic_cfg = 0;  // box shape for the modes the marching kernel does not provide
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
  // P2 tiles: seam points of one macro lattice and tile-row starts, per tile
  // shape; partial sums of the seam points (operator scratch)
  DevBuf<int> seam[kNumTileCfg], rowstart[kNumTileCfg];
  int nseam[kNumTileCfg] = {0}, nby[kNumTileCfg] = {0}, tpm[kNumTileCfg] = {0};
  DevBuf<uint8_t> partial;
  size_t partial_bytes[kNumTileCfg] = {0};  // partial sums of one apply, per tile shape
  DevBuf<uint8_t> seaminst[kNumTileCfg];  // one SeamInst of the op's precision
  DevBuf<int4> seamwork[kNumTileCfg];     // interface-group entries, then seam entries
  int nseamwork[kNumTileCfg] = {0}, nseamonly[kNumTileCfg] = {0}, ngroupwork[kNumTileCfg] = {0};
  DevBuf<uint32_t> shared;                // per macro: zero patterns with copies in other macros
  DevBuf<int64_t> gpos;                   // per interface-group member: macro << 32 | packed lattice point
  DevBuf<int> gpl;                        // per interface-group member: position << 16 | group size
  DevBuf<int8_t> sign;                    // N1: per slot, global / lattice orientation of its edge (0: vertex)
  DevBuf<uint8_t> mat;                    // stored local matrices (tmf_op_store_matrices)
  int mat_cfg = -1;                       // tile shape they were stored for (-1: none)
  int seamrows[kNumTileCfg] = {0};        // tile-row table entries per macro, per tile shape
};

// tile shape of an element-kernel launch: the chosen shape, or the chosen box
// shape when the chosen one is a marching shape and the mode is not a plain
// scalar P2 apply
inline int mode_cfg(int cfg, int box_cfg, int mode) {
  const bool plain = mode == TMF_P2_LAPLACE || mode == TMF_P2_DIVKGRAD;
  return (kTileMarch[cfg] != 0 && !plain) ? box_cfg : cfg;
}

// seam-reduction descriptor of an op with tile shape `cfg` at offset `yoff`
template <typename T>
inline SeamInst<T> seam_inst(const tmf_op *op, int cfg, int64_t yoff) {
  SeamInst<T> a;
  a.pts = op->seam[cfg].p;
  a.npts = op->nseam[cfg];
  a.rowstart = op->rowstart[cfg].p;
  a.nby = op->nby[cfg];
  a.tpm = op->tpm[cfg];
  a.n = op->mesh->n;
  a.N = op->N;
  a.L = static_cast<int>(op->L);
  a.dirichlet = op->bc == TMF_BC_DIRICHLET_ZERO;
  a.n_local = op->n_local;
  a.yoff = yoff;
  a.bnd = op->bnd.p;
  a.partial = reinterpret_cast<const T *>(op->partial.p);
  a.shared = op->shared.p;
  a.gidx = op->gidx.p;
  a.gpos = op->gpos.p;
  a.gpl = op->gpl.p;
  return a;
}

// seam points per thread of an op's seam work entries
inline int seam_ppt(const tmf_op *op) { return op->ncomp == 1 ? kSeamPointsPerThread : 1; }
// seam work entries (instance, macro, first point, 0) of an op
inline void seam_work(const tmf_op *op, int cfg, int inst, std::vector<int4> &w) {
  const int chunk = 256 * seam_ppt(op);
  for (int64_t m = 0; m < op->mesh->nt; ++m)
    for (int p0 = 0; p0 < op->nseam[cfg]; p0 += chunk) w.push_back(make_int4(inst, static_cast<int>(m), p0, 0));
}
// interface work entries (instance, first member, end member, 1) of an op:
// whole groups, at most 256 members per entry
inline void group_work(const tmf_op *op, int inst, std::vector<int4> &w) {
  const std::vector<int64_t> &gp = op->mesh->sp[op->space].gptr;
  int64_t q0 = 0;
  for (size_t g = 0; g + 1 < gp.size(); ++g) {
    if (gp[g + 1] - q0 > 256) {
      w.push_back(make_int4(inst, static_cast<int>(q0), static_cast<int>(gp[g]), 1));
      q0 = gp[g];
    }
  }
  if (gp.size() > 1 && gp.back() > q0) w.push_back(make_int4(inst, static_cast<int>(q0), static_cast<int>(gp.back()), 1));
}
// tile-row table entries staged in LDS by the seam reduction (0: read from global memory)
inline int seam_rows_lds(int nrows) { return nrows <= kSeamRowsLds ? nrows : 0; }

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
  d.sign = op->sign.p;
  d.partial = reinterpret_cast<T *>(op->partial.p);
  d.geo = reinterpret_cast<const TypeGeo<T> *>(op->geo.p);
  d.mgeo = reinterpret_cast<const MacroGeo<T> *>(op->mgeo.p);
  return d;
}


namespace tmf {
// autotuner cache (tune_cache.cpp): device tag "<arch>/<CUs>cu"; lookup returns
// 1 (found: cfg, box shape and time set), 0 (not found) or -1 (unreadable file)
std::string device_tag();
int tune_cache_lookup(const char *path, const std::string &key, int *cfg, int *box, float *ms);
tmf_status tune_cache_store(const char *path, const std::string &key, int cfg, int box, float ms);

inline bool has_coeff(int kind) {
  return kind == TMF_P1_DIVKGRAD || kind == TMF_P2_DIVKGRAD || kind == TMF_P2V_EPSILON || kind == TMF_N1_CURLCURL;
}
}  // namespace tmf
