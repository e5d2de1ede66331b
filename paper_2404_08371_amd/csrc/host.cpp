// Host runtime and C ABI of the tetmf library.
//
// Mesh creation validates the macro mesh and derives, per macro-tet, the
// boundary classification of its lattice points and the duplicate groups of
// DoFs shared between macro-tets.  Operator creation computes the per-(macro,
// micro-tet type) geometry constants in FP64 (the loop invariants of section
// "Automatic Identification of Loop Invariants": translation invariance makes
// every micro-tet of one type share its Jacobian) and uploads them with the
// tile lists the element kernels walk.  Apply calls only validate and launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "host_internal.h"

using namespace tmf;

namespace tmf {

thread_local std::string g_err;

tmf_status fail(tmf_status code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

tmf_status hip_fail(hipError_t e, const char *what) {
  return fail(TMF_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace tmf

namespace {

using Key = std::array<int64_t, 8>;
struct KeyHash {
  size_t operator()(const Key &k) const {
    uint64_t h = 0x9E3779B97F4A7C15ull;
    for (int64_t v : k) {
      h ^= static_cast<uint64_t>(v) + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
    }
    return static_cast<size_t>(h);
  }
};

// canonical key of lattice point (i,j,k) of a macro with vertex ids g
Key point_key(const int64_t g[4], int i, int j, int k, int N) {
  const int64_t a[4] = {N - i - j - k, i, j, k};
  std::array<std::pair<int64_t, int64_t>, 4> p;
  int n = 0;
  for (int f = 0; f < 4; ++f)
    if (a[f] > 0) p[n++] = {g[f], a[f]};
  std::sort(p.begin(), p.begin() + n);
  Key key;
  for (int q = 0; q < 4; ++q) {
    key[2 * q] = q < n ? p[q].first : -1;
    key[2 * q + 1] = q < n ? p[q].second : 0;
  }
  return key;
}

void inv3(const double J[9], double Ji[9], double *det) {
  Ji[0] = J[4] * J[8] - J[5] * J[7];
  Ji[1] = J[2] * J[7] - J[1] * J[8];
  Ji[2] = J[1] * J[5] - J[2] * J[4];
  Ji[3] = J[5] * J[6] - J[3] * J[8];
  Ji[4] = J[0] * J[8] - J[2] * J[6];
  Ji[5] = J[2] * J[3] - J[0] * J[5];
  Ji[6] = J[3] * J[7] - J[4] * J[6];
  Ji[7] = J[1] * J[6] - J[0] * J[7];
  Ji[8] = J[0] * J[4] - J[1] * J[3];
  *det = J[0] * Ji[0] + J[1] * Ji[3] + J[2] * Ji[6];
  for (int q = 0; q < 9; ++q) Ji[q] /= *det;
}

}  // namespace

void tmf_build_layout(tmf_mesh *m, int space) {
  SpaceLayout &S = m->sp[space];
  if (S.built) return;
  S.N = m->n * space;
  S.L = c3(S.N);
  S.n_local = m->nt * S.L;
  std::unordered_map<Key, std::vector<int64_t>, KeyHash> groups;
  const int N = S.N;
  for (int64_t mac = 0; mac < m->nt; ++mac) {
    const int64_t *g = &m->T[4 * mac];
    for (int k = 0; k <= N; ++k)
      for (int j = 0; j <= N - k; ++j)
        for (int i = 0; i <= N - k - j; ++i) {
          if (zero_pattern(i, j, k, N) == 0) continue;
          groups[point_key(g, i, j, k, N)].push_back(mac * S.L + row_base(j, k, N) + i);
        }
  }
  S.owner.assign(S.n_local, 1);
  std::vector<std::vector<int64_t> *> list;
  for (auto &kv : groups)
    if (kv.second.size() > 1) list.push_back(&kv.second);
  for (auto *v : list) std::sort(v->begin(), v->end());
  std::sort(list.begin(), list.end(),
            [](const std::vector<int64_t> *a, const std::vector<int64_t> *b) { return (*a)[0] < (*b)[0]; });
  S.gptr.assign(1, 0);
  S.gidx.clear();
  int64_t dup = 0;
  for (auto *v : list) {
    for (size_t q = 0; q < v->size(); ++q) {
      S.gidx.push_back((*v)[q]);
      if (q > 0) S.owner[(*v)[q]] = 0;
    }
    dup += static_cast<int64_t>(v->size()) - 1;
    S.gptr.push_back(static_cast<int64_t>(S.gidx.size()));
  }
  S.n_unique = S.n_local - dup;
  S.built = true;
}

extern "C" {

const char *tmf_version(void) { return "tetmf 0.1 (gfx950)"; }
const char *tmf_last_error(void) { return g_err.c_str(); }
const char *tmf_status_string(tmf_status s) {
  switch (s) {
    case TMF_OK: return "ok";
    case TMF_EINVAL: return "invalid argument";
    case TMF_ENOMEM: return "out of memory";
    case TMF_EDEVICE: return "device error";
    case TMF_EUNSUPPORTED: return "unsupported";
    case TMF_ENOTCONV: return "not converged";
    default: return "unknown status";
  }
}

tmf_status tmf_mesh_create(const double *vertices, int64_t nv, const int64_t *tets, int64_t nt,
                           int level, int map, tmf_mesh **out) {
  if (!out) return fail(TMF_EINVAL, "out is NULL");
  *out = nullptr;
  if (!vertices || !tets) return fail(TMF_EINVAL, "vertices or tets is NULL");
  if (nv < 4 || nt < 1) return fail(TMF_EINVAL, "need nv >= 4 and nt >= 1 (got %lld, %lld)",
                                    (long long)nv, (long long)nt);
  if (level < 0 || level > TMF_MAX_LEVEL_P1)
    return fail(TMF_EINVAL, "level %d outside [0, %d]", level, TMF_MAX_LEVEL_P1);
  if (map != TMF_MAP_AFFINE && map != TMF_MAP_SHELL_RADIAL) return fail(TMF_EINVAL, "bad map %d", map);
  for (int64_t q = 0; q < 3 * nv; ++q)
    if (!std::isfinite(vertices[q])) return fail(TMF_EINVAL, "non-finite vertex coordinate");
  double scale = 0;
  for (int64_t q = 0; q < 3 * nv; ++q) scale = std::max(scale, std::fabs(vertices[q]));
  if (scale == 0) return fail(TMF_EINVAL, "all vertices at the origin");
  std::map<std::array<int64_t, 3>, int> faces;
  for (int64_t t = 0; t < nt; ++t) {
    const int64_t *g = tets + 4 * t;
    for (int a = 0; a < 4; ++a) {
      if (g[a] < 0 || g[a] >= nv) return fail(TMF_EINVAL, "tet %lld: vertex id out of range", (long long)t);
      for (int b = 0; b < a; ++b)
        if (g[a] == g[b]) return fail(TMF_EINVAL, "tet %lld: repeated vertex id", (long long)t);
    }
    double J[9];
    for (int d = 0; d < 3; ++d)
      for (int c = 0; c < 3; ++c) J[3 * d + c] = vertices[3 * g[c + 1] + d] - vertices[3 * g[0] + d];
    const double det = J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6]) +
                       J[2] * (J[3] * J[7] - J[4] * J[6]);
    if (!(std::fabs(det) > 1e-12 * scale * scale * scale))
      return fail(TMF_EINVAL, "tet %lld has (nearly) zero volume", (long long)t);
    for (int f = 0; f < 4; ++f) {
      std::array<int64_t, 3> key;
      int q = 0;
      for (int a = 0; a < 4; ++a)
        if (a != f) key[q++] = g[a];
      std::sort(key.begin(), key.end());
      if (++faces[key] > 2) return fail(TMF_EINVAL, "a face is shared by more than two tets");
    }
  }
  auto *m = new (std::nothrow) tmf_mesh;
  if (!m) return fail(TMF_ENOMEM, "host allocation failed");
  m->level = level;
  m->n = 1 << level;
  m->map = map;
  m->nv = nv;
  m->nt = nt;
  m->V.assign(vertices, vertices + 3 * nv);
  m->T.assign(tets, tets + 4 * nt);
  m->sgn.assign(3 * nt, 1.0);
  if (map == TMF_MAP_SHELL_RADIAL) {
    for (int64_t t = 0; t < nt; ++t) {
      const int64_t *g = tets + 4 * t;
      for (int d = 0; d < 3; ++d) {
        double c = 0;
        for (int a = 0; a < 4; ++a) c += vertices[3 * g[a] + d];
        const double s = c >= 0 ? 1.0 : -1.0;
        for (int a = 0; a < 4; ++a)
          if (s * vertices[3 * g[a] + d] < -1e-14 * scale) {
            delete m;
            return fail(TMF_EINVAL, "tet %lld is not inside one coordinate octant", (long long)t);
          }
        m->sgn[3 * t + d] = s;
      }
      for (int a = 0; a < 4; ++a) {
        const double *p = vertices + 3 * g[a];
        if (std::sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]) < 1e-12 * scale) {
          delete m;
          return fail(TMF_EINVAL, "tet %lld touches the origin", (long long)t);
        }
      }
    }
  }
  // domain boundary: faces of a single tet, with their edges and vertices
  std::map<std::vector<int64_t>, bool> bsimp;
  for (auto &kv : faces) {
    if (kv.second != 1) continue;
    const auto &f = kv.first;
    bsimp[{f[0], f[1], f[2]}] = true;
    bsimp[{f[0], f[1]}] = true;
    bsimp[{f[0], f[2]}] = true;
    bsimp[{f[1], f[2]}] = true;
    bsimp[{f[0]}] = true;
    bsimp[{f[1]}] = true;
    bsimp[{f[2]}] = true;
  }
  m->bnd.assign(nt, 0u);
  for (int64_t t = 0; t < nt; ++t) {
    const int64_t *g = tets + 4 * t;
    uint32_t mask = 0;
    for (int z = 1; z < 15; ++z) {
      std::vector<int64_t> s;
      for (int f = 0; f < 4; ++f)
        if (!((z >> f) & 1)) s.push_back(g[f]);
      std::sort(s.begin(), s.end());
      if (bsimp.count(s)) mask |= 1u << z;
    }
    m->bnd[t] = mask;
  }
  *out = m;
  return TMF_OK;
}

void tmf_mesh_destroy(tmf_mesh *mesh) { delete mesh; }

tmf_status tmf_mesh_layout(const tmf_mesh *mesh, int space, int64_t *n_local, int64_t *n_unique) {
  if (!mesh) return fail(TMF_EINVAL, "mesh is NULL");
  if (space != 1 && space != 2) return fail(TMF_EINVAL, "space must be 1 or 2");
  if (space == 2 && mesh->level > TMF_MAX_LEVEL_P2)
    return fail(TMF_EINVAL, "P2 space supports level <= %d", TMF_MAX_LEVEL_P2);
  tmf_build_layout(const_cast<tmf_mesh *>(mesh), space);
  if (n_local) *n_local = mesh->sp[space].n_local;
  if (n_unique) *n_unique = mesh->sp[space].n_unique;
  return TMF_OK;
}

tmf_status tmf_mesh_dof_info(const tmf_mesh *mesh, int space, int64_t *keys, double *xyz, uint8_t *owner,
                             uint8_t *boundary) {
  tmf_status st = tmf_mesh_layout(mesh, space, nullptr, nullptr);
  if (st != TMF_OK) return st;
  const SpaceLayout &S = mesh->sp[space];
  const int N = S.N;
  for (int64_t mac = 0; mac < mesh->nt; ++mac) {
    const int64_t *g = &mesh->T[4 * mac];
    const uint32_t bm = mesh->bnd[mac];
    for (int k = 0; k <= N; ++k)
      for (int j = 0; j <= N - k; ++j)
        for (int i = 0; i <= N - k - j; ++i) {
          const int64_t slot = mac * S.L + row_base(j, k, N) + i;
          if (keys) {
            Key key = point_key(g, i, j, k, N);
            std::memcpy(keys + 8 * slot, key.data(), sizeof(Key));
          }
          if (xyz) {
            const double a[4] = {double(N - i - j - k), double(i), double(j), double(k)};
            double p[3] = {0, 0, 0};
            for (int f = 0; f < 4; ++f)
              for (int d = 0; d < 3; ++d) p[d] += a[f] * mesh->V[3 * g[f] + d];
            for (int d = 0; d < 3; ++d) p[d] /= N;
            if (mesh->map == TMF_MAP_SHELL_RADIAL) {
              const double l1 = std::fabs(p[0]) + std::fabs(p[1]) + std::fabs(p[2]);
              const double l2 = std::sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
              for (int d = 0; d < 3; ++d) p[d] *= l1 / l2;
            }
            for (int d = 0; d < 3; ++d) xyz[3 * slot + d] = p[d];
          }
          if (owner) owner[slot] = S.owner[slot];
          if (boundary) boundary[slot] = (bm >> zero_pattern(i, j, k, N)) & 1u;
        }
  }
  return TMF_OK;
}

}  // extern "C"

namespace {


template <typename T>
void fill_geometry(const tmf_mesh *m, std::vector<TypeGeo<T>> &geo, std::vector<T> &w15,
                   std::vector<MacroGeo<T>> &mg) {
  geo.assign(6 * m->nt, TypeGeo<T>{});
  w15.assign(16 * 15 * m->nt, T(0));
  mg.assign(m->nt, MacroGeo<T>{});
  for (int64_t mac = 0; mac < m->nt; ++mac) {
    const int64_t *g = &m->T[4 * mac];
    double JM[9];
    for (int d = 0; d < 3; ++d)
      for (int c = 0; c < 3; ++c) JM[3 * d + c] = m->V[3 * g[c + 1] + d] - m->V[3 * g[0] + d];
    for (int d = 0; d < 3; ++d) {
      mg[mac].v0[d] = T(m->V[3 * g[0] + d]);
      mg[mac].s[d] = T(m->sgn[3 * mac + d]);
    }
    for (int q = 0; q < 9; ++q) mg[mac].JM[q] = T(JM[q]);
    double w[16][15] = {{0}};
    for (int t = 0; t < 6; ++t) {
      double E[9], J[9], Ji[9], det;
      for (int d = 0; d < 3; ++d)
        for (int c = 0; c < 3; ++c) E[3 * d + c] = kOff[t][c + 1][d] - kOff[t][0][d];
      for (int d = 0; d < 3; ++d)
        for (int c = 0; c < 3; ++c) {
          double s = 0;
          for (int q = 0; q < 3; ++q) s += JM[3 * d + q] * E[3 * q + c];
          J[3 * d + c] = s / m->n;
        }
      inv3(J, Ji, &det);
      const double vol = std::fabs(det) / 6.0;
      double gr[4][3];
      for (int d = 0; d < 3; ++d) {
        gr[1][d] = Ji[0 * 3 + d];
        gr[2][d] = Ji[1 * 3 + d];
        gr[3][d] = Ji[2 * 3 + d];
        gr[0][d] = -(gr[1][d] + gr[2][d] + gr[3][d]);
      }
      TypeGeo<T> &tg = geo[6 * mac + t];
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
          const double v = vol * (gr[a][0] * gr[b][0] + gr[a][1] * gr[b][1] + gr[a][2] * gr[b][2]);
          tg.Gp[4 * a + b] = T(v);
          if (a > 0) tg.Gs[4 * (a - 1) + b] = T(v / 210.0);
        }
      for (int a = 0; a < 4; ++a)
        for (int d = 0; d < 3; ++d) tg.grad[3 * a + d] = T(gr[a][d]);
      tg.vol = T(vol);
      for (int q = 0; q < 9; ++q) tg.JT[q] = T(J[q]);
      // 15-point stencils per boundary class z (zero pattern of the point):
      // micro-tet (t, slot a) exists unless the point lies on a macro face the
      // tet would have to cross
      for (int a = 0; a < 4; ++a) {
        const int ox = kOff[t][a][0], oy = kOff[t][a][1], oz = kOff[t][a][2];
        const int bad = (ox + oy + oz < kLim[t] ? 1 : 0) | (ox ? 2 : 0) | (oy ? 4 : 0) | (oz ? 8 : 0);
        for (int z = 0; z < 16; ++z) {
          if (z & bad) continue;
          for (int c = 0; c < 4; ++c)
            w[z][vslot(t, a, c)] += vol * (gr[a][0] * gr[c][0] + gr[a][1] * gr[c][1] + gr[a][2] * gr[c][2]);
        }
      }
    }
    for (int z = 0; z < 16; ++z)
      for (int q = 0; q < 15; ++q) w15[(16 * mac + z) * 15 + q] = T(w[z][q]);
  }
}

template <typename T>
void fill_qtab(const double *qb, const double *qw, int nq, std::vector<T> &out) {
  out.assign(static_cast<size_t>(nq) * kQStride, T(0));
  for (int q = 0; q < nq; ++q) {
    T *Q = out.data() + static_cast<size_t>(q) * kQStride;
    const double *l = qb + 4 * q;
    Q[0] = T(qw[q]);
    for (int a = 0; a < 4; ++a) Q[1 + a] = T(l[a]);
    for (int a = 0; a < 4; ++a) Q[5 + a] = T(l[a] * (2 * l[a] - 1));
    for (int e = 0; e < 6; ++e) Q[9 + e] = T(4 * l[kEdge[e][0]] * l[kEdge[e][1]]);
  }
}

template <typename T>
tmf_status upload_vec(DevBuf<uint8_t> &buf, const std::vector<T> &v) {
  return buf.upload(v.data(), v.size() * sizeof(T));
}

}  // namespace

namespace {
// XCD (0..7) that runs tile ti of an element launch over ntiles tiles:
// workgroups go round-robin over the 8 XCDs, and the element kernels give
// XCD x the contiguous run of tiles from x q + min(x, r) (q, r = ntiles / 8, ntiles % 8)
int tile_xcd(int ti, int ntiles) {
  const int q = ntiles / 8, rem = ntiles % 8;
  for (int x = 7; x > 0; --x)
    if (ti >= x * q + std::min(x, rem)) return x;
  return 0;
}
// seam work entries in launch order: entry i (counted from the first seam
// entry, which starts at a multiple of 8) runs on XCD i mod 8, so it is given
// an entry whose partial sums that XCD wrote where one is left (else one of
// the XCD with the most left); each XCD's entries keep their order
void seam_work_xcd(const std::vector<std::pair<int4, int>> &ent, std::vector<int4> &w) {
  std::vector<int4> q[8];
  for (const auto &e : ent) q[e.second].push_back(e.first);
  size_t pos[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (size_t i = 0; i < ent.size(); ++i) {
    int x = static_cast<int>(i % 8);
    if (pos[x] == q[x].size()) {
      size_t left = 0;
      for (int y = 0; y < 8; ++y)
        if (q[y].size() - pos[y] > left) {
          left = q[y].size() - pos[y];
          x = y;
        }
    }
    w.push_back(q[x][pos[x]++]);
  }
}
}  // namespace

extern "C" {

tmf_status tmf_op_create(const tmf_mesh *mesh, int kind, int prec, int bc, const double *qbary,
                         const double *qw, int nq, tmf_op **out) {
  if (!out) return fail(TMF_EINVAL, "out is NULL");
  *out = nullptr;
  if (!mesh) return fail(TMF_EINVAL, "mesh is NULL");
  if (kind < TMF_P1_LAPLACE || kind > TMF_N1_CURLCURL) return fail(TMF_EINVAL, "bad operator kind %d", kind);
  if (prec != TMF_F64 && prec != TMF_F32) return fail(TMF_EINVAL, "bad precision %d", prec);
  if (bc != TMF_BC_NONE && bc != TMF_BC_DIRICHLET_ZERO) return fail(TMF_EINVAL, "bad boundary condition %d", bc);
  const int space = kind <= TMF_P1_DIVKGRAD ? 1 : 2;
  if (space == 2 && mesh->level > TMF_MAX_LEVEL_P2)
    return fail(TMF_EINVAL, "P2 operators support level <= %d", TMF_MAX_LEVEL_P2);
  // a rule defines the blended epsilon operator, or the quadrature
  // (under-integration) variant of the affine P2 div(k grad) operator
  const bool quad_variant = mesh->map == TMF_MAP_AFFINE && kind == TMF_P2_DIVKGRAD && (qbary || qw || nq != 0);
  if (mesh->map == TMF_MAP_SHELL_RADIAL || quad_variant) {
    if (mesh->map == TMF_MAP_SHELL_RADIAL && kind != TMF_P2V_EPSILON)
      return fail(TMF_EUNSUPPORTED, "the blended shell map is supported for the epsilon operator only");
    if (!qbary || !qw || nq < 1 || nq > TMF_MAX_QUAD)
      return fail(TMF_EINVAL, "the quadrature rule needs 1..%d points", TMF_MAX_QUAD);
    double wsum = 0;
    for (int q = 0; q < nq; ++q) {
      double s = 0;
      for (int a = 0; a < 4; ++a) {
        if (!std::isfinite(qbary[4 * q + a])) return fail(TMF_EINVAL, "non-finite quadrature point");
        s += qbary[4 * q + a];
      }
      if (std::fabs(s - 1.0) > 1e-12) return fail(TMF_EINVAL, "quadrature point %d: barycentric sum != 1", q);
      if (!std::isfinite(qw[q])) return fail(TMF_EINVAL, "non-finite quadrature weight");
      wsum += qw[q];
    }
    if (std::fabs(wsum - 1.0 / 6.0) > 1e-12) return fail(TMF_EINVAL, "quadrature weights must sum to 1/6");
  } else if (qbary || qw || nq != 0) {
    return fail(TMF_EINVAL, "this affine operator is integrated exactly: pass no quadrature rule");
  }
  tmf_mesh *mm = const_cast<tmf_mesh *>(mesh);
  tmf_build_layout(mm, space);
  const SpaceLayout &S = mesh->sp[space];

  auto *op = new (std::nothrow) tmf_op;
  if (!op) return fail(TMF_ENOMEM, "host allocation failed");
  op->mesh = mesh;
  op->kind = kind;
  op->prec = prec;
  op->bc = bc;
  op->space = space;
  op->ncomp = kind == TMF_P2V_EPSILON ? 3 : 1;
  op->N = S.N;
  op->L = S.L;
  op->n_local = S.n_local;
  op->n_unique = S.n_unique;
  op->nq = (mesh->map == TMF_MAP_SHELL_RADIAL || quad_variant) ? nq : 0;
  tmf_status st = TMF_OK;
  if (prec == TMF_F64) {
    std::vector<TypeGeo<double>> g;
    std::vector<double> w;
    std::vector<MacroGeo<double>> mg;
    fill_geometry(mesh, g, w, mg);
    st = upload_vec(op->geo, g);
    if (st == TMF_OK) st = upload_vec(op->w15, w);
    if (st == TMF_OK) st = upload_vec(op->mgeo, mg);
    if (st == TMF_OK && op->nq) {
      std::vector<double> q;
      fill_qtab(qbary, qw, nq, q);
      st = upload_vec(op->qtab, q);
    }
  } else {
    std::vector<TypeGeo<float>> g;
    std::vector<float> w;
    std::vector<MacroGeo<float>> mg;
    fill_geometry(mesh, g, w, mg);
    st = upload_vec(op->geo, g);
    if (st == TMF_OK) st = upload_vec(op->w15, w);
    if (st == TMF_OK) st = upload_vec(op->mgeo, mg);
    if (st == TMF_OK && op->nq) {
      std::vector<float> q;
      fill_qtab(qbary, qw, nq, q);
      st = upload_vec(op->qtab, q);
    }
  }
  if (st == TMF_OK) st = op->bnd.upload(mesh->bnd.data(), mesh->bnd.size());
  if (st == TMF_OK && space == 1) {
    std::vector<int4> ch;
    const int N = S.N;
    if (kind == P1_LAPLACE) {
      // stencil tiles (2.5-D blocking): rows j0 .. j0+kStencilRows-1, points
      // i0 .. i0+61, planes k0 .. k0+3 (the planes where the tile has
      // points).  i0 varies fastest: concurrent wavefronts cover whole rows of
      // the same planes, so memory is read in long contiguous runs.
      for (int k0 = 0; k0 <= N; k0 += 4)
        for (int j0 = 0; j0 <= N - k0; j0 += kStencilRows)
          for (int i0 = 0; i0 <= N - j0 - k0; i0 += 62)
            ch.push_back(make_int4(j0, i0, k0, std::min(k0 + 4, N - i0 - j0 + 1)));
    } else {
      // row march: plane k, 62 points i0.., rows j0 .. j1-1 (8 rows; the rows
      // of the plane with points at i >= i0)
      for (int k = 0; k <= N; ++k)
        for (int i0 = 0; i0 <= N - k; i0 += 62) {
          const int jend = N - k - i0 + 1;
          for (int j0 = 0; j0 < jend; j0 += 8) ch.push_back(make_int4(k, i0, j0, std::min(j0 + 8, jend)));
        }
    }
    op->nchunks = static_cast<int>(ch.size());
    st = op->chunks.upload(ch.data(), ch.size());
  }
  if (st == TMF_OK && kind == TMF_N1_CURLCURL) {
    // orientation of each edge slot: the lattice direction D of a midpoint
    // m (the micro-edge direction whose odd coordinates are those of m, first
    // nonzero component positive) runs from (m - D) / 2 to (m + D) / 2; the
    // DoF's global orientation follows the canonical keys of the endpoints
    static const int kDir[8][3] = {{0, 0, 0},  {1, 0, 0},  {0, 1, 0},  {1, -1, 0},
                                   {0, 0, 1},  {1, 0, -1}, {0, 1, -1}, {1, -1, 1}};
    const int N = S.N;
    std::vector<int8_t> sg(static_cast<size_t>(S.n_local), 0);
    for (int64_t mac = 0; mac < mesh->nt; ++mac) {
      const int64_t *g = &mesh->T[4 * mac];
      for (int k = 0; k <= N; ++k)
        for (int j = 0; j <= N - k; ++j)
          for (int i = 0; i <= N - k - j; ++i) {
            const int odd = (i & 1) | ((j & 1) << 1) | ((k & 1) << 2);
            if (odd == 0) continue;
            const int *D = kDir[odd];
            const Key kp = point_key(g, i - D[0], j - D[1], k - D[2], N);
            const Key kq = point_key(g, i + D[0], j + D[1], k + D[2], N);
            sg[static_cast<size_t>(mac * S.L + row_base(j, k, N) + i)] = kp < kq ? 1 : -1;
          }
    }
    st = op->sign.upload(sg.data(), sg.size());
  }
  if (st == TMF_OK && space == 2) {
    const int n = mesh->n, N = S.N;
    size_t partial_bytes = 0;
    std::vector<std::pair<int4, int>> seam_entries[kNumTileCfg];
    for (int cfg = 0; cfg < kNumTileCfg && st == TMF_OK; ++cfg) {
      const int TX = kTileCfg[cfg][0], TY = kTileCfg[cfg][1], TZ = kTileCfg[cfg][2];
      // tiles, macro-major; .w = tile id within the operator
      std::vector<int4> tl;
      for (int64_t mac = 0; mac < mesh->nt; ++mac)
        for (int bz = 0; bz < n; bz += TZ)
          for (int by = 0; by < n - bz; by += TY)
            for (int bx = 0; bx < n - bz - by; bx += TX)
              tl.push_back(make_int4(0, int(mac), pack_base(bx, by, bz), static_cast<int>(tl.size())));
      op->ntiles[cfg] = static_cast<int>(tl.size());
      st = op->tiles[cfg].upload(tl.data(), tl.size());
      // first tile id of each box row (bz, by) within a macro
      const int nbz = (n + TZ - 1) / TZ, nby = (n + TY - 1) / TY;
      std::vector<int> rs(static_cast<size_t>(nbz) * nby, -1);
      int id = 0;
      for (int bz = 0; bz < n; bz += TZ)
        for (int by = 0; by < n - bz; by += TY) {
          rs[static_cast<size_t>(bz / TZ) * nby + by / TY] = id;
          for (int bx = 0; bx < n - bz - by; bx += TX) ++id;
        }
      op->tpm[cfg] = id;
      op->nby[cfg] = nby;
      op->seamrows[cfg] = nbz * nby;
      if (st == TMF_OK) st = op->rowstart[cfg].upload(rs.data(), rs.size());
      // seam points: a lattice coordinate that is a positive multiple of the
      // box extent (2 T points) lies on a face shared by two boxes
      std::vector<int> pts;
      for (int qz = 0; qz <= N; ++qz)
        for (int qy = 0; qy <= N - qz; ++qy)
          for (int qx = 0; qx <= N - qz - qy; ++qx)
            if ((qx > 0 && qx % (2 * TX) == 0) || (qy > 0 && qy % (2 * TY) == 0) || (qz > 0 && qz % (2 * TZ) == 0))
              pts.push_back(qx | (qy << 10) | (qz << 20));
      op->nseam[cfg] = static_cast<int>(pts.size());
      if (st == TMF_OK) st = op->seam[cfg].upload(pts.data(), pts.size());
      // seam work entries and the XCD that wrote (most of) their partial sums:
      // the one running the tile below the middle point of the entry's chunk
      {
        const int chunk = 256 * seam_ppt(op), ntl = static_cast<int>(tl.size());
        for (int64_t mac = 0; mac < mesh->nt; ++mac)
          for (int p0 = 0; p0 < static_cast<int>(pts.size()); p0 += chunk) {
            const int pk = pts[std::min<size_t>(p0 + chunk / 2, pts.size() - 1)];
            const int q[3] = {pk & 1023, (pk >> 10) & 1023, pk >> 20}, T3[3] = {TX, TY, TZ};
            int b[3];
            for (int d = 0; d < 3; ++d)
              b[d] = (q[d] > 0 && q[d] % (2 * T3[d]) == 0) ? q[d] / 2 - T3[d] : T3[d] * (q[d] / (2 * T3[d]));
            const int ti = static_cast<int>(mac) * id + rs[static_cast<size_t>(b[2] / TZ) * nby + b[1] / TY] + b[0] / TX;
            seam_entries[cfg].push_back({make_int4(0, static_cast<int>(mac), p0, 0), tile_xcd(ti, ntl)});
          }
      }
      const size_t R = static_cast<size_t>(2 * TX + 1) * (2 * TY + 1) * (2 * TZ + 1);
      const size_t per_tile = R * op->ncomp * (prec == TMF_F64 ? 8 : 4);
      op->partial_bytes[cfg] = tl.size() * per_tile;
      partial_bytes = std::max(partial_bytes, tl.size() * per_tile);
      // the gather addresses one macro's partial sums by 32-bit byte offsets
      if (st == TMF_OK && (tl.size() / static_cast<size_t>(mesh->nt)) * per_tile > 0xffffffffull)
        st = fail(TMF_EINVAL, "partial sums of one macro exceed 4 GiB at this level");
    }
    if (st == TMF_OK) st = op->partial.alloc(partial_bytes);
    // interface-group members as (macro, lattice point), and per macro the
    // zero patterns whose points have copies in other macros
    {
      std::vector<int> pk(static_cast<size_t>(S.L));
      size_t l = 0;
      for (int qz = 0; qz <= N; ++qz)
        for (int qy = 0; qy <= N - qz; ++qy)
          for (int qx = 0; qx <= N - qz - qy; ++qx) pk[l++] = qx | (qy << 10) | (qz << 20);
      std::vector<int64_t> gpos(S.gidx.size());
      std::vector<int> gpl(S.gidx.size());
      std::vector<uint32_t> shm(static_cast<size_t>(mesh->nt), 0u);
      if (S.gidx.size() > 0x7fffffff) st = fail(TMF_EINVAL, "too many interface copies for the seam reduction");
      for (size_t g = 0; g + 1 < S.gptr.size() && st == TMF_OK; ++g) {
        const int64_t len = S.gptr[g + 1] - S.gptr[g];
        if (len > 256) {
          st = fail(TMF_EINVAL, "an interface group has %lld copies (at most 256 supported)", (long long)len);
          break;
        }
        for (int64_t q = S.gptr[g]; q < S.gptr[g + 1]; ++q) {
          const int64_t slot = S.gidx[q], mac = slot / S.L;
          const int p = pk[static_cast<size_t>(slot - mac * S.L)];
          gpos[q] = (mac << 32) | static_cast<int64_t>(p);
          gpl[q] = static_cast<int>(((q - S.gptr[g]) << 16) | len);
          shm[mac] |= 1u << zero_pattern(p & 1023, (p >> 10) & 1023, p >> 20, N);
        }
      }
      if (st == TMF_OK) st = op->gpos.upload(gpos.data(), gpos.size());
      if (st == TMF_OK) st = op->gpl.upload(gpl.data(), gpl.size());
      if (st == TMF_OK) st = op->shared.upload(shm.data(), shm.size());
    }
    op->ngroups = static_cast<int64_t>(S.gptr.size()) - 1;
    if (st == TMF_OK) st = op->gptr.upload(S.gptr.data(), S.gptr.size());
    if (st == TMF_OK) st = op->gidx.upload(S.gidx.data(), S.gidx.size());
    for (int cfg = 0; cfg < kNumTileCfg && st == TMF_OK; ++cfg) {
      if (prec == TMF_F64) {
        SeamInst<double> si = seam_inst<double>(op, cfg, 0);
        st = op->seaminst[cfg].upload(reinterpret_cast<uint8_t *>(&si), sizeof(si));
      } else {
        SeamInst<float> si = seam_inst<float>(op, cfg, 0);
        st = op->seaminst[cfg].upload(reinterpret_cast<uint8_t *>(&si), sizeof(si));
      }
      // interface groups first: their chains of dependent loads then overlap
      // the bulk of the seam points instead of forming the launch's tail
      std::vector<int4> w;
      group_work(op, 0, w);
      // (padded with empty group entries to a multiple of 8, so that the
      // seam entries keep their XCD whether or not the groups are launched)
      while (w.size() % 8 != 0) w.push_back(make_int4(0, 0, 0, 1));
      op->ngroupwork[cfg] = static_cast<int>(w.size());
      seam_work_xcd(seam_entries[cfg], w);
      op->nseamwork[cfg] = static_cast<int>(w.size());
      op->nseamonly[cfg] = op->nseamwork[cfg] - op->ngroupwork[cfg];
      if (st == TMF_OK) st = op->seamwork[cfg].upload(w.data(), w.size());
    }
  }
  if (st == TMF_OK) {
    if (prec == TMF_F64) {
      InstDesc<double> d = make_desc<double>(op, 0);
      st = op->desc.upload(&d, sizeof(d));
    } else {
      InstDesc<float> d = make_desc<float>(op, 0);
      st = op->desc.upload(&d, sizeof(d));
    }
  }
  if (st == TMF_OK) {
    if (space == 1) {
      op->ngroups = static_cast<int64_t>(S.gptr.size()) - 1;
      st = op->gptr.upload(S.gptr.data(), S.gptr.size());
      if (st == TMF_OK) st = op->gidx.upload(S.gidx.data(), S.gidx.size());
    }
    if (st == TMF_OK) st = op->owner.upload(S.owner.data(), S.owner.size());
  }
  if (st != TMF_OK) {
    delete op;
    return st;
  }
  *out = op;
  return TMF_OK;
}

void tmf_op_destroy(tmf_op *op) { delete op; }

tmf_status tmf_op_info(const tmf_op *op, int64_t *n_local, int64_t *n_unique, int *ncomp, int *has_c) {
  if (!op) return fail(TMF_EINVAL, "op is NULL");
  if (n_local) *n_local = op->n_local;
  if (n_unique) *n_unique = op->n_unique;
  if (ncomp) *ncomp = op->ncomp;
  if (has_c) *has_c = has_coeff(op->kind) ? 1 : 0;
  return TMF_OK;
}

}  // extern "C"

namespace {

template <typename T>
LatticeArgs<T> lattice_args(const tmf_op *op) {
  LatticeArgs<T> L;
  L.n = op->mesh->n;
  L.N = op->N;
  L.nt = static_cast<int>(op->mesh->nt);
  L.L = static_cast<int>(op->L);
  L.dirichlet = op->bc == TMF_BC_DIRICHLET_ZERO;
  L.bnd = op->bnd.p;
  L.geo = reinterpret_cast<const TypeGeo<T> *>(op->geo.p);
  return L;
}

GroupArgs group_args(const tmf_op *op) {
  GroupArgs g;
  g.ptr = op->gptr.p;
  g.idx = op->gidx.p;
  g.ngroups = op->ngroups;
  g.n_local = op->n_local;
  g.ncomp = op->ncomp;
  return g;
}

// P2 and epsilon: element kernel (mode `kind`: an operator kind or a diagonal
// mode), then the seam reduction, with the interface sums unless a
// macro-local result is asked for
template <typename T>
hipError_t tile_path(tmf_op *op, int kind, const void *coeff, const void *x, T *yy, hipStream_t s, hipEvent_t ev0,
                     hipEvent_t ev1, bool interface, const void *x2 = nullptr, int seam_flags = 0,
                     int ncomp_out = 0, void *mat = nullptr, int cfg = -1, bool gather = true,
                     T *partial = nullptr) {
  hipError_t e;
  const int c = cfg >= 0 ? cfg : mode_cfg(op->tile_cfg, op->classic_cfg, kind);
  TileArgs<T> a;
  a.inst = reinterpret_cast<const InstDesc<T> *>(op->desc.p);
  a.tiles = op->tiles[c].p;
  a.ntiles = op->ntiles[c];
  a.mat = static_cast<T *>(mat);
  a.active = nullptr;
  a.qtab = reinterpret_cast<const T *>(op->qtab.p);
  a.nq = op->nq;
  a.k = static_cast<const T *>(coeff);
  a.x = static_cast<const T *>(x);
  a.x2 = static_cast<const T *>(x2);
  a.y = yy;
  a.partial = partial;
  if (ev0 && (e = hipEventRecord(ev0, s)) != hipSuccess) return e;
  e = launch_tile_apply<T>(a, kind, op->mesh->map, c, s);
  if (e == hipSuccess && ev1) e = hipEventRecord(ev1, s);
  if (e == hipSuccess && gather)
    e = launch_seam_gather<T>(reinterpret_cast<const SeamInst<T> *>(op->seaminst[c].p),
                              op->seamwork[c].p + (interface ? 0 : op->ngroupwork[c]),
                              interface ? op->nseamwork[c] : op->nseamonly[c], yy, nullptr,
                              (interface ? 0 : kSeamLocal) | seam_flags,
                              ncomp_out ? ncomp_out : op->ncomp, seam_ppt(op), c, seam_rows_lds(op->seamrows[c]), s,
                              partial);
  return e;
}

template <typename T>
hipError_t apply_t(tmf_op *op, const void *coeff, const void *x, void *y, hipStream_t s,
                   hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr, bool interface = true,
                   T *partial = nullptr) {
  hipError_t e;
  T *yy = static_cast<T *>(y);
  if (op->space == 1) {
    P1Args<T> a;
    a.lat = lattice_args<T>(op);
    a.w15 = reinterpret_cast<const T *>(op->w15.p);
    a.k = static_cast<const T *>(coeff);
    a.x = static_cast<const T *>(x);
    a.y = yy;
    if (ev0 && (e = hipEventRecord(ev0, s)) != hipSuccess) return e;
    e = launch_p1_apply<T>(a, op->kind, op->chunks.p, op->nchunks, s);
    if (e == hipSuccess && ev1) e = hipEventRecord(ev1, s);
  } else {
    const int mode = op->kind == TMF_P2_DIVKGRAD && op->nq > 0 ? P2_DIVKGRAD_Q : op->kind;
    return tile_path<T>(op, mode, coeff, x, yy, s, ev0, ev1, interface, nullptr, 0, 0, nullptr, -1, true, partial);
  }
  if (e != hipSuccess || !interface) return e;
  return launch_interface_sum<T>(group_args(op), yy, s);
}

template <typename T>
hipError_t adjoint_t(tmf_op *op, const void *coeff, const void *x, const void *gy, void *gx, void *gk,
                     hipStream_t s) {
  if (op->kind == TMF_P2_DIVKGRAD || op->kind == TMF_P2V_EPSILON) {
    // gx = L(k) gy: the macro-local apply; gk: the coefficient-gradient mode
    // of the element kernel (a scalar field), reduced per copy, Dirichlet
    // coefficient nodes kept
    hipError_t e = tile_path<T>(op, op->kind, coeff, gy, static_cast<T *>(gx), s, nullptr, nullptr, false);
    const int mode = op->kind == TMF_P2_DIVKGRAD ? P2_DIVKGRAD_GRADK : P2V_EPSILON_GRADMU;
    if (e == hipSuccess && gk)
      e = tile_path<T>(op, mode, nullptr, x, static_cast<T *>(gk), s, nullptr, nullptr, false, gy, kSeamKeepBoundary,
                       1);
    return e;
  }
  P1AdjArgs<T> a;
  a.lat = lattice_args<T>(op);
  a.k = static_cast<const T *>(coeff);
  a.x = static_cast<const T *>(x);
  a.gy = static_cast<const T *>(gy);
  a.gx = static_cast<T *>(gx);
  a.gk = static_cast<T *>(gk);
  return launch_p1_adjoint<T>(a, op->chunks.p, op->nchunks, s);
}

}  // namespace

extern "C" {

static tmf_status check_apply(tmf_op *op, const void *coeff, const void *x, void *y) {
  if (!op) return fail(TMF_EINVAL, "op is NULL");
  if (!x || !y) return fail(TMF_EINVAL, "x or y is NULL");
  if (has_coeff(op->kind) != (coeff != nullptr))
    return fail(TMF_EINVAL, has_coeff(op->kind) ? "this operator needs a coefficient field"
                                                : "this operator takes no coefficient field");
  if (y == x || (coeff && y == coeff)) return fail(TMF_EINVAL, "y must not alias x or the coefficient");
  return TMF_OK;
}

tmf_status tmf_apply_timed(tmf_op *op, const void *coeff, const void *x, void *y, tmf_stream stream,
                           void *ev_before, void *ev_after) {
  tmf_status st = check_apply(op, coeff, x, y);
  if (st != TMF_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0 = static_cast<hipEvent_t>(ev_before), e1 = static_cast<hipEvent_t>(ev_after);
  hipError_t e = op->prec == TMF_F64 ? apply_t<double>(op, coeff, x, y, s, e0, e1)
                                     : apply_t<float>(op, coeff, x, y, s, e0, e1);
  if (e != hipSuccess) return hip_fail(e, "apply launch");
  return TMF_OK;
}

tmf_status tmf_apply(tmf_op *op, const void *coeff, const void *x, void *y, tmf_stream stream) {
  return tmf_apply_timed(op, coeff, x, y, stream, nullptr, nullptr);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free apply.  The seam partial sums of one apply (the only device
// memory an apply uses beyond its inputs and outputs) go to a static device
// array of kScratchBytes, which the runtime places on every GPU the library
// is loaded on, instead of to the operator's own buffer.  Its device address
// is looked up once per device, on the first call with that device current.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {nullptr};

tmf_status scratch_address(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(TMF_EUNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[dev] == nullptr) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress of the static scratch");
    if (p == nullptr) return fail(TMF_EDEVICE, "the static scratch has no device address");
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return TMF_OK;
}
}  // namespace

extern "C" {

tmf_status tmf_apply_noalloc(tmf_op *op, const void *coeff, const void *x, void *y, tmf_stream stream) {
  tmf_status st = check_apply(op, coeff, x, y);
  if (st != TMF_OK) return st;
  void *ptr = nullptr;
  if (op->space == 2) {
    // the tile shape the apply runs with, and the partial sums it writes
    const int mode = op->kind == TMF_P2_DIVKGRAD && op->nq > 0 ? P2_DIVKGRAD_Q : op->kind;
    const int c = mode_cfg(op->tile_cfg, op->classic_cfg, mode);
    if (op->partial_bytes[c] > kScratchBytes)
      return fail(TMF_EINVAL, "this apply needs %zu bytes of partial sums; the static scratch holds %zu",
                  op->partial_bytes[c], kScratchBytes);
    st = scratch_address(&ptr);
    if (st != TMF_OK) return st;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = op->prec == TMF_F64
                     ? apply_t<double>(op, coeff, x, y, s, nullptr, nullptr, true, static_cast<double *>(ptr))
                     : apply_t<float>(op, coeff, x, y, s, nullptr, nullptr, true, static_cast<float *>(ptr));
  if (e != hipSuccess) return hip_fail(e, "apply launch");
  return TMF_OK;
}

tmf_status tmf_apply_local(tmf_op *op, const void *coeff, const void *x, void *y, tmf_stream stream) {
  tmf_status st = check_apply(op, coeff, x, y);
  if (st != TMF_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = op->prec == TMF_F64 ? apply_t<double>(op, coeff, x, y, s, nullptr, nullptr, false)
                                     : apply_t<float>(op, coeff, x, y, s, nullptr, nullptr, false);
  if (e != hipSuccess) return hip_fail(e, "apply launch");
  return TMF_OK;
}

}  // extern "C"

namespace {
// diag(A) of a P1 kind: one vertex-centric launch, then the interface sum
template <typename T>
hipError_t p1_diagonal(tmf_op *op, const void *coeff, void *d, hipStream_t s) {
  P1Args<T> a;
  a.lat = lattice_args<T>(op);
  a.w15 = reinterpret_cast<const T *>(op->w15.p);
  a.k = static_cast<const T *>(coeff);
  a.x = nullptr;
  a.y = static_cast<T *>(d);
  hipError_t e = launch_p1_apply<T>(a, op->kind == TMF_P1_LAPLACE ? P1_LAPLACE_DIAG : P1_DIVKGRAD_DIAG,
                                    op->chunks.p, op->nchunks, s);
  if (e != hipSuccess) return e;
  return launch_interface_sum<T>(group_args(op), static_cast<T *>(d), s);
}
}  // namespace

extern "C" {

tmf_status tmf_diagonal(tmf_op *op, const void *coeff, void *d, tmf_stream stream) {
  if (!op || !d) return fail(TMF_EINVAL, "op or d is NULL");
  if (op->kind == TMF_N1_CURLCURL || (op->nq > 0 && op->kind != TMF_P2V_EPSILON))
    return fail(TMF_EUNSUPPORTED, "the diagonal is provided for the P1, exact scalar P2 and epsilon kinds");
  if (has_coeff(op->kind) != (coeff != nullptr))
    return fail(TMF_EINVAL, has_coeff(op->kind) ? "this operator needs a coefficient field"
                                                : "this operator takes no coefficient field");
  if (coeff && d == coeff) return fail(TMF_EINVAL, "d must not alias the coefficient");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (op->space == 1) {
    e = op->prec == TMF_F64 ? p1_diagonal<double>(op, coeff, d, s) : p1_diagonal<float>(op, coeff, d, s);
  } else {
    const int dk = op->kind == TMF_P2_LAPLACE   ? P2_LAPLACE_DIAG
                   : op->kind == TMF_P2_DIVKGRAD ? P2_DIVKGRAD_DIAG
                                                 : P2V_EPSILON_DIAG;
    // the diagonal modes read no x; the output pointer stands in for it
    e = op->prec == TMF_F64 ? tile_path<double>(op, dk, coeff, d, static_cast<double *>(d), s, nullptr, nullptr, true)
                            : tile_path<float>(op, dk, coeff, d, static_cast<float *>(d), s, nullptr, nullptr, true);
  }
  if (e != hipSuccess) return hip_fail(e, "diagonal launch");
  return TMF_OK;
}

tmf_status tmf_op_store_matrices(tmf_op *op, const void *coeff, tmf_stream stream) {
  if (!op || !coeff) return fail(TMF_EINVAL, "op or coeff is NULL");
  if (op->kind != TMF_P2_DIVKGRAD || op->nq > 0)
    return fail(TMF_EUNSUPPORTED, "stored local matrices are provided for the exact TMF_P2_DIVKGRAD");
  const int cfg = mode_cfg(op->tile_cfg, op->classic_cfg, P2_DIVKGRAD_STORE);
  const size_t esz = op->prec == TMF_F64 ? 8 : 4;
  const size_t cubes = static_cast<size_t>(kTileCfg[cfg][0]) * kTileCfg[cfg][1] * kTileCfg[cfg][2];
  const size_t bytes = static_cast<size_t>(op->ntiles[cfg]) * 6 * kStoredEntries * cubes * esz;
  if (op->mat.n != bytes) {
    op->mat_cfg = -1;
    tmf_status st = op->mat.alloc(bytes);
    if (st != TMF_OK) return st;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the store mode reads only k and writes only the matrices (no x, no y,
  // no gather); coeff stands in for the unused vector pointers
  hipError_t e =
      op->prec == TMF_F64
          ? tile_path<double>(op, P2_DIVKGRAD_STORE, coeff, coeff, const_cast<double *>(static_cast<const double *>(coeff)),
                              s, nullptr, nullptr, true, nullptr, 0, 0, op->mat.p, cfg, false)
          : tile_path<float>(op, P2_DIVKGRAD_STORE, coeff, coeff, const_cast<float *>(static_cast<const float *>(coeff)),
                             s, nullptr, nullptr, true, nullptr, 0, 0, op->mat.p, cfg, false);
  if (e != hipSuccess) return hip_fail(e, "matrix store launch");
  op->mat_cfg = cfg;
  return TMF_OK;
}

tmf_status tmf_apply_stored(tmf_op *op, const void *x, void *y, tmf_stream stream) {
  if (!op || !x || !y) return fail(TMF_EINVAL, "op, x or y is NULL");
  if (op->mat_cfg < 0) return fail(TMF_EINVAL, "no stored matrices: call tmf_op_store_matrices first");
  if (x == y) return fail(TMF_EINVAL, "y must not alias x");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = op->prec == TMF_F64
                     ? tile_path<double>(op, P2_STORED_APPLY, nullptr, x, static_cast<double *>(y), s, nullptr, nullptr,
                                         true, nullptr, 0, 0, op->mat.p, op->mat_cfg, true)
                     : tile_path<float>(op, P2_STORED_APPLY, nullptr, x, static_cast<float *>(y), s, nullptr, nullptr,
                                        true, nullptr, 0, 0, op->mat.p, op->mat_cfg, true);
  if (e != hipSuccess) return hip_fail(e, "stored apply launch");
  return TMF_OK;
}

tmf_status tmf_interface_sum(tmf_op *op, void *v, tmf_stream stream) {
  if (!op || !v) return fail(TMF_EINVAL, "op or v is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = op->prec == TMF_F64 ? launch_interface_sum<double>(group_args(op), static_cast<double *>(v), s)
                                     : launch_interface_sum<float>(group_args(op), static_cast<float *>(v), s);
  if (e != hipSuccess) return hip_fail(e, "interface sum launch");
  return TMF_OK;
}

static int num_tiles(const tmf_op *op) {
  if (op->space == 1) return 1;
  if (op->kind == TMF_P2V_EPSILON) return 2;
  // the marching shapes serve the exactly integrated scalar P2 applies
  const bool march = (op->kind == TMF_P2_LAPLACE || op->kind == TMF_P2_DIVKGRAD) && op->nq == 0;
  return march ? kNumTileCfg : kNumClassicTileCfg;
}

tmf_status tmf_op_num_tiles(const tmf_op *op, int *count) {
  if (!op || !count) return fail(TMF_EINVAL, "NULL argument");
  *count = num_tiles(op);
  return TMF_OK;
}

tmf_status tmf_op_tile_shape(const tmf_op *op, int cfg, int *tx, int *ty, int *tz) {
  if (!op) return fail(TMF_EINVAL, "op is NULL");
  if (cfg < 0 || cfg >= num_tiles(op)) return fail(TMF_EINVAL, "tile shape %d out of range", cfg);
  if (tx) *tx = op->space == 1 ? 1 : kTileCfg[cfg][0];
  if (ty) *ty = op->space == 1 ? 1 : kTileCfg[cfg][1];
  if (tz) *tz = op->space == 1 ? 1 : kTileCfg[cfg][2];
  return TMF_OK;
}

tmf_status tmf_op_set_tile(tmf_op *op, int cfg) {
  if (!op) return fail(TMF_EINVAL, "op is NULL");
  if (cfg < 0 || cfg >= num_tiles(op)) return fail(TMF_EINVAL, "tile shape %d out of range", cfg);
  op->tile_cfg = cfg;
  if (kTileMarch[cfg] == 0) op->classic_cfg = cfg;
  return TMF_OK;
}

tmf_status tmf_op_get_tile(const tmf_op *op, int *cfg) {
  if (!op || !cfg) return fail(TMF_EINVAL, "NULL argument");
  *cfg = op->tile_cfg;
  return TMF_OK;
}

tmf_status tmf_op_autotune(tmf_op *op, const void *coeff, const void *x, void *y, tmf_stream stream, int reps,
                           int *best_cfg, float *best_ms) {
  tmf_status st = check_apply(op, coeff, x, y);
  if (st != TMF_OK) return st;
  if (reps < 1) return fail(TMF_EINVAL, "reps must be >= 1");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(TMF_EDEVICE, "hipEventCreate failed");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(TMF_EDEVICE, "hipEventCreate failed");
  }
  int best = op->tile_cfg, best_box = op->classic_cfg;
  float best_t = 0, best_box_t = 0;
  const int keep = op->tile_cfg;
  for (int cfg = 0; cfg < num_tiles(op) && st == TMF_OK; ++cfg) {
    op->tile_cfg = cfg;
    for (int w = 0; w < 2 && st == TMF_OK; ++w) st = tmf_apply(op, coeff, x, y, stream);
    if (st != TMF_OK) break;
    hipError_t e = hipEventRecord(e0, s);
    for (int r = 0; r < reps && st == TMF_OK && e == hipSuccess; ++r) st = tmf_apply(op, coeff, x, y, stream);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) st = hip_fail(e, "autotune timing");
    ms /= reps;
    if (st == TMF_OK && (cfg == 0 || ms < best_t)) {
      best_t = ms;
      best = cfg;
    }
    if (st == TMF_OK && kTileMarch[cfg] == 0 && (cfg == 0 || ms < best_box_t)) {
      best_box_t = ms;
      best_box = cfg;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != TMF_OK) {
    op->tile_cfg = keep;
    return st;
  }
  op->tile_cfg = best;
  op->classic_cfg = best_box;
  if (best_cfg) *best_cfg = best;
  if (best_ms) *best_ms = best_t;
  return TMF_OK;
}

tmf_status tmf_op_tune(tmf_op *op, const void *coeff, const void *x, void *y, tmf_stream stream, int reps,
                       const char *cache_json_path, int *best_cfg, float *best_ms) {
  if (!op) return fail(TMF_EINVAL, "op is NULL");
  char key[256];
  std::snprintf(key, sizeof(key), "op kind=%d prec=%d bc=%d nq=%d map=%d level=%d macros=%lld dev=%s", op->kind,
                op->prec, op->bc, op->nq, op->mesh->map, op->mesh->level, static_cast<long long>(op->mesh->nt),
                device_tag().c_str());
  int cfg = 0, box = 0;
  float ms = 0;
  if (cache_json_path) {
    const int r = tune_cache_lookup(cache_json_path, key, &cfg, &box, &ms);
    if (r < 0) return fail(TMF_EINVAL, "tile cache %s is not a cache file this library wrote", cache_json_path);
    if (r == 1 && cfg >= 0 && cfg < num_tiles(op) && box >= 0 && box < num_tiles(op) && kTileMarch[box] == 0) {
      op->tile_cfg = cfg;
      op->classic_cfg = box;
      if (best_cfg) *best_cfg = cfg;
      if (best_ms) *best_ms = ms;
      return TMF_OK;
    }
  }
  tmf_status st = tmf_op_autotune(op, coeff, x, y, stream, reps, &cfg, &ms);
  if (st == TMF_OK && cache_json_path) st = tune_cache_store(cache_json_path, key, cfg, op->classic_cfg, ms);
  if (st != TMF_OK) return st;
  if (best_cfg) *best_cfg = cfg;
  if (best_ms) *best_ms = ms;
  return TMF_OK;
}

tmf_status tmf_apply_adjoint(tmf_op *op, const void *coeff, const void *x, const void *gy, void *gx, void *gk,
                             tmf_stream stream) {
  if (!op) return fail(TMF_EINVAL, "op is NULL");
  if (op->kind != TMF_P1_DIVKGRAD && op->kind != TMF_P2_DIVKGRAD && op->kind != TMF_P2V_EPSILON)
    return fail(TMF_EUNSUPPORTED, "the adjoint is implemented for the div(k grad) and epsilon kinds");
  if (op->kind == TMF_P2_DIVKGRAD && op->nq > 0)
    return fail(TMF_EUNSUPPORTED, "the adjoint of the quadrature variant is not provided");
  if (!coeff || !x || !gy || !gx) return fail(TMF_EINVAL, "coeff, x, gy and gx are required");
  const void *ins[3] = {coeff, x, gy};
  for (const void *p : ins)
    if (p == gx || (gk && p == gk)) return fail(TMF_EINVAL, "outputs must not alias inputs");
  if (gk && gk == gx) return fail(TMF_EINVAL, "gx and gk must differ");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = op->prec == TMF_F64 ? adjoint_t<double>(op, coeff, x, gy, gx, gk, s)
                                     : adjoint_t<float>(op, coeff, x, gy, gx, gk, s);
  if (e != hipSuccess) return hip_fail(e, "adjoint launch");
  return TMF_OK;
}

}  // extern "C"
