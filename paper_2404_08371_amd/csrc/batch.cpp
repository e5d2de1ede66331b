// Batched operators and the mixed-precision iterative-refinement CG solver.
//
// A batch applies many operator instances -- uneven refinement levels and
// coefficients, vectors concatenated -- in one launch of the element kernel:
// the tile lists of all instances form one work list (largest instances
// first), so small instances do not each pay a launch and large ones do not
// serialise.  The solver refines an FP64 solution with conjugate-gradient
// corrections in the inner batch's precision (FP32, or FP64 for plain FP64
// CG): the outer residual b - A x, the norms and the solution update are
// FP64, the inner CG runs the inner operator with FP64-accumulated dot
// products, and a block of inner iterations is captured once into a HIP graph
// and replayed.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "host_internal.h"
#include "solver_internal.h"

struct tmf_batch {
  int count = 0, prec = 0, kind = 0, ncomp = 1;
  std::vector<tmf_op *> ops;
  std::vector<int64_t> off;  // count + 1 offsets into the concatenated vectors
  DevBuf<uint8_t> desc;
  DevBuf<int4> tiles[kNumTileCfg];
  int ntiles[kNumTileCfg] = {0};
  int tile_cfg = 0;
  int classic_cfg = 0;  // box shape for the diagonal mode when tile_cfg is a marching shape
  // reduction chunks over the concatenated vectors
  DevBuf<ChunkDesc> chunks;
  int nchunks = 0;
  DevBuf<int> first;
  DevBuf<uint8_t> owner;  // only when some instance has several macros
  // seam reduction of all instances in one launch, per tile shape
  DevBuf<uint8_t> seaminst[kNumTileCfg];
  DevBuf<int4> seamwork[kNumTileCfg];
  int nseamwork[kNumTileCfg] = {0};
  int seamrows[kNumTileCfg] = {0};  // tile-row table entries staged in LDS by the seam reduction
};

struct tmf_ir {
  tmf_batch *b64 = nullptr, *b32 = nullptr;  // outer (FP64) and inner (FP32 or FP64) batches
  bool inner64 = false;                      // inner iteration in FP64 (plain FP64 CG)
  tmf_ir_options opt{};
  hipStream_t stream = nullptr;
  DevBuf<double> Ax, r64, part1, part2, scal;
  DevBuf<uint8_t> r32, p, q, d, dinv;  // inner vectors, element type of the inner batch
  DevBuf<int> it;
  DevBuf<uint8_t> flags;
  BlasCtx ctx{};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void *graph_k32 = nullptr;
  ~tmf_ir() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (stream) (void)hipStreamDestroy(stream);
  }
};

namespace {

// mode: the batch's kind, or a diagonal mode of the element kernel.  Every
// entry of an active instance is written by the element kernel or the seam
// reduction; inactive instances are set to zero if zero_inactive (the
// solver's own applies skip that: its vector kernels never read them).
template <typename T>
hipError_t batch_apply_t(tmf_batch *b, int mode, const void *coeff, const void *x, void *y, const uint8_t *active,
                         hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, bool zero_inactive) {
  T *yy = static_cast<T *>(y);
  hipError_t e = hipSuccess;
  if (active && zero_inactive) e = launch_fill<T>(yy, b->off[b->count], T(0), s);
  if (e != hipSuccess) return e;
  const int c = mode_cfg(b->tile_cfg, b->classic_cfg, mode);
  TileArgs<T> a;
  a.inst = reinterpret_cast<const InstDesc<T> *>(b->desc.p);
  a.tiles = b->tiles[c].p;
  a.ntiles = b->ntiles[c];
  a.active = active;
  a.qtab = nullptr;
  a.nq = 0;
  a.k = static_cast<const T *>(coeff);
  a.x = static_cast<const T *>(x);
  a.y = yy;
  if (ev0 && (e = hipEventRecord(ev0, s)) != hipSuccess) return e;
  e = launch_tile_apply<T>(a, mode, TMF_MAP_AFFINE, c, s);
  if (e == hipSuccess && ev1) e = hipEventRecord(ev1, s);
  if (e != hipSuccess) return e;
  // seam and interface reduction of every instance, one launch
  return launch_seam_gather<T>(reinterpret_cast<const SeamInst<T> *>(b->seaminst[c].p), b->seamwork[c].p,
                               b->nseamwork[c], yy, active, 0, b->ncomp, seam_ppt(b->ops[0]), c, b->seamrows[c], s);
}

// tile shapes of a batch: epsilon has two; the scalar P2 kinds also take the marching shapes
int batch_num_tiles(const tmf_batch *b) { return b->kind == TMF_P2V_EPSILON ? 2 : kNumTileCfg; }

tmf_status batch_apply(tmf_batch *b, const void *coeff, const void *x, void *y, const uint8_t *active,
                       hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr, bool zero_inactive = true) {
  hipError_t e = b->prec == TMF_F64
                     ? batch_apply_t<double>(b, b->kind, coeff, x, y, active, s, ev0, ev1, zero_inactive)
                     : batch_apply_t<float>(b, b->kind, coeff, x, y, active, s, ev0, ev1, zero_inactive);
  if (e != hipSuccess) return hip_fail(e, "batch apply launch");
  return TMF_OK;
}

tmf_status batch_diagonal(tmf_batch *b, const void *coeff, void *d, hipStream_t s) {
  if (b->kind != TMF_P2_LAPLACE && b->kind != TMF_P2_DIVKGRAD)
    return fail(TMF_EUNSUPPORTED, "the diagonal is provided for the scalar P2 kinds");
  const int mode = b->kind == TMF_P2_LAPLACE ? P2_LAPLACE_DIAG : P2_DIVKGRAD_DIAG;
  // the diagonal modes read no x; the output pointer stands in for it
  hipError_t e = b->prec == TMF_F64
                     ? batch_apply_t<double>(b, mode, coeff, d, d, nullptr, s, nullptr, nullptr, true)
                     : batch_apply_t<float>(b, mode, coeff, d, d, nullptr, s, nullptr, nullptr, true);
  if (e != hipSuccess) return hip_fail(e, "batch diagonal launch");
  return TMF_OK;
}

tmf_status check_batch_apply(tmf_batch *b, const void *coeff, const void *x, void *y) {
  if (!b) return fail(TMF_EINVAL, "batch is NULL");
  if (!x || !y) return fail(TMF_EINVAL, "x or y is NULL");
  if (has_coeff(b->kind) != (coeff != nullptr))
    return fail(TMF_EINVAL, has_coeff(b->kind) ? "this operator needs a coefficient field"
                                               : "this operator takes no coefficient field");
  if (y == x || (coeff && y == coeff)) return fail(TMF_EINVAL, "y must not alias x or the coefficient");
  return TMF_OK;
}

}  // namespace

extern "C" {

tmf_status tmf_batch_create(tmf_op *const *ops, int count, tmf_batch **out) {
  if (!out) return fail(TMF_EINVAL, "out is NULL");
  *out = nullptr;
  if (!ops || count < 1) return fail(TMF_EINVAL, "need at least one operator");
  const tmf_op *o0 = ops[0];
  if (!o0) return fail(TMF_EINVAL, "operator 0 is NULL");
  for (int i = 0; i < count; ++i) {
    const tmf_op *o = ops[i];
    if (!o) return fail(TMF_EINVAL, "operator %d is NULL", i);
    if (o->space != 2 || o->kind == TMF_N1_CURLCURL)
      return fail(TMF_EUNSUPPORTED, "batches hold P2 / epsilon operators (element kernels)");
    if (o->kind != o0->kind || o->prec != o0->prec)
      return fail(TMF_EINVAL, "operator %d differs in kind or precision from operator 0", i);
    if (o->mesh->map != TMF_MAP_AFFINE || o->nq > 0)
      return fail(TMF_EUNSUPPORTED, "batches hold exactly integrated operators on affine meshes");
    for (int j = 0; j < i; ++j)
      if (ops[j] == o) return fail(TMF_EINVAL, "operator %d appears twice", i);
  }
  auto *b = new (std::nothrow) tmf_batch;
  if (!b) return fail(TMF_ENOMEM, "host allocation failed");
  b->count = count;
  b->prec = o0->prec;
  b->kind = o0->kind;
  b->ncomp = o0->ncomp;
  b->ops.assign(ops, ops + count);
  b->off.assign(count + 1, 0);
  for (int i = 0; i < count; ++i) b->off[i + 1] = b->off[i] + ops[i]->ncomp * ops[i]->n_local;
  tmf_status st = TMF_OK;
  if (b->prec == TMF_F64) {
    std::vector<InstDesc<double>> d;
    for (int i = 0; i < count; ++i) d.push_back(make_desc<double>(ops[i], b->off[i]));
    st = b->desc.upload(d.data(), d.size() * sizeof(d[0]));
  } else {
    std::vector<InstDesc<float>> d;
    for (int i = 0; i < count; ++i) d.push_back(make_desc<float>(ops[i], b->off[i]));
    st = b->desc.upload(d.data(), d.size() * sizeof(d[0]));
  }
  // tile lists: all instances, largest first (their long tails start early)
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int c) { return ops[a]->n_local > ops[c]->n_local; });
  for (int cfg = 0; cfg < kNumTileCfg && st == TMF_OK; ++cfg) {
    const int TX = kTileCfg[cfg][0], TY = kTileCfg[cfg][1], TZ = kTileCfg[cfg][2];
    std::vector<int4> tl;
    for (int i : order) {
      const int n = ops[i]->mesh->n;
      for (int64_t mac = 0; mac < ops[i]->mesh->nt; ++mac)
        for (int bz = 0; bz < n; bz += TZ)
          for (int by = 0; by < n - bz; by += TY)
            for (int bx = 0; bx < n - bz - by; bx += TX) tl.push_back(make_int4(i, int(mac), pack_base(bx, by, bz), 0));
    }
    // .w = tile id within the instance (the operator's own enumeration order)
    {
      std::vector<int> next(count, 0);
      for (int4 &t4 : tl) t4.w = next[t4.x]++;
    }
    b->ntiles[cfg] = static_cast<int>(tl.size());
    st = b->tiles[cfg].upload(tl.data(), tl.size());
  }
  for (int cfg = 0; cfg < kNumTileCfg && st == TMF_OK; ++cfg) {
    std::vector<int4> w;
    for (int i = 0; i < count; ++i) group_work(ops[i], i, w);
    for (int i = 0; i < count; ++i) seam_work(ops[i], cfg, i, w);
    b->nseamwork[cfg] = static_cast<int>(w.size());
    for (int i = 0; i < count; ++i) b->seamrows[cfg] = std::max(b->seamrows[cfg], seam_rows_lds(ops[i]->seamrows[cfg]));
    st = b->seamwork[cfg].upload(w.data(), w.size());
    if (st != TMF_OK) break;
    if (b->prec == TMF_F64) {
      std::vector<SeamInst<double>> si;
      for (int i = 0; i < count; ++i) si.push_back(seam_inst<double>(ops[i], cfg, b->off[i]));
      st = b->seaminst[cfg].upload(reinterpret_cast<uint8_t *>(si.data()), si.size() * sizeof(si[0]));
    } else {
      std::vector<SeamInst<float>> si;
      for (int i = 0; i < count; ++i) si.push_back(seam_inst<float>(ops[i], cfg, b->off[i]));
      st = b->seaminst[cfg].upload(reinterpret_cast<uint8_t *>(si.data()), si.size() * sizeof(si[0]));
    }
  }
  // reduction chunks
  std::vector<ChunkDesc> ch;
  std::vector<int> first(count + 1, 0);
  bool need_owner = false;
  for (int i = 0; i < count; ++i) {
    first[i] = static_cast<int>(ch.size());
    for (int64_t s = b->off[i]; s < b->off[i + 1]; s += kChunkLen)
      ch.push_back(ChunkDesc{s, static_cast<int>(std::min<int64_t>(kChunkLen, b->off[i + 1] - s)), i});
    if (ops[i]->mesh->nt > 1) need_owner = true;
  }
  first[count] = static_cast<int>(ch.size());
  b->nchunks = static_cast<int>(ch.size());
  if (st == TMF_OK) st = b->chunks.upload(ch.data(), ch.size());
  if (st == TMF_OK) st = b->first.upload(first.data(), first.size());
  if (st == TMF_OK && need_owner) {
    st = b->owner.alloc(b->off[count]);
    for (int i = 0; i < count && st == TMF_OK; ++i)
      for (int c = 0; c < ops[i]->ncomp && st == TMF_OK; ++c) {
        hipError_t e = hipMemcpy(b->owner.p + b->off[i] + c * ops[i]->n_local, ops[i]->owner.p, ops[i]->n_local,
                                 hipMemcpyDeviceToDevice);
        if (e != hipSuccess) st = hip_fail(e, "hipMemcpy");
      }
  }
  if (st != TMF_OK) {
    delete b;
    return st;
  }
  *out = b;
  return TMF_OK;
}

void tmf_batch_destroy(tmf_batch *b) { delete b; }

tmf_status tmf_batch_info(const tmf_batch *b, int *count, int64_t *offsets) {
  if (!b) return fail(TMF_EINVAL, "batch is NULL");
  if (count) *count = b->count;
  if (offsets)
    for (int i = 0; i <= b->count; ++i) offsets[i] = b->off[i];
  return TMF_OK;
}

tmf_status tmf_batch_apply(tmf_batch *b, const void *coeff, const void *x, void *y, const uint8_t *active,
                           tmf_stream stream) {
  tmf_status st = check_batch_apply(b, coeff, x, y);
  if (st != TMF_OK) return st;
  return batch_apply(b, coeff, x, y, active, static_cast<hipStream_t>(stream));
}

tmf_status tmf_batch_apply_timed(tmf_batch *b, const void *coeff, const void *x, void *y, const uint8_t *active,
                                 tmf_stream stream, void *ev_before, void *ev_after) {
  tmf_status st = check_batch_apply(b, coeff, x, y);
  if (st != TMF_OK) return st;
  return batch_apply(b, coeff, x, y, active, static_cast<hipStream_t>(stream), static_cast<hipEvent_t>(ev_before),
                     static_cast<hipEvent_t>(ev_after));
}

tmf_status tmf_batch_diagonal(tmf_batch *b, const void *coeff, void *d, tmf_stream stream) {
  if (!b || !d) return fail(TMF_EINVAL, "batch or d is NULL");
  if (has_coeff(b->kind) != (coeff != nullptr))
    return fail(TMF_EINVAL, has_coeff(b->kind) ? "this operator needs a coefficient field"
                                               : "this operator takes no coefficient field");
  if (coeff && d == coeff) return fail(TMF_EINVAL, "d must not alias the coefficient");
  return batch_diagonal(b, coeff, d, static_cast<hipStream_t>(stream));
}

tmf_status tmf_batch_set_tile(tmf_batch *b, int cfg) {
  if (!b) return fail(TMF_EINVAL, "batch is NULL");
  if (cfg < 0 || cfg >= batch_num_tiles(b)) return fail(TMF_EINVAL, "tile shape %d out of range", cfg);
  b->tile_cfg = cfg;
  if (kTileMarch[cfg] == 0) b->classic_cfg = cfg;
  return TMF_OK;
}

tmf_status tmf_batch_autotune(tmf_batch *b, const void *coeff, const void *x, void *y, tmf_stream stream, int reps,
                              int *best_cfg, float *best_ms) {
  tmf_status st = check_batch_apply(b, coeff, x, y);
  if (st != TMF_OK) return st;
  if (reps < 1) return fail(TMF_EINVAL, "reps must be >= 1");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(TMF_EDEVICE, "hipEventCreate failed");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(TMF_EDEVICE, "hipEventCreate failed");
  }
  const int keep = b->tile_cfg;
  int best = keep, best_box = b->classic_cfg;
  float best_t = 0, best_box_t = 0;
  const int nt = batch_num_tiles(b);
  for (int cfg = 0; cfg < nt && st == TMF_OK; ++cfg) {
    b->tile_cfg = cfg;
    for (int w = 0; w < 2 && st == TMF_OK; ++w) st = batch_apply(b, coeff, x, y, nullptr, s);
    if (st != TMF_OK) break;
    hipError_t e = hipEventRecord(e0, s);
    for (int r = 0; r < reps && st == TMF_OK && e == hipSuccess; ++r) st = batch_apply(b, coeff, x, y, nullptr, s);
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
  b->tile_cfg = st == TMF_OK ? best : keep;
  if (st == TMF_OK) b->classic_cfg = best_box;
  if (st != TMF_OK) return st;
  if (best_cfg) *best_cfg = best;
  if (best_ms) *best_ms = best_t;
  return TMF_OK;
}

tmf_status tmf_batch_tune(tmf_batch *b, const void *coeff, const void *x, void *y, tmf_stream stream, int reps,
                          const char *cache_json_path, int *best_cfg, float *best_ms) {
  if (!b) return fail(TMF_EINVAL, "batch is NULL");
  std::string key = "batch kind=" + std::to_string(b->kind) + " prec=" + std::to_string(b->prec) +
                    " count=" + std::to_string(b->count) + " levels=";
  for (int i = 0; i < b->count; ++i)
    key += (i ? "," : "") + std::to_string(b->ops[i]->mesh->level) + ":" + std::to_string(b->ops[i]->mesh->nt);
  key += " dev=" + device_tag();
  int cfg = 0, box = 0;
  float ms = 0;
  if (cache_json_path) {
    const int r = tune_cache_lookup(cache_json_path, key, &cfg, &box, &ms);
    if (r < 0) return fail(TMF_EINVAL, "tile cache %s is not a cache file this library wrote", cache_json_path);
    const int nt = batch_num_tiles(b);
    if (r == 1 && cfg >= 0 && cfg < nt && box >= 0 && box < nt && kTileMarch[box] == 0) {
      b->tile_cfg = cfg;
      b->classic_cfg = box;
      if (best_cfg) *best_cfg = cfg;
      if (best_ms) *best_ms = ms;
      return TMF_OK;
    }
  }
  tmf_status st = tmf_batch_autotune(b, coeff, x, y, stream, reps, &cfg, &ms);
  if (st == TMF_OK && cache_json_path) st = tune_cache_store(cache_json_path, key, cfg, b->classic_cfg, ms);
  if (st != TMF_OK) return st;
  if (best_cfg) *best_cfg = cfg;
  if (best_ms) *best_ms = ms;
  return TMF_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ solver
namespace {

template <typename V>
V *vec(DevBuf<uint8_t> &b) {
  return reinterpret_cast<V *>(b.p);
}

// one inner iteration; par = parity of the iteration within its block (the
// slot of r.z it reads)
template <typename V>
tmf_status inner_step_t(tmf_ir *S, const void *k32, int par, hipStream_t s) {
  tmf_status st = batch_apply(S->b32, k32, S->p.p, S->q.p, S->ctx.sc.iact, s, nullptr, nullptr, false);
  if (st != TMF_OK) return st;
  hipError_t e = blas_cg_step_after_apply<V>(S->ctx, vec<V>(S->d), vec<V>(S->r32), vec<V>(S->p), vec<V>(S->q),
                                             S->part1.p, S->part2.p, S->opt.inner_rtol * S->opt.inner_rtol,
                                             S->opt.inner_maxit, par, s);
  if (e != hipSuccess) return hip_fail(e, "CG step launch");
  return TMF_OK;
}

tmf_status inner_step(tmf_ir *S, const void *k32, int par, hipStream_t s) {
  return S->inner64 ? inner_step_t<double>(S, k32, par, s) : inner_step_t<float>(S, k32, par, s);
}

tmf_status capture(tmf_ir *S, const void *k32) {
  if (S->exec) {
    (void)hipGraphExecDestroy(S->exec);
    S->exec = nullptr;
  }
  if (S->graph) {
    (void)hipGraphDestroy(S->graph);
    S->graph = nullptr;
  }
  hipError_t e = hipStreamBeginCapture(S->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
  tmf_status st = TMF_OK;
  for (int i = 0; i < S->opt.graph_iters && st == TMF_OK; ++i) st = inner_step(S, k32, i & 1, S->stream);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(S->stream, &g);
  if (st != TMF_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  S->graph = g;
  e = hipGraphInstantiate(&S->exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  S->graph_k32 = k32;
  return TMF_OK;
}

}  // namespace

extern "C" {

tmf_status tmf_ir_create(tmf_batch *b64, tmf_batch *b32, const tmf_ir_options *opt, tmf_ir **out) {
  if (!out) return fail(TMF_EINVAL, "out is NULL");
  *out = nullptr;
  if (!b64 || !b32) return fail(TMF_EINVAL, "both batches are required");
  if (b64->prec != TMF_F64) return fail(TMF_EINVAL, "the outer batch must be FP64");
  if (b64->count != b32->count || b64->kind != b32->kind) return fail(TMF_EINVAL, "batches do not match");
  for (int i = 0; i < b64->count; ++i)
    if (b64->ops[i]->mesh != b32->ops[i]->mesh || b64->ops[i]->bc != b32->ops[i]->bc)
      return fail(TMF_EINVAL, "instance %d differs between the batches", i);
  if (b64->ncomp != 1) return fail(TMF_EUNSUPPORTED, "the solver handles scalar operators");
  tmf_ir_options o = opt ? *opt : tmf_ir_options{1e-10, 30, 1e-4, 2000, 16, 1, TMF_PRECOND_JACOBI};
  if (!(o.tol > 0) || o.max_outer < 1 || !(o.inner_rtol > 0) || o.inner_maxit < 1 || o.graph_iters < 2 ||
      (o.graph_iters & 1) || (o.precond != TMF_PRECOND_NONE && o.precond != TMF_PRECOND_JACOBI))
    return fail(TMF_EINVAL, "bad solver options (graph_iters must be even and at least 2)");
  if (o.precond == TMF_PRECOND_JACOBI && b64->kind != TMF_P2_LAPLACE && b64->kind != TMF_P2_DIVKGRAD)
    return fail(TMF_EUNSUPPORTED, "the Jacobi preconditioner needs a scalar P2 kind");
  auto *S = new (std::nothrow) tmf_ir;
  if (!S) return fail(TMF_ENOMEM, "host allocation failed");
  S->b64 = b64;
  S->b32 = b32;
  S->inner64 = b32->prec == TMF_F64;
  S->opt = o;
  const int64_t n = b64->off[b64->count];
  const size_t vb = static_cast<size_t>(n) * (S->inner64 ? 8 : 4);
  const int c = b64->count;
  tmf_status st = S->Ax.alloc(n);
  if (st == TMF_OK) st = S->r64.alloc(n);
  if (st == TMF_OK) st = S->r32.alloc(vb);
  if (st == TMF_OK) st = S->p.alloc(vb);
  if (st == TMF_OK) st = S->q.alloc(vb);
  if (st == TMF_OK) st = S->d.alloc(vb);
  if (st == TMF_OK && o.precond == TMF_PRECOND_JACOBI) st = S->dinv.alloc(vb);
  if (st == TMF_OK) st = S->part1.alloc(b64->nchunks);
  if (st == TMF_OK) st = S->part2.alloc(b64->nchunks);
  if (st == TMF_OK) st = S->scal.alloc(7 * static_cast<size_t>(c));
  if (st == TMF_OK) st = S->it.alloc(c);
  if (st == TMF_OK) st = S->flags.alloc(2 * static_cast<size_t>(c));
  if (st == TMF_OK) {
    hipError_t e = hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking);
    if (e != hipSuccess) st = hip_fail(e, "hipStreamCreate");
  }
  if (st == TMF_OK) {
    // one eager FP32 apply on the zeroed workspace: initialises the launch
    // configuration outside any graph capture
    hipError_t e = S->inner64 ? launch_fill<double>(vec<double>(S->p), n, 0.0, S->stream)
                              : launch_fill<float>(vec<float>(S->p), n, 0.0f, S->stream);
    if (e != hipSuccess) st = hip_fail(e, "workspace fill");
    if (st == TMF_OK) st = batch_apply(b32, has_coeff(b32->kind) ? S->p.p : nullptr, S->p.p, S->q.p, nullptr, S->stream);
    if (st == TMF_OK && (e = hipStreamSynchronize(S->stream)) != hipSuccess) st = hip_fail(e, "warm-up");
  }
  if (st != TMF_OK) {
    delete S;
    return st;
  }
  BlasCtx &x = S->ctx;
  x.chunks = b64->chunks.p;
  x.nchunks = b64->nchunks;
  x.first = b64->first.p;
  x.count = c;
  x.owner = b64->owner.p;
  x.dinv = o.precond == TMF_PRECOND_JACOBI ? S->dinv.p : nullptr;
  x.sc.rnorm = S->scal.p;
  x.sc.bnorm = S->scal.p + c;
  x.sc.rr = S->scal.p + 2 * c;  // two slots
  x.sc.rr0 = S->scal.p + 4 * c;
  x.sc.alpha = S->scal.p + 5 * c;
  x.sc.beta = S->scal.p + 6 * c;
  x.sc.count = c;
  x.sc.it = S->it.p;
  x.sc.oact = S->flags.p;
  x.sc.iact = S->flags.p + c;
  *out = S;
  return TMF_OK;
}

void tmf_ir_destroy(tmf_ir *s) { delete s; }

tmf_status tmf_ir_solve(tmf_ir *S, const double *coeff64, const void *coeff32, const double *b, double *x,
                        tmf_ir_stats *stats, double *relres, tmf_stream stream) {
  if (!S) return fail(TMF_EINVAL, "solver is NULL");
  if (!b || !x || x == b) return fail(TMF_EINVAL, "b and x are required and must differ");
  if (has_coeff(S->b64->kind) != (coeff64 != nullptr && coeff32 != nullptr))
    return fail(TMF_EINVAL, "coefficient fields do not match the operator kind");
  const auto t0 = std::chrono::steady_clock::now();
  const int c = S->b64->count;
  hipStream_t s = S->stream;
  // order the solve after the caller's pending work
  hipEvent_t ev;
  hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
  if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
  e = hipEventRecord(ev, static_cast<hipStream_t>(stream));
  if (e == hipSuccess) e = hipStreamWaitEvent(s, ev, 0);
  (void)hipEventDestroy(ev);
  if (e != hipSuccess) return hip_fail(e, "stream ordering");
  // Jacobi: the inverse diagonal of the FP64 operators for these coefficients
  // (the FP64 residual buffer serves as scratch for the diagonal)
  if (S->opt.precond == TMF_PRECOND_JACOBI) {
    tmf_status sd = batch_diagonal(S->b64, coeff64, S->Ax.p, s);
    if (sd != TMF_OK) return sd;
    e = S->inner64 ? blas_inverse_diagonal<double>(S->ctx, S->Ax.p, vec<double>(S->dinv), s)
                   : blas_inverse_diagonal<float>(S->ctx, S->Ax.p, vec<float>(S->dinv), s);
    if (e != hipSuccess) return hip_fail(e, "inverse diagonal");
  }
  std::vector<uint8_t> flags(2 * c);
  std::vector<double> norms(2 * c);
  std::vector<int> its(c);
  tmf_ir_stats st_out{};
  tmf_status st = TMF_OK;
  bool converged = false;
  for (int outer = 0; outer <= S->opt.max_outer && st == TMF_OK; ++outer) {
    st = batch_apply(S->b64, coeff64, x, S->Ax.p, nullptr, s);
    if (st != TMF_OK) break;
    e = blas_residual(S->ctx, b, S->Ax.p, S->r64.p, S->part1.p, S->part2.p, S->opt.tol, s);
    if (e == hipSuccess) e = hipMemcpyAsync(norms.data(), S->scal.p, 2 * c * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(flags.data(), S->flags.p, c, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      st = hip_fail(e, "outer residual");
      break;
    }
    int active = 0;
    for (int i = 0; i < c; ++i) active += flags[i];
    if (relres)
      for (int i = 0; i < c; ++i) relres[i] = norms[c + i] > 0 ? norms[i] / norms[c + i] : norms[i];
    if (active == 0) {
      converged = true;
      break;
    }
    if (outer == S->opt.max_outer) break;
    st_out.outer = outer + 1;
    e = S->inner64 ? blas_start_inner<double>(S->ctx, S->r64.p, vec<double>(S->r32), vec<double>(S->p),
                                              vec<double>(S->d), S->part1.p, s)
                   : blas_start_inner<float>(S->ctx, S->r64.p, vec<float>(S->r32), vec<float>(S->p),
                                             vec<float>(S->d), S->part1.p, s);
    if (e != hipSuccess) {
      st = hip_fail(e, "inner start");
      break;
    }
    if (S->opt.use_graph && (!S->exec || S->graph_k32 != coeff32)) {
      st = capture(S, coeff32);
      if (st != TMF_OK) break;
    }
    for (;;) {
      if (S->opt.use_graph) {
        e = hipGraphLaunch(S->exec, s);
        if (e != hipSuccess) {
          st = hip_fail(e, "hipGraphLaunch");
          break;
        }
        st_out.graph_launches++;
      } else {
        for (int i = 0; i < S->opt.graph_iters && st == TMF_OK; ++i) st = inner_step(S, coeff32, i & 1, s);
        if (st != TMF_OK) break;
      }
      e = hipMemcpyAsync(flags.data() + c, S->flags.p + c, c, hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipMemcpyAsync(its.data(), S->it.p, c * sizeof(int), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) {
        st = hip_fail(e, "inner convergence check");
        break;
      }
      int inner_active = 0;
      for (int i = 0; i < c; ++i) inner_active += flags[c + i];
      if (inner_active == 0) break;
    }
    if (st != TMF_OK) break;
    int itmax = 0;
    for (int i = 0; i < c; ++i) itmax = std::max(itmax, its[i]);
    st_out.inner_total += itmax;
    e = S->inner64 ? blas_update_x<double>(S->ctx, x, vec<double>(S->d), s)
                   : blas_update_x<float>(S->ctx, x, vec<float>(S->d), s);
    if (e != hipSuccess) st = hip_fail(e, "solution update");
  }
  if (st == TMF_OK) {
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = hip_fail(e, "final synchronise");
  }
  st_out.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  st_out.converged = converged ? 1 : 0;
  if (stats) *stats = st_out;
  if (st != TMF_OK) return st;
  if (!converged) return fail(TMF_ENOTCONV, "iterative refinement did not reach %g in %d outer steps", S->opt.tol,
                              S->opt.max_outer);
  return TMF_OK;
}

}  // extern "C"
