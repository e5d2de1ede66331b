#!/usr/bin/env python3
"""Benchmark: matrix-free finite-element operator apply on one MI355X.

Headline workload (one "step" = one operator application y = A(k) x, the
whole apply path: element kernel with boundary masking, then the seam and
interface reduction):
the P2 variable-coefficient diffusion operator -div(k grad) (equation P2V) in
FP64 on the unit cube split into 6 macro-tetrahedra, refinement level 6
(2,146,689 DoFs), k = 1 + 0.5 sin(2 pi x) cos(2 pi y) z interpolated at the
nodes, x ~ U[-1,1] hashed from the DoF keys (seed 2), homogeneous Dirichlet
rows and columns.  Inputs are resident in HBM before timing starts.

Also reported under "forms": the other operators and precisions on their
workloads (P1 Laplacian at levels 4 and 9, the P1 div(k grad) forward and
fused adjoint at levels 7 and 9, the P2 FP32 apply, the P2 FP64 apply at
level 7, the P2 div(k grad) adjoint on the headline workload, the vector
epsilon operator on the radially blended shell in FP64 and FP32 and its
FP64 adjoint, the N1 curl-curl + mass operator on the cube at level 6 in FP64
and FP32, the stored-local-matrix apply and the degree-2 quadrature variant
on the headline workload) and the
batched FP32-in-FP64 refinement solve (Jacobi-preconditioned and plain).

Prints one JSON line.  `--gpus N` with N > 1 exits: this build runs on one GPU.
"""
import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM = 8.0e12       # B/s, MI355X HBM3E
PEAK_FP64 = 78.6e12     # FLOP/s, vector FP64
PEAK_FP32 = 157.3e12    # FLOP/s, vector FP32

# Arithmetic of each kernel's formulation, counted from the source (add, sub,
# mul = 1 flop, fused multiply-add = 2), per unit the kernel processes.
FLOPS = {
    "p2_divkgrad": 276,        # per micro-tet: gradient coefficients (40), exact k-weights x 840 (58),
                               # W^T sp (84), sigma = (W^T sp) Gs (68), outputs (26)
    "p2_laplace": 184,         # per micro-tet: same without the coefficient weights
    "p1_laplace": 30,          # per DoF: 15-point stencil
    "p1_divkgrad": 312,        # per DoF: 24 incident micro-tets x (4x4 row, mean k, accumulate)
    "p1_adjoint": 1200,        # per DoF: forward row (312) + 24 x bilinear form (37)
    "p2_adjoint": 625,         # per micro-tet: forward apply of gy (276) + coefficient gradient (349:
                               # gradient coefficients 40, h 72, Gam 44, M 112, closed-form derivative of the
                               # collected weights 81)
    "eps_affine": 970,         # per micro-tet
    "n1": 440,                 # per micro-tet: 6 curls, curl u, curl part, U_p, B (beta weights), V, mass part
    "p2_stored": 200,          # per micro-tet: symmetric 10 x 10 matrix-vector product from 55 stored entries
    "p2_quad_per_q": 60,       # per micro-tet and quadrature point: k(q) (10 FMA) and 10 weight updates
    "p2_no_weights": 266,      # per micro-tet: the quadrature-variant apply without its weights (h = sp Gp form)
    "eps_blended_per_q": 321,  # per micro-tet and quadrature point: map point and its closed-form inverse (44),
                               # gradients in xi from P1 coefficients and pulled through the inverse (108), mu (19),
                               # stress (33), pulled back and added to 4 x 9 accumulators (117)
    "eps_blended_per_elem": 600,        # per micro-tet once: 3 x gradient coefficients in xi, 3 x P2 output map
    "eps_blended_adjoint_per_q": 644,   # forward of gy (321) + mu gradient (323: map point and inverse, gradient
                                        # of x pulled through it, its symmetric part pushed through the transpose
                                        # and contracted with the gradient of gy in xi, 10-node scatter)
    "eps_blended_adjoint_per_elem": 1200,  # forward (600) + 6 x gradient coefficients in xi of the mu gradient
}


def parse():
    p = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=100)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--main-only", action="store_true", help="skip the other forms")
    p.add_argument("--form-steps", type=int, default=20)
    p.add_argument("--forms", default=None,
                   help="comma-separated names of the forms to run (default: all), e.g. for profiler runs")
    p.add_argument("--copy-probe", action="store_true",
                   help="accepted for profiler runs: the 1 GiB device copy (a plain copy kernel of known "
                        "size, used to scale HBM byte counters) now always runs first")
    return p.parse_args()


class Hip:
    """HIP events through the runtime PyTorch loaded (same process-wide instance)."""

    def __init__(self):
        self.L = ctypes.CDLL("libamdhip64.so.7")
        self.L.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.L.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.L.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                               ctypes.c_void_p]
        self.L.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]

    def event(self):
        e = ctypes.c_void_p()
        if self.L.hipEventCreate(ctypes.byref(e)) != 0:
            raise RuntimeError("hipEventCreate failed")
        return e

    def elapsed_ms(self, a, b):
        f = ctypes.c_float()
        if self.L.hipEventElapsedTime(ctypes.byref(f), a, b) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return f.value

    def destroy(self, e):
        self.L.hipEventDestroy(e)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def device_inputs(mesh, op, seed, torch, kind_family):
    import workloads as W
    info = mesh.dof_info(op.space, owner=False, boundary=False)
    keys, xyz = info["keys"], info["xyz"]
    x = np.concatenate([W.uniform_from_keys(seed, keys, stream=c) for c in range(op.ncomp)])
    if kind_family == "p2_divkgrad":
        k = W.fields.cube_k(xyz)
    elif kind_family == "p1_divkgrad":
        k = W.fields.perturbed_k(keys, 5)
    elif kind_family == "eps":
        k = W.fields.shell_mu(keys, xyz, 3)
    elif kind_family == "n1":
        k = W.fields.n1_coeff(xyz)
    else:
        k = None
    dt = op.dtype
    xt = torch.tensor(x, dtype=dt, device="cuda")
    kt = torch.tensor(k, dtype=dt, device="cuda") if k is not None else None
    return xt, kt


# Event pairs bracket the element kernel of every EVENT_EVERY-th step of the
# timed region: an event record is a queue packet of its own, and a pair on
# every step added about 6 us to a 55 us step.
EVENT_EVERY = 10


def sampled_events(hip, steps):
    """Event pairs for the sampled steps of a timed region of `steps` steps (None elsewhere)."""
    return [(hip.event(), hip.event()) if i % EVENT_EVERY == 0 else (None, None) for i in range(steps)]


def kernel_mean_ms(hip, evs, stats=None):
    """Mean element-kernel duration over the sampled steps (median and minimum into `stats`);
    releases the events."""
    ms = [hip.elapsed_ms(b, a) for b, a in evs if b is not None]
    for b, a in evs:
        if b is not None:
            hip.destroy(b)
            hip.destroy(a)
    if stats is not None:
        stats["kernel_ms_median"] = round(float(np.median(ms)), 5)
        stats["kernel_ms_min"] = round(float(np.min(ms)), 5)
    return float(np.mean(ms))


def clock_state():
    """Current GPU clocks as rocm-smi reports them (None when it is not available).

    rocm-smi is a Python script: it is run by this interpreter directly, since
    its `env` shebang would replace a process by another one.  Under a profiler
    (a preloaded tool library, which would also load into the child) no clocks
    are read."""
    import shutil
    import subprocess
    env = os.environ
    if ("rocprof" in env.get("LD_PRELOAD", "") + env.get("HSA_TOOLS_LIB", "")
            or any(k.startswith("ROCPROF") for k in env)):
        return None
    smi = shutil.which("rocm-smi")
    if smi is None:
        return None
    try:
        r = subprocess.run([sys.executable, smi, "--showclocks"], capture_output=True, text=True, timeout=20)
    except (OSError, subprocess.SubprocessError):
        return None
    lines = [ln.strip() for ln in r.stdout.splitlines() if "clock level" in ln.lower() or "Mhz" in ln]
    return lines[:8] or None


def time_apply(op, x, k, y, steps, warmup, hip, torch, fn=None, stats=None):
    """Warm up, then time exactly `steps` applies; returns (wall ms/step, kernel ms mean)."""
    import paper_2404_08371_amd as T
    L = T.lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    pk = ctypes.c_void_p(k.data_ptr()) if k is not None else None
    px, py = ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr())
    for _ in range(warmup):
        T.check(L.tmf_apply(op.handle, pk, px, py, stream)) if fn is None else fn(None, None)
    evs = sampled_events(hip, steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b, a in evs:
        if fn is None:
            T.check(L.tmf_apply_timed(op.handle, pk, px, py, stream, b, a))
        else:
            fn(b, a)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    return wall, kernel_mean_ms(hip, evs, stats)


def graph_rate(op, x, k, y, torch, per_graph=50, replays=5):
    """`per_graph` applies captured into one HIP graph (torch's graph capture on a side stream)
    and replayed `replays` times: (us per apply, whether the replayed result equals an eager
    apply bit for bit).  Launch overhead is paid once per replay instead of once per apply."""
    ref = torch.empty_like(y)
    op.apply(x, k, out=ref)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        op.apply(x, k, out=y)  # anything the apply sets up lazily, outside the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(per_graph):
            op.apply(x, k, out=y)
    y.zero_()
    g.replay()
    torch.cuda.synchronize()
    same = bool(torch.equal(y, ref))
    t0 = time.perf_counter()
    for _ in range(replays):
        g.replay()
    torch.cuda.synchronize()
    us = (time.perf_counter() - t0) * 1e6 / (replays * per_graph)
    del g
    return us, same


def n_elements(mesh_nt, level):
    n = 2 ** level
    return mesh_nt * n ** 3


KERNEL_SOURCES = ("kernels_tile.hip", "tmf_internal.h")


def kernel_code_hash(sources=KERNEL_SOURCES, csrc=None):
    """Hash of the element kernels' code with comments and whitespace removed: counters taken
    on one version stay valid across edits of its comments, and only those."""
    import re
    csrc = csrc or os.path.join(ROOT, "paper_2404_08371_amd", "csrc")
    h = hashlib.sha256()
    for name in sources:
        with open(os.path.join(csrc, name)) as f:
            txt = f.read()
        txt = re.sub(r"/\*.*?\*/", " ", txt, flags=re.S)
        txt = re.sub(r"//[^\n]*", " ", txt)
        h.update(name.encode() + b"\0" + " ".join(txt.split()).encode() + b"\0")
    return h.hexdigest()[:16]


# tile-shape indices from this one on are the marching shapes (see the tile-shape table of the library)
MARCH_CFG0 = 4


def traffic_for(kernel_key, tile, field="bytes_per_launch_by_tile"):
    """HBM bytes per launch of one element-kernel tile shape, keyed "TXxTYxTZ" (a marching column:
    "march:TXxTYxTZ"), or, with field "seam_bytes_per_launch_by_tile", of the seam reduction
    launched after it, from the committed
    rocprofv3 counter runs (FETCH_SIZE and WRITE_SIZE, each scaled by what it reads for a 1 GiB copy);
    None when the kernel code has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    ent = data.get(kernel_key)
    if not ent or kernel_code_hash(tuple(ent.get("sources", ()))) != ent.get("code_sha256_16"):
        return None
    return ent.get(field, {}).get(tile)


def batched_solve(torch, T, W, hip, steps):
    """Batched P2 div(k grad): FP32 / FP64 batched applies and the refined solve to 1e-10."""
    levels = W.fields.batch_levels()
    a, phi = W.fields.batch_k_params()
    v, t = W.meshes.ref_tet()
    meshes = [T.Mesh(v, t, int(lv)) for lv in levels]
    infos = [mm.dof_info(2, owner=False) for mm in meshes]
    ops64 = [T.Operator(mm, T.P2_DIVKGRAD, T.F64) for mm in meshes]
    ops32 = [T.Operator(mm, T.P2_DIVKGRAD, T.F32) for mm in meshes]
    b64, b32 = T.Batch(ops64), T.Batch(ops32)
    K = b64.concat([torch.tensor(W.fields.batch_k(inf["xyz"], a[i], phi[i]), device="cuda")
                    for i, inf in enumerate(infos)])
    Xs = b64.concat([torch.tensor(W.uniform_from_keys(11, inf["keys"]) * (~inf["boundary"]), device="cuda")
                     for inf in infos])
    B = b64.apply(Xs, K)
    dofs = sum(op.n_unique for op in ops64)
    res = {"instances": len(levels), "levels": [int(lv) for lv in levels], "dofs": dofs}
    L = T.lib()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for name, b, kk, xx in (("fp64", b64, K, Xs), ("fp32", b32, K.float(), Xs.float())):
        yy = torch.empty_like(xx)
        cfg, ms = b.autotune(xx, kk, yy, reps=3)
        evs = sampled_events(hip, steps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for e0, e1 in evs:
            T.check(L.tmf_batch_apply_timed(b.handle, ctypes.c_void_p(kk.data_ptr()), ctypes.c_void_p(xx.data_ptr()),
                                            ctypes.c_void_p(yy.data_ptr()), None, st, e0, e1))
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / steps
        kern = kernel_mean_ms(hip, evs)
        res["apply_%s_mdofs" % name] = round(dofs / (wall * 1e-3) / 1e6, 1)
        res["apply_%s_kernel_ms" % name] = round(kern, 4)
        res["apply_%s_tile" % name] = cfg
    # the default inner iteration is Jacobi-preconditioned CG; the plain CG
    # solve is reported beside it
    for tag, pc in (("", T.PRECOND_JACOBI), ("_noprecond", T.PRECOND_NONE)):
        solver = T.IRSolver(b64, b32, tol=1e-10, precond=pc)
        X = torch.zeros_like(B)
        solver.solve(B, X, K, K.float())  # warm-up (graph capture)
        X.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats, relres = solver.solve(B, X, K, K.float())
        tsol = time.perf_counter() - t0
        err = float(((X - Xs).norm() / Xs.norm()).item())
        res.update({"solve_s" + tag: round(tsol, 4), "outer" + tag: stats["outer"],
                    "inner_iterations" + tag: stats["inner_total"], "graph_launches" + tag: stats["graph_launches"],
                    "max_relres_fp64" + tag: float(relres.max()), "rel_err_vs_exact" + tag: err,
                    "converged" + tag: stats["converged"]})
        del solver
    # the plain FP64 form on the same GPU: Jacobi-preconditioned CG with the FP64 apply and FP64
    # vectors (the same solver with the FP64 batch as its inner batch, inner tolerance below the
    # outer one, so the first outer step solves and the second confirms)
    solver = T.IRSolver(b64, b64, tol=1e-10, inner_rtol=1e-11, precond=T.PRECOND_JACOBI)
    X = torch.zeros_like(B)
    solver.solve(B, X, K, K)  # warm-up (graph capture)
    X.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats, relres = solver.solve(B, X, K, K)
    tsol = time.perf_counter() - t0
    err = float(((X - Xs).norm() / Xs.norm()).item())
    res.update({"solve_s_fp64_cg": round(tsol, 4), "outer_fp64_cg": stats["outer"],
                "inner_iterations_fp64_cg": stats["inner_total"], "max_relres_fp64_cg": float(relres.max()),
                "rel_err_vs_exact_fp64_cg": err, "converged_fp64_cg": stats["converged"],
                "refined_speedup_vs_fp64_cg": round(tsol / res["solve_s"], 3)})
    del solver
    return res


def host_cpu():
    """Host CPU description from lscpu (model, sockets, cores per socket, threads per core)."""
    import subprocess
    try:
        r = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20)
    except (OSError, subprocess.SubprocessError):
        return None
    want = {"Model name": "model", "Socket(s)": "sockets", "Core(s) per socket": "cores_per_socket",
            "Thread(s) per core": "threads_per_core", "CPU(s)": "logical_cpus"}
    out = {}
    for ln in r.stdout.splitlines():
        k, _, v = ln.partition(":")
        if k.strip() in want:
            out[want[k.strip()]] = v.strip()
    return out or None


def usable_cores():
    """Cores this process may run on (its affinity mask), at most 16: the CPU share of one GPU."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


_BASE = {}


def _baseline_share(i):
    """Worker: one share of the oracle's element loop, written into row i of the shared buffer."""
    from threadpoolctl import threadpool_limits
    b = _BASE
    with threadpool_limits(1):
        b["out"][i, :] = b["pr"].local_sum(b["x"], b["k"], share=(i, b["nw"]))
    return i


def cpu_baseline_c2(reps=10):
    """The oracle, as it stands, on full applies of the headline workload, its element loop split
    over the host's cores.  Each worker process runs a share of the oracle's element batches
    (single-threaded numpy); the parent adds the shares, then runs the oracle's interface sum and
    mask.  Runs before anything touches the GPU: the workers are forked from this process."""
    import mmap
    import multiprocessing as mp
    import oracle as O
    import workloads as W
    v, t = W.meshes.kuhn_cube()
    pr = O.Problem(v, t, 6, O.P2_DIVKGRAD, O.BC_DIRICHLET_ZERO)
    x = W.uniform_from_keys(2, pr.keys)
    k = W.fields.cube_k(pr.xyz)
    nw = usable_cores()
    buf = mmap.mmap(-1, nw * x.size * 8)  # anonymous shared memory, inherited by the forked workers
    out = np.frombuffer(buf, dtype=np.float64).reshape(nw, x.size)
    _BASE.update(pr=pr, x=x, k=k, nw=nw, out=out)
    times = []
    with mp.get_context("fork").Pool(nw) as pool:
        for _ in range(reps):
            t0 = time.perf_counter()
            pool.map(_baseline_share, range(nw))
            y = pr.finish(out.sum(0))
            times.append(time.perf_counter() - t0)
    _BASE.clear()
    del out
    buf.close()
    ref_norm = float(np.linalg.norm(y))
    dt = float(np.median(times))
    return {"value": pr.n_unique / dt / 1e6, "unit": "MDoF/s", "cores": nw, "kind": "oracle",
            "host": host_cpu(), "reps": reps, "s_per_apply_median": round(dt, 4),
            "s_per_apply_min": round(float(np.min(times)), 4), "y_norm": ref_norm,
            "sample": "%d full FP64 applies of the headline workload (Kuhn cube, level 6, %d DoFs) by the numpy "
                      "oracle, its element batches split over %d single-threaded worker processes, shares added "
                      "and finished (interface sum, mask) in the parent; setup excluded; median %.2f s per apply"
                      % (reps, pr.n_unique, nw, dt)}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (sharding by "
              "macro-tetrahedra is described in DESIGN.md); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    cpu_base = None
    if not args.no_cpu_baseline:
        # first, while no GPU handle exists in this process (its workers are forked)
        log("cpu baseline (oracle) ...")
        cpu_base = cpu_baseline_c2()
        log("cpu baseline %.3f MDoF/s on %d cores" % (cpu_base["value"], cpu_base["cores"]))
    import torch
    import paper_2404_08371_amd as T
    import workloads as W
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    hip = Hip()
    torch.manual_seed(0)
    # achievable bandwidth of a plain device copy (1 GiB read + 1 GiB written),
    # reported beside the published HBM peak; with --copy-probe it also serves
    # to scale the HBM byte counters of a profiler run
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 3 * 2 * src.numel() * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    log("device copy: %.0f GB/s" % copy_gbs)
    del src, dst

    # ------------------------------------------------------------ headline
    log("headline: P2 div(k grad) FP64, Kuhn cube level 6")
    v, t = W.meshes.kuhn_cube()
    mesh = T.Mesh(v, t, 6)
    op = T.Operator(mesh, T.P2_DIVKGRAD, T.F64, T.BC_DIRICHLET_ZERO)
    x, k = device_inputs(mesh, op, 2, torch, "p2_divkgrad")
    y = torch.empty_like(x)
    cfg, ms = ctypes.c_int(), ctypes.c_float()
    T.check(T.lib().tmf_op_autotune(op.handle, ctypes.c_void_p(k.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                    ctypes.c_void_p(y.data_ptr()),
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), 10,
                                    ctypes.byref(cfg), ctypes.byref(ms)))
    tx, ty, tz = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    T.check(T.lib().tmf_op_tile_shape(op.handle, cfg.value, ctypes.byref(tx), ctypes.byref(ty), ctypes.byref(tz)))
    log("autotuned tile", (tx.value, ty.value, tz.value), "%.4f ms" % ms.value)
    kstats = {}
    wall, kern = time_apply(op, x, k, y, args.steps, args.warmup, hip, torch, stats=kstats)
    # cold variant: a 512 MB write before each apply evicts the 256 MB last-level
    # cache (the headline's 52.7 MB of inputs fit in it); element kernel and whole
    # apply timed with events around each call
    scratch = torch.empty(1 << 26, dtype=torch.float64, device="cuda")
    L0 = T.lib()
    st0 = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    cold_k, cold_s = [], []
    for _ in range(10):
        scratch.fill_(1.0)
        e0, e1, e2, e3 = hip.event(), hip.event(), hip.event(), hip.event()
        hip.L.hipEventRecord(e0, st0)
        T.check(L0.tmf_apply_timed(op.handle, ctypes.c_void_p(k.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                   ctypes.c_void_p(y.data_ptr()), st0, e1, e2))
        hip.L.hipEventRecord(e3, st0)
        torch.cuda.synchronize()
        cold_k.append(hip.elapsed_ms(e1, e2))
        cold_s.append(hip.elapsed_ms(e0, e3))
        for e in (e0, e1, e2, e3):
            hip.destroy(e)
    del scratch
    kstats["cold_kernel_ms_median"] = round(float(np.median(cold_k)), 5)
    kstats["cold_step_ms_median"] = round(float(np.median(cold_s)), 5)
    # the same step replayed from a HIP graph of 100 applies (launch overhead amortised)
    gus, gsame = graph_rate(op, x, k, y, torch, per_graph=100)
    kstats["graph_step_ms"] = round(gus * 1e-3, 5)
    kstats["graph_step_equals_eager"] = gsame
    nel = n_elements(6, 6)
    flops = nel * FLOPS["p2_divkgrad"]
    bytes_alg = 3 * op.n_local * 8
    t_alu, t_hbm = flops / PEAK_FP64, bytes_alg / PEAK_HBM
    bound = "alu" if t_alu >= t_hbm else "hbm"
    if bound == "alu":
        achieved, peak, unit = flops / (kern * 1e-3) / 1e12, PEAK_FP64 / 1e12, "TFLOP/s"
    else:
        achieved, peak, unit = bytes_alg / (kern * 1e-3) / 1e9, PEAK_HBM / 1e9, "GB/s"
    tile = (tx.value, ty.value, tz.value)
    # marching shapes (a column of 4 x 4 x 4 sub-boxes) run another kernel than a box of the same size
    tkey = ("march:" if cfg.value >= MARCH_CFG0 else "") + "x".join(str(v) for v in tile)
    traffic = traffic_for("p2_divkgrad_fp64_cube6", tkey)
    seam_traffic = traffic_for("p2_divkgrad_fp64_cube6", tkey, "seam_bytes_per_launch_by_tile")
    value = op.n_unique / (wall * 1e-3) / 1e6
    out = {
        "metric": "operator-apply MDoF/s (FP64 vs FP32-refined, fwd+adjoint) and % HBM roofline",
        "value": round(value, 2), "unit": "MDoF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(wall, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "P2 -div(k grad) apply, FP64, unit cube as 6 macro-tets, level 6, "
                               "k=1+0.5 sin(2 pi x)cos(2 pi y)z nodal, Dirichlet, x~U[-1,1] seed 2",
                   "dofs": op.n_unique, "local_slots": op.n_local, "micro_tets": nel,
                   "tile": [tx.value, ty.value, tz.value], "parallelism": "single GPU"},
        "roofline": {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
                     "frac": round(achieved / peak, 4), "traffic": traffic,
                     "kernel_ms": round(kern, 5), "flops_per_launch": flops,
                     "alg_bytes_per_launch": bytes_alg,
                     "hbm_frac": round(bytes_alg / (kern * 1e-3) / PEAK_HBM, 4),
                     # the whole apply (element kernel and seam / interface reduction), timed as the
                     # step: its algorithmic bytes over the step time, and its measured HBM bytes
                     "step_ms": round(wall, 5),
                     "step_hbm_frac": round(bytes_alg / (wall * 1e-3) / PEAK_HBM, 4),
                     "step_traffic": (traffic + seam_traffic) if traffic is not None and seam_traffic is not None
                     else None,
                     "device_copy_GBps": round(copy_gbs, 1), **kstats},
        "clocks": clock_state(),
    }
    log("headline %.1f MDoF/s, kernel %.4f ms, step %.4f ms" % (value, kern, wall))

    # --------------------------------------------------------------- forms
    if not args.main_only:
        forms = {}

        sel = None if args.forms is None else set(args.forms.split(","))

        def want(name):
            return sel is None or name in sel

        def form(name, mesh, op, fam, seed, flops_launch, bytes_launch, peak_flops, steps, adjoint=False,
                 dofs=None, graph=False):
            if not want(name):
                return
            xx, kk = device_inputs(mesh, op, seed, torch, fam)
            yy = torch.empty_like(xx)
            if op.space == 2:
                c2, m2 = ctypes.c_int(), ctypes.c_float()
                T.check(T.lib().tmf_op_autotune(op.handle, ctypes.c_void_p(kk.data_ptr()) if kk is not None else None,
                                                ctypes.c_void_p(xx.data_ptr()), ctypes.c_void_p(yy.data_ptr()),
                                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), 3,
                                                ctypes.byref(c2), ctypes.byref(m2)))
            fn = None
            if adjoint:
                gk = torch.empty_like(kk)
                gy = xx.clone()
                L = T.lib()
                st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

                def fn(b, a):
                    if b is not None:
                        hip.L.hipEventRecord(b, st)
                    T.check(L.tmf_apply_adjoint(op.handle, ctypes.c_void_p(kk.data_ptr()),
                                                ctypes.c_void_p(xx.data_ptr()), ctypes.c_void_p(gy.data_ptr()),
                                                ctypes.c_void_p(yy.data_ptr()), ctypes.c_void_p(gk.data_ptr()), st))
                    if a is not None:
                        hip.L.hipEventRecord(a, st)
            w, kms = time_apply(op, xx, kk, yy, steps, 3, hip, torch, fn)
            nd = dofs if dofs is not None else op.n_unique * op.ncomp
            r = {"dofs": nd, "mdofs": round(nd / (w * 1e-3) / 1e6, 2),
                 "ms_per_apply": round(w, 5), "kernel_ms": round(kms, 5),
                 "hbm_frac": round(bytes_launch / (kms * 1e-3) / PEAK_HBM, 4),
                 "alu_frac": round(flops_launch / (kms * 1e-3) / peak_flops, 4)}
            if graph:
                gus, same = graph_rate(op, xx, kk, yy, torch)
                r["us_per_launch"] = round(w * 1e3, 2)
                r["graph_us_per_apply"] = round(gus, 2)
                r["graph_mdofs"] = round(nd / (gus * 1e-6) / 1e6, 2)
                r["graph_equals_eager"] = same
            forms[name] = r
            log(name, r)
            del xx, kk, yy

        vr, tr = W.meshes.ref_tet()
        for lvl in (4, 9):
            m1 = T.Mesh(vr, tr, lvl)
            o1 = T.Operator(m1, T.P1_LAPLACE, T.F64)
            form("p1_laplace_fp64_reftet_l%d" % lvl, m1, o1, "p1", 1, o1.n_local * FLOPS["p1_laplace"],
                 16 * o1.n_local, PEAK_FP64, args.form_steps, graph=lvl == 4)
        for lvl in (7, 9):
            m1 = T.Mesh(vr, tr, lvl)
            o1 = T.Operator(m1, T.P1_DIVKGRAD, T.F64)
            form("p1_divkgrad_fwd_fp64_reftet_l%d" % lvl, m1, o1, "p1_divkgrad", 6,
                 o1.n_local * FLOPS["p1_divkgrad"], 24 * o1.n_local, PEAK_FP64, args.form_steps)
            form("p1_divkgrad_adjoint_fp64_reftet_l%d" % lvl, m1, o1, "p1_divkgrad", 6,
                 o1.n_local * FLOPS["p1_adjoint"], 40 * o1.n_local, PEAK_FP64, args.form_steps, adjoint=True)
        o32 = T.Operator(mesh, T.P2_DIVKGRAD, T.F32)
        form("p2_divkgrad_fp32_cube_l6", mesh, o32, "p2_divkgrad", 2, nel * FLOPS["p2_divkgrad"],
             12 * o32.n_local, PEAK_FP32, args.form_steps)
        m7 = T.Mesh(v, t, 7)
        o7 = T.Operator(m7, T.P2_DIVKGRAD, T.F64)
        form("p2_divkgrad_fp64_cube_l7", m7, o7, "p2_divkgrad", 2, n_elements(6, 7) * FLOPS["p2_divkgrad"],
             24 * o7.n_local, PEAK_FP64, args.form_steps)
        del o7, m7
        # N1 curl-curl + mass on the cube, level 6: DoFs = edges (unique P2 slots minus vertices);
        # bytes: x, y (8 B) and the orientation sign (1 B) per slot, alpha and beta per vertex slot
        nv_local, nv_unique = mesh.layout(1)
        for prec, nm, pk, bpd in ((T.F64, "fp64", PEAK_FP64, 8), (T.F32, "fp32", PEAK_FP32, 4)):
            on = T.Operator(mesh, T.N1_CURLCURL, prec)
            form("n1_curlcurl_%s_cube_l6" % nm, mesh, on, "n1", 5, nel * FLOPS["n1"],
                 (2 * bpd + 1) * on.n_local + 2 * bpd * nv_local, pk, args.form_steps,
                 dofs=on.n_unique - nv_unique)
            del on
        # quadrature (under-integration) variant with the 4-point degree-2 rule, headline workload
        oq = T.Operator(mesh, T.P2_DIVKGRAD, T.F64, rule=W.quadrature.rule_degree2())
        form("p2_divkgrad_quad_degree2_fp64_cube_l6", mesh, oq, "p2_divkgrad", 2,
             nel * (FLOPS["p2_no_weights"] + 4 * FLOPS["p2_quad_per_q"]), 24 * oq.n_local, PEAK_FP64,
             args.form_steps)
        del oq
        # stored local matrices (the precomputed-matrix comparison) on the headline workload:
        # 55 FP64 entries per micro-tet streamed from HBM, plus x and y
        def stored_form():
            ost = T.Operator(mesh, T.P2_DIVKGRAD, T.F64)
            xs_, ks_ = device_inputs(mesh, ost, 2, torch, "p2_divkgrad")
            ost.store_matrices(ks_)
            ys_ = torch.empty_like(xs_)
            Ls = T.lib()
            sts = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

            def fn_stored(b, a):
                if b is not None:
                    hip.L.hipEventRecord(b, sts)
                T.check(Ls.tmf_apply_stored(ost.handle, ctypes.c_void_p(xs_.data_ptr()), ctypes.c_void_p(ys_.data_ptr()),
                                            sts))
                if a is not None:
                    hip.L.hipEventRecord(a, sts)
            w_s, k_s = time_apply(ost, xs_, ks_, ys_, args.form_steps, 3, hip, torch, fn_stored)
            b_s = 55 * 8 * nel + 16 * ost.n_local
            forms["p2_divkgrad_stored_matrices_fp64_cube_l6"] = {
                "dofs": ost.n_unique, "mdofs": round(ost.n_unique / (w_s * 1e-3) / 1e6, 2), "ms_per_apply": round(w_s, 5),
                "kernel_ms": round(k_s, 5), "stored_bytes": 55 * 8 * nel,
                "hbm_frac": round(b_s / (k_s * 1e-3) / PEAK_HBM, 4),
                "alu_frac": round(nel * FLOPS["p2_stored"] / (k_s * 1e-3) / PEAK_FP64, 4),
                "matrix_free_speedup": round(w_s / wall, 2)}
            log("p2_divkgrad_stored_matrices_fp64_cube_l6", forms["p2_divkgrad_stored_matrices_fp64_cube_l6"])
            del ost, xs_, ks_, ys_

        if want("p2_divkgrad_stored_matrices_fp64_cube_l6"):
            stored_form()
        # P2 adjoint (gx = L(k) gy and gk), two element launches + two seam reductions;
        # 48 B per slot (gy, k -> gx; x, gy -> gk)
        o6a = T.Operator(mesh, T.P2_DIVKGRAD, T.F64)
        form("p2_divkgrad_adjoint_fp64_cube_l6", mesh, o6a, "p2_divkgrad", 2, nel * FLOPS["p2_adjoint"],
             48 * o6a.n_local, PEAK_FP64, args.form_steps, adjoint=True)
        del o6a
        vs, ts = W.meshes.octahedral_shell()
        ms6 = T.Mesh(vs, ts, 6, T.MAP_SHELL_RADIAL)
        rule = W.quadrature.rule_degree5()
        for prec, nm, pk, bpd in ((T.F64, "fp64", PEAK_FP64, 8), (T.F32, "fp32", PEAK_FP32, 4)):
            oe = T.Operator(ms6, T.P2V_EPSILON, prec, T.BC_DIRICHLET_ZERO, rule=rule)
            form("eps_blended_%s_shell_l6" % nm, ms6, oe, "eps", 4,
                 n_elements(24, 6) * (14 * FLOPS["eps_blended_per_q"] + FLOPS["eps_blended_per_elem"]),
                 7 * bpd * oe.n_local, pk, 5)
            if prec == T.F64:
                # adjoint: gx = L(mu) gy and the mu gradient (gy, mu -> gx; x, gy -> gmu)
                form("eps_blended_adjoint_fp64_shell_l6", ms6, oe, "eps", 4,
                     n_elements(24, 6) * (14 * FLOPS["eps_blended_adjoint_per_q"]
                                          + FLOPS["eps_blended_adjoint_per_elem"]), 14 * bpd * oe.n_local, pk, 5,
                     adjoint=True)
            del oe
        # batched mixed-precision solve: 32 reference-tet instances, levels in {3..7}
        if want("batched_ir_cg_p2_divkgrad_32x"):
            log("batched FP32-in-FP64 refinement, 32 instances")
            forms["batched_ir_cg_p2_divkgrad_32x"] = batched_solve(torch, T, W, hip, args.form_steps)
            log("batched_ir_cg_p2_divkgrad_32x", forms["batched_ir_cg_p2_divkgrad_32x"])
        out["forms"] = forms

    if cpu_base is not None:
        out["cpu_baseline"] = cpu_base
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
