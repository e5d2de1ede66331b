"""GPU parity at the full sizes of the benchmark workloads.

* P1 Laplacian, reference tet, level 4 (969 DoFs): every entry vs the oracle;
  and at level 7 (both boundary conditions) and on the 6-macro cube at level 6,
  where the stencil kernel's tiles repeat in every direction.
* P2 -div(k grad), unit cube as 6 macro-tets, level 6 (2,146,689 DoFs), in the
  launch configuration the benchmark times (autotuned tile shape): every entry
  vs the oracle, FP64 relative 1e-12.
* Vector epsilon operator on the radially blended shell (24 macro-tets,
  level 6, 25,363,206 DoFs), FP64 and FP32: 400 seeded sample rows (with all
  their copies) computed one by one by the oracle; plus the property that
  constant fields are in the kernel of the operator without boundary
  conditions, at full size.
* P1 Laplacian at level 9 (22.6M DoFs, the bandwidth benchmark): properties
  that hold at any size -- A 1 = 0 and A (linear) = 0 on interior rows
  without boundary conditions, symmetry x.Ay = y.Ax with them.
* Batched P2 -div(k grad): 32 reference-tet instances, levels drawn from
  {3..7}, refined FP32-in-FP64 CG to relative residual 1e-10, the residual
  re-evaluated by the oracle's FP64 operator.
"""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2404_08371_amd as T
import workloads as W

pytestmark = pytest.mark.gpu


def rel(y, ref):
    return np.linalg.norm(y - ref) / np.linalg.norm(ref), np.abs(y - ref).max() / np.abs(ref).max()


def test_p1_laplace_reference_tet_level4_full():
    v, t = W.meshes.ref_tet()
    m = T.Mesh(v, t, 4)
    op = T.Operator(m, T.P1_LAPLACE, T.F64)
    info = m.dof_info(1)
    y = op.apply(torch.tensor(W.uniform_from_keys(1, info["keys"]), device="cuda")).cpu().numpy()
    pr = O.Problem(v, t, 4, O.P1_LAPLACE)
    e2, ei = rel(y, pr.apply(W.uniform_from_keys(1, pr.keys)))
    assert e2 <= 1e-12 and ei <= 1e-12
    assert pr.n_unique == 969 and (~pr.boundary).sum() == 455


@pytest.mark.parametrize("mesh,level,bc", [("ref", 7, O.BC_DIRICHLET_ZERO), ("ref", 7, O.BC_NONE),
                                           ("cube", 6, O.BC_DIRICHLET_ZERO)])
def test_p1_laplace_multi_tile_full(mesh, level, bc):
    """Every entry vs the oracle at sizes where the stencil kernel's tiles
    (62 points x 4 rows x 4 planes) repeat in every direction with ragged ends."""
    print("P1 multi-tile case", mesh, level, bc, flush=True)
    v, t = {"ref": W.meshes.ref_tet, "cube": W.meshes.kuhn_cube}[mesh]()
    m = T.Mesh(v, t, level)
    op = T.Operator(m, T.P1_LAPLACE, T.F64, bc)
    info = m.dof_info(1, owner=False, boundary=False)
    y = op.apply(torch.tensor(W.uniform_from_keys(1, info["keys"]), device="cuda")).cpu().numpy()
    pr = O.Problem(v, t, level, O.P1_LAPLACE, bc)
    e2, ei = rel(y, pr.apply(W.uniform_from_keys(1, pr.keys)))
    print("errors", e2, ei)
    assert e2 <= 1e-12 and ei <= 1e-12


def test_p2_divkgrad_cube_level6_full_in_bench_configuration():
    print("C2 full-size case", flush=True)
    v, t = W.meshes.kuhn_cube()
    m = T.Mesh(v, t, 6)
    op = T.Operator(m, T.P2_DIVKGRAD, T.F64)
    info = m.dof_info(2, owner=False, boundary=False)
    x = torch.tensor(W.uniform_from_keys(2, info["keys"]), device="cuda")
    k = torch.tensor(W.fields.cube_k(info["xyz"]), device="cuda")
    import ctypes
    y = torch.empty_like(x)
    cfg, ms = ctypes.c_int(), ctypes.c_float()
    T.check(T.lib().tmf_op_autotune(op.handle, ctypes.c_void_p(k.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                    ctypes.c_void_p(y.data_ptr()),
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), 3,
                                    ctypes.byref(cfg), ctypes.byref(ms)))
    y = op.apply(x, k).cpu().numpy()
    pr = O.Problem(v, t, 6, O.P2_DIVKGRAD, O.BC_DIRICHLET_ZERO)
    assert pr.n_unique == 129 ** 3
    ref = pr.apply(W.uniform_from_keys(2, pr.keys), W.fields.cube_k(pr.xyz))
    e2, ei = rel(y, ref)
    print("C2 tile cfg", cfg.value, "errors", e2, ei)
    assert e2 <= 1e-12 and ei <= 1e-12


@pytest.fixture(scope="module")
def shell6():
    vs, ts = W.meshes.octahedral_shell()
    qb, qw = W.quadrature.rule_degree5()
    m = T.Mesh(vs, ts, 6, T.MAP_SHELL_RADIAL)
    info = m.dof_info(2, owner=False, boundary=False)
    pr = O.Problem(vs, ts, 6, O.P2V_EPSILON, O.BC_DIRICHLET_ZERO, map_=O.MAP_SHELL_RADIAL, qbary=qb, qw=qw)
    return m, info, pr, (qb, qw)


@pytest.mark.parametrize("prec", [T.F64, T.F32])
def test_epsilon_shell_level6_sampled_rows(shell6, prec):
    print("C3 sampled case", prec, flush=True)
    m, info, pr, rule = shell6
    assert pr.n_unique * 3 == 25363206
    op = T.Operator(m, T.P2V_EPSILON, prec, T.BC_DIRICHLET_ZERO, rule=rule)
    dt = op.dtype
    x = np.concatenate([W.uniform_from_keys(4, info["keys"], stream=c) for c in range(3)])
    mu = W.fields.shell_mu(info["keys"], info["xyz"], 3)
    y = op.apply(torch.tensor(x, dtype=dt, device="cuda"), torch.tensor(mu, dtype=dt, device="cuda"))
    y = y.double().cpu().numpy()
    rows = np.random.default_rng(12).choice(pr.n_local, 400, replace=False)
    xo = np.concatenate([W.uniform_from_keys(4, pr.keys, stream=c) for c in range(3)])
    ref = pr.apply(xo, W.fields.shell_mu(pr.keys, pr.xyz, 3), rows=rows)
    idx = np.concatenate([rows + c * pr.n_local for c in range(3)])
    scale = np.abs(ref[idx]).max()
    err = np.abs(y[idx] - ref[idx]).max() / scale
    print("C3 sampled max rel err", err)
    assert err <= (1e-12 if prec == T.F64 else 1e-5)


def test_epsilon_shell_level6_constants_in_kernel(shell6):
    m, info, pr, rule = shell6
    op = T.Operator(m, T.P2V_EPSILON, T.F64, T.BC_NONE, rule=rule)
    mu = torch.tensor(W.fields.shell_mu(info["keys"], info["xyz"], 3), device="cuda")
    u = torch.zeros(3 * op.n_local, dtype=torch.float64, device="cuda")
    u[op.n_local:2 * op.n_local] = 1.0
    y = op.apply(u, mu)
    xr = torch.tensor(np.concatenate([W.uniform_from_keys(4, info["keys"], stream=c) for c in range(3)]),
                      device="cuda")
    scale = op.apply(xr, mu).abs().max().item()
    assert y.abs().max().item() <= 1e-11 * scale


def test_p1_laplace_level9_properties():
    print("P1 level 9 properties", flush=True)
    v, t = W.meshes.ref_tet()
    m = T.Mesh(v, t, 9)
    opn = T.Operator(m, T.P1_LAPLACE, T.F64, T.BC_NONE)
    opd = T.Operator(m, T.P1_LAPLACE, T.F64, T.BC_DIRICHLET_ZERO)
    info = m.dof_info(1, keys=False, owner=False)
    ones = torch.ones(opn.n_local, dtype=torch.float64, device="cuda")
    r = torch.rand(opn.n_local, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(0))
    scale = opn.apply(r).abs().max().item()
    assert opn.apply(ones).abs().max().item() <= 1e-12 * scale
    # The linear field is built on the device, with no host copy between it and
    # the apply (so stream ordering is exercised), by elementwise products; it is
    # checked against the host's evaluation first.  torch's matrix-vector product
    # of the 22.6M x 3 position array is evaluated too and its deviation printed:
    # it returned wrong values on the test machine once, so it is not used.
    v3 = np.array([0.3, -1.1, 2.0])
    lin_h = info["xyz"] @ v3 + 0.5
    xyz_t = torch.tensor(info["xyz"], device="cuda")
    v3_t = torch.tensor(v3, device="cuda")
    lin = (xyz_t[:, 0] * v3_t[0] + xyz_t[:, 1] * v3_t[1]) + (xyz_t[:, 2] * v3_t[2] + 0.5)
    lin_mm = xyz_t @ v3_t + 0.5
    dev_ew = np.abs(lin.cpu().numpy() - lin_h).max()
    dev_mm = np.abs(lin_mm.cpu().numpy() - lin_h).max()
    print("linear field: device elementwise vs host %.3e, torch matvec vs host %.3e" % (dev_ew, dev_mm))
    del lin_mm, xyz_t
    assert dev_ew <= 1e-14
    y = opn.apply(lin)
    interior = torch.tensor(~info["boundary"], device="cuda")
    assert y[interior].abs().max().item() <= 1e-12 * scale
    s = torch.rand(opn.n_local, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(1))
    a, b = (s * opd.apply(r)).sum().item(), (r * opd.apply(s)).sum().item()
    assert abs(a - b) <= 1e-12 * abs(a)
    assert opd.apply(ones)[~interior].abs().max().item() == 0.0


def test_batched_refined_solve_32_instances():
    print("C5 batched solve", flush=True)
    levels = W.fields.batch_levels()
    a, phi = W.fields.batch_k_params()
    v, t = W.meshes.ref_tet()
    meshes = [T.Mesh(v, t, int(l)) for l in levels]
    infos = [mm.dof_info(2, owner=False) for mm in meshes]
    b64 = T.Batch([T.Operator(mm, T.P2_DIVKGRAD, T.F64) for mm in meshes])
    b32 = T.Batch([T.Operator(mm, T.P2_DIVKGRAD, T.F32) for mm in meshes])
    K = b64.concat([torch.tensor(W.fields.batch_k(inf["xyz"], a[i], phi[i]), device="cuda")
                    for i, inf in enumerate(infos)])
    Xs = b64.concat([torch.tensor(W.uniform_from_keys(11, inf["keys"]) * (~inf["boundary"]), device="cuda")
                     for inf in infos])
    B = b64.apply(Xs, K)
    X = torch.zeros_like(B)
    stats, relres = T.IRSolver(b64, b32, tol=1e-10).solve(B, X, K, K.float())
    print("C5 stats", stats, "max relres", relres.max())
    assert stats["converged"] and relres.max() <= 1e-10
    Bn, Xn, Xsn = B.cpu().numpy(), X.cpu().numpy(), Xs.cpu().numpy()
    worst_res, worst_err = 0.0, 0.0
    for i, lvl in enumerate(levels):
        s0, s1 = b64.offsets[i], b64.offsets[i + 1]
        pr = O.Problem(v, t, int(lvl), O.P2_DIVKGRAD, O.BC_DIRICHLET_ZERO)
        r = Bn[s0:s1] - pr.apply(Xn[s0:s1], W.fields.batch_k(pr.xyz, a[i], phi[i]))
        worst_res = max(worst_res, np.linalg.norm(r) / np.linalg.norm(Bn[s0:s1]))
        worst_err = max(worst_err, np.linalg.norm(Xn[s0:s1] - Xsn[s0:s1]) / np.linalg.norm(Xsn[s0:s1]))
    print("C5 oracle-evaluated max relres", worst_res, "max |x - x*|/|x*|", worst_err)
    assert worst_res <= 1.01e-10
