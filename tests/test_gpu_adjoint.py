"""GPU reverse mode of the div(k grad) and epsilon operators (hand-written adjoint kernels).

Epsilon (at the end): dL/dx and dL/dmu on the affine shell (level 2) and the
radially blended shell (level 1, 14-point rule) against the oracle, FP64
1e-12; FP32 against FP64.

P2 div(k grad) (the same checks, below the P1 ones): reference tet at level 5
and the 6-macro Kuhn cube at level 3 against the oracle's gradients; 16
central-difference directions each for x and k; FP32 against FP64; and
d/dk (w . A(k) x) . dk = w . (A(k + dk) x - A(k) x) on the cube (A linear in k).

P1 div(k grad):

Workload: one macro tet (the reference tetrahedron) at level 7 (366,145
DoFs), k = 1 + 0.9 U[-1,1) per node, x and b ~ U[-1,1), Dirichlet rows and
columns, loss L = 0.5 |A(k) x - b|^2.

* dL/dx and dL/dk against the oracle's gradients (FP64, relative 1e-12);
* 64 random unit directions each for x and k against central differences
  with h = 1e-6.  L is exactly quadratic in x and, A being linear in k, in k,
  so central differences have no truncation error: the difference to the
  analytic directional derivative is rounding, ~ eps |L| / h.  Bound:
  1e-6 relative to max(|dL.d|, 1e-3 |L|).
"""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2404_08371_amd as T
from paper_2404_08371_amd.autograd import TmfApply
import workloads as W

pytestmark = pytest.mark.gpu


def setup(level, mesh="ref"):
    v, t = W.meshes.ref_tet() if mesh == "ref" else W.meshes.kuhn_cube()
    m = T.Mesh(v, t, level)
    op = T.Operator(m, T.P1_DIVKGRAD, T.F64, T.BC_DIRICHLET_ZERO)
    info = m.dof_info(1)
    keys = info["keys"]
    k = W.fields.perturbed_k(keys, 5)
    x = W.uniform_from_keys(6, keys)
    b = W.uniform_from_keys(7, keys)
    return m, op, info, k, x, b


def loss_and_grads(op, k, x, b, owner):
    kt = torch.tensor(k, device="cuda", requires_grad=True)
    xt = torch.tensor(x, device="cuda", requires_grad=True)
    bt = torch.tensor(b, device="cuda")
    own = torch.tensor(owner, device="cuda", dtype=torch.float64)
    y = TmfApply.apply(xt, kt, op)
    L = 0.5 * (((y - bt) ** 2) * own).sum()
    L.backward()
    return L.item(), xt.grad.cpu().numpy(), kt.grad.cpu().numpy()


@pytest.mark.parametrize("level,mesh", [(7, "ref"), (3, "cube")])
def test_gradients_match_oracle(level, mesh):
    print("adjoint oracle case", level, mesh, flush=True)
    m, op, info, k, x, b = setup(level, mesh)
    L, gx, gk = loss_and_grads(op, k, x, b, info["owner"])
    v, t = W.meshes.ref_tet() if mesh == "ref" else W.meshes.kuhn_cube()
    pr = O.Problem(v, t, level, O.P1_DIVKGRAD, O.BC_DIRICHLET_ZERO)
    ko, xo, bo = (W.fields.perturbed_k(pr.keys, 5), W.uniform_from_keys(6, pr.keys),
                  W.uniform_from_keys(7, pr.keys))
    Lo, gxo, gko = pr.loss_gradients(ko, xo, bo)
    assert abs(L - Lo) <= 1e-12 * abs(Lo)
    # the torch loss counts each DoF once through the owner mask, so gradients of
    # duplicated DoFs are split over copies: compare the per-DoF totals
    own = info["owner"]
    for g, go in ((gx, gxo), (gk, gko)):
        tot = np.zeros(pr.n_unique)
        np.add.at(tot, pr.uid, g)
        assert np.linalg.norm(tot - pr.to_unique(go)) <= 1e-12 * np.linalg.norm(go), mesh


def test_central_differences_64_directions():
    print("adjoint FD case", flush=True)
    m, op, info, k, x, b = setup(7)
    L, gx, gk = loss_and_grads(op, k, x, b, info["owner"])
    kt, xt, bt = (torch.tensor(a, device="cuda") for a in (k, x, b))

    def loss(xv, kv):
        y = op.apply(xv, kv)
        return 0.5 * float(((y - bt) ** 2).sum())

    rng = np.random.default_rng(8)
    h = 1e-6
    worst = 0.0
    for which in ("x", "k"):
        for _ in range(64):
            d = rng.uniform(-1, 1, x.size)
            d /= np.linalg.norm(d)
            dt = torch.tensor(d, device="cuda")
            if which == "x":
                fd = (loss(xt + h * dt, kt) - loss(xt - h * dt, kt)) / (2 * h)
                an = float(gx @ d)
            else:
                fd = (loss(xt, kt + h * dt) - loss(xt, kt - h * dt)) / (2 * h)
                an = float(gk @ d)
            err = abs(fd - an) / max(abs(an), 1e-3 * L)
            worst = max(worst, err)
            assert err <= 1e-6, (which, fd, an)
    print("worst relative FD mismatch", worst)


def test_adjoint_fp32_matches_fp64():
    m, op, info, k, x, b = setup(5)
    op32 = T.Operator(m, T.P1_DIVKGRAD, T.F32, T.BC_DIRICHLET_ZERO)
    gy = torch.tensor(b, device="cuda")
    gx64, gk64 = op.adjoint(torch.tensor(k, device="cuda"), torch.tensor(x, device="cuda"), gy)
    gx32, gk32 = op32.adjoint(torch.tensor(k, device="cuda", dtype=torch.float32),
                              torch.tensor(x, device="cuda", dtype=torch.float32), gy.float())
    for a64, a32 in ((gx64, gx32), (gk64, gk32)):
        a64, a32 = a64.cpu().numpy(), a32.double().cpu().numpy()
        assert np.abs(a64 - a32).max() <= 1e-5 * np.abs(a64).max()


def test_backward_is_the_transpose_of_the_forward_map():
    """<grad_x (w . y), d> = w . A d for any (also inconsistent) direction d on a 6-macro mesh."""
    v, t = W.meshes.kuhn_cube()
    m = T.Mesh(v, t, 2)
    for kind in (T.P2_DIVKGRAD, T.P2_LAPLACE):
        op = T.Operator(m, kind, T.F64)
        info = m.dof_info(2)
        k = torch.tensor(W.fields.cube_k(info["xyz"]), device="cuda") if op.has_coeff else None
        x = torch.tensor(W.uniform_from_keys(1, info["keys"]), device="cuda", requires_grad=True)
        w = torch.tensor(W.uniform_from_keys(2, info["keys"]), device="cuda")
        (TmfApply.apply(x, k, op) * w).sum().backward()
        d = torch.tensor(np.random.default_rng(3).uniform(-1, 1, op.n_local), device="cuda")
        lhs = (x.grad * d).sum().item()
        rhs = (w * op.apply(d, k)).sum().item()
        assert abs(lhs - rhs) <= 1e-12 * abs(rhs)
    op = T.Operator(T.Mesh(v, t, 3), T.P1_DIVKGRAD, T.F64)
    info = op.mesh.dof_info(1)
    k = torch.tensor(W.fields.perturbed_k(info["keys"], 5), device="cuda", requires_grad=True)
    x = torch.tensor(W.uniform_from_keys(1, info["keys"]), device="cuda", requires_grad=True)
    w = torch.tensor(W.uniform_from_keys(2, info["keys"]), device="cuda")
    (TmfApply.apply(x, k, op) * w).sum().backward()
    rng = np.random.default_rng(4)
    dx = torch.tensor(rng.uniform(-1, 1, op.n_local), device="cuda")
    dk = torch.tensor(rng.uniform(-1, 1, op.n_local), device="cuda")
    assert abs((x.grad * dx).sum().item() - (w * op.apply(dx, k)).sum().item()) <= 1e-12 * (w.abs().sum().item())
    # A is linear in k: d/dk (w . A(k) x) . dk = w . (A(k + dk) x - A(k) x)
    lin = (w * (op.apply(x.detach(), k.detach() + dk) - op.apply(x.detach(), k.detach()))).sum().item()
    assert abs((k.grad * dk).sum().item() - lin) <= 1e-11 * max(abs(lin), 1.0)


# ------------------------------------------------------------------ P2
def setup_p2(level, mesh="ref", prec=T.F64):
    v, t = W.meshes.ref_tet() if mesh == "ref" else W.meshes.kuhn_cube()
    m = T.Mesh(v, t, level)
    op = T.Operator(m, T.P2_DIVKGRAD, prec, T.BC_DIRICHLET_ZERO)
    info = m.dof_info(2)
    keys = info["keys"]
    return m, op, info, W.fields.perturbed_k(keys, 5), W.uniform_from_keys(6, keys), W.uniform_from_keys(7, keys)


@pytest.mark.parametrize("level,mesh", [(5, "ref"), (3, "cube")])
def test_p2_gradients_match_oracle(level, mesh):
    print("p2 adjoint oracle case", level, mesh, flush=True)
    m, op, info, k, x, b = setup_p2(level, mesh)
    L, gx, gk = loss_and_grads(op, k, x, b, info["owner"])
    v, t = W.meshes.ref_tet() if mesh == "ref" else W.meshes.kuhn_cube()
    pr = O.Problem(v, t, level, O.P2_DIVKGRAD, O.BC_DIRICHLET_ZERO)
    ko, xo, bo = (W.fields.perturbed_k(pr.keys, 5), W.uniform_from_keys(6, pr.keys),
                  W.uniform_from_keys(7, pr.keys))
    Lo, gxo, gko = pr.loss_gradients(ko, xo, bo)
    assert abs(L - Lo) <= 1e-12 * abs(Lo)
    for g, go in ((gx, gxo), (gk, gko)):
        tot = np.zeros(pr.n_unique)
        np.add.at(tot, pr.uid, g)
        assert np.linalg.norm(tot - pr.to_unique(go)) <= 1e-12 * np.linalg.norm(go), mesh


def test_p2_central_differences():
    print("p2 adjoint FD case", flush=True)
    m, op, info, k, x, b = setup_p2(5)
    L, gx, gk = loss_and_grads(op, k, x, b, info["owner"])
    kt, xt, bt = (torch.tensor(a, device="cuda") for a in (k, x, b))

    def loss(xv, kv):
        y = op.apply(xv, kv)
        return 0.5 * float(((y - bt) ** 2).sum())

    rng = np.random.default_rng(9)
    h = 1e-6
    for which in ("x", "k"):
        for _ in range(16):
            d = rng.uniform(-1, 1, x.size)
            d /= np.linalg.norm(d)
            dt = torch.tensor(d, device="cuda")
            if which == "x":
                fd = (loss(xt + h * dt, kt) - loss(xt - h * dt, kt)) / (2 * h)
                an = float(gx @ d)
            else:
                fd = (loss(xt, kt + h * dt) - loss(xt, kt - h * dt)) / (2 * h)
                an = float(gk @ d)
            assert abs(fd - an) / max(abs(an), 1e-3 * L) <= 1e-6, (which, fd, an)


def test_p2_adjoint_fp32_matches_fp64():
    m, op, info, k, x, b = setup_p2(4)
    op32 = T.Operator(m, T.P2_DIVKGRAD, T.F32, T.BC_DIRICHLET_ZERO)
    gy = torch.tensor(b, device="cuda")
    gx64, gk64 = op.adjoint(torch.tensor(k, device="cuda"), torch.tensor(x, device="cuda"), gy)
    gx32, gk32 = op32.adjoint(torch.tensor(k, device="cuda", dtype=torch.float32),
                              torch.tensor(x, device="cuda", dtype=torch.float32), gy.float())
    for a64, a32 in ((gx64, gx32), (gk64, gk32)):
        a64, a32 = a64.cpu().numpy(), a32.double().cpu().numpy()
        assert np.abs(a64 - a32).max() <= 1e-5 * np.abs(a64).max()


def test_p2_coefficient_gradient_is_the_linear_part():
    v, t = W.meshes.kuhn_cube()
    op = T.Operator(T.Mesh(v, t, 2), T.P2_DIVKGRAD, T.F64)
    info = op.mesh.dof_info(2)
    k = torch.tensor(W.fields.perturbed_k(info["keys"], 5), device="cuda", requires_grad=True)
    x = torch.tensor(W.uniform_from_keys(1, info["keys"]), device="cuda")
    w = torch.tensor(W.uniform_from_keys(2, info["keys"]), device="cuda")
    (TmfApply.apply(x, k, op) * w).sum().backward()
    dk = torch.tensor(np.random.default_rng(4).uniform(-1, 1, op.n_local), device="cuda")
    lin = (w * (op.apply(x, k.detach() + dk) - op.apply(x, k.detach()))).sum().item()
    assert abs((k.grad * dk).sum().item() - lin) <= 1e-11 * max(abs(lin), 1.0)



# ------------------------------------------------------------- epsilon
def eps_problem(mesh, level, prec=T.F64):
    from helpers import MESHES, inputs
    mk, mp = MESHES[mesh]
    v, t = mk()
    m = T.Mesh(v, t, level, mp)
    rule = W.quadrature.rule_degree5() if mp == 1 else None
    op = T.Operator(m, T.P2V_EPSILON, prec, T.BC_DIRICHLET_ZERO, rule=rule)
    info = m.dof_info(2)
    x, mu = inputs(O.P2V_EPSILON, info["keys"], info["xyz"], 6)
    b = np.concatenate([W.uniform_from_keys(7, info["keys"], stream=c) for c in range(3)])
    return m, op, info, mu, x, b


@pytest.mark.parametrize("mesh,level", [("flatshell", 2), ("shell", 1), ("flatshell", 3), ("shell", 3)])
def test_eps_gradients_match_oracle(mesh, level):
    """Affine and radially blended epsilon operator: dL/dx and dL/dmu against the oracle (FP64, 1e-12).
    At level 3 a macro spans four 4 x 4 x 4 tile boxes, so both gradients pass through the
    seam reduction of neighbouring tiles' partial sums."""
    from helpers import inputs, oracle_problem
    print("eps adjoint case", mesh, level, flush=True)
    m, op, info, mu, x, b = eps_problem(mesh, level)
    mut = torch.tensor(mu, device="cuda", requires_grad=True)
    xt = torch.tensor(x, device="cuda", requires_grad=True)
    own = torch.tensor(np.tile(info["owner"], 3), device="cuda", dtype=torch.float64)
    y = TmfApply.apply(xt, mut, op)
    L = 0.5 * (((y - torch.tensor(b, device="cuda")) ** 2) * own).sum()
    L.backward()
    pr = oracle_problem(mesh, level, O.P2V_EPSILON, O.BC_DIRICHLET_ZERO)
    xo, muo = inputs(O.P2V_EPSILON, pr.keys, pr.xyz, 6)
    bo = np.concatenate([W.uniform_from_keys(7, pr.keys, stream=c) for c in range(3)])
    Lo, gxo, gmo = pr.loss_gradients(muo, xo, bo)
    assert abs(L.item() - Lo) <= 1e-12 * abs(Lo)
    gx, gm = xt.grad.cpu().numpy(), mut.grad.cpu().numpy()
    tx = np.zeros(3 * pr.n_unique)
    for c in range(3):
        np.add.at(tx, c * pr.n_unique + pr.uid, gx[c * pr.n_local:(c + 1) * pr.n_local])
    assert np.linalg.norm(tx - pr.to_unique(gxo)) <= 1e-12 * np.linalg.norm(gxo)
    tm = np.zeros(pr.n_unique)
    np.add.at(tm, pr.uid, gm)
    gmu = np.zeros(pr.n_unique)
    gmu[pr.uid] = gmo
    assert np.linalg.norm(tm - gmu) <= 1e-12 * np.linalg.norm(gmu)


@pytest.mark.parametrize("level", [2, 3])
def test_eps_adjoint_fp32_matches_fp64(level):
    print("eps adjoint fp32 case", level, flush=True)
    m, op, info, mu, x, b = eps_problem("shell", level)
    op32 = T.Operator(m, T.P2V_EPSILON, T.F32, T.BC_DIRICHLET_ZERO, rule=W.quadrature.rule_degree5())
    gy = torch.tensor(b, device="cuda")
    gx64, gm64 = op.adjoint(torch.tensor(mu, device="cuda"), torch.tensor(x, device="cuda"), gy)
    gx32, gm32 = op32.adjoint(torch.tensor(mu, device="cuda", dtype=torch.float32),
                              torch.tensor(x, device="cuda", dtype=torch.float32), gy.float())
    for a64, a32 in ((gx64, gx32), (gm64, gm32)):
        a64, a32 = a64.cpu().numpy(), a32.double().cpu().numpy()
        assert np.abs(a64 - a32).max() <= 1e-5 * np.abs(a64).max()
