"""Gauss (Gauss-Legendre) volume points through the C ABI against the oracle's
Gauss operator (pinned in test_oracle_gauss.py): FP64 within 1e-12 and FP32
within 1e-5 (relative 2-norm), both bases; affine meshes give the GLL
operator; the operator is symmetric; switching back restores the GLL apply
bit for bit; CG and GMRES solve the oracle's Gauss system; the calls that
assume GLL points refuse."""

from __future__ import annotations

import numpy as np
import pytest

import synth
from tests.parity import rel, rel2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2504_03573_amd as P
    return P


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle




def _affine(N, orders, seed, deform=0.0, rotate=False, lam=2.0):
    m = synth.affine_mesh(3, N, seed=seed, order=1, lam=lam, deform_frac=deform)
    m.order = np.random.default_rng(seed + 7).integers(orders[0], orders[1] + 1, size=m.n_elems).astype(np.int32)
    return synth.rotate_elements(m, seed + 11) if rotate else m


CASES = {
    "random_p1to4_n3_rot": lambda: synth.small_mesh(3, 3, ("random", 1, 4), seed=5, rotate=True, lam=1.5),
    "w3_p3to6_n4": lambda: synth.workload(3, N=4),
    "random_p7to8_n2_rot": lambda: synth.small_mesh(3, 2, ("random", 7, 8), seed=9, rotate=True, lam=0.5),
    "partly_affine_p2to5_n4": lambda: _affine(4, (2, 5), 62, deform=0.35),
    "mostly_affine_p3to5_n4_rot": lambda: _affine(4, (3, 5), 68, deform=0.05, rotate=True),
    "single_elem_p3": lambda: synth.small_mesh(3, 1, 3, seed=1, lam=2.0),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request, P):
    print(f"[gauss case {request.param}]", flush=True)
    mesh = CASES[request.param]()
    op = P.SipdgOperator(mesh)
    return request.param, mesh, op


@pytest.mark.parametrize("basis", ["legendre", "modal"])
def test_apply_parity(case, orc, basis):
    name, mesh, op = case
    om = orc.prepare(mesh, basis, points="gl")
    x = synth.random_coefficients(mesh, 7101)
    y_ref = om.apply(x)
    op.basis = basis
    op.points = "gauss"
    try:
        assert op.points == "gauss" and op.variant == "gather_fold"
        xt = torch.tensor(x, device="cuda")
        y = op.apply(xt).cpu().numpy()
        y32 = op.apply(xt.float()).double().cpu().numpy()
        print(f"{name} {basis}: gauss fp64 {rel(y, y_ref):.2e} fp32 {rel(y32, y_ref):.2e}")
        assert rel(y, y_ref) <= 1e-12
        assert rel(y32, y_ref) <= 1e-5
        assert torch.equal(op.apply(xt), op.apply(xt))
    finally:
        op.points = "gll"
        op.basis = "legendre"


def test_switch_back_bitwise(P):
    m = synth.small_mesh(3, 3, ("random", 2, 5), seed=71, rotate=True, lam=1.0)
    op = P.SipdgOperator(m)
    x = torch.tensor(synth.random_coefficients(m, 7102), device="cuda")
    y0 = op.apply(x)
    op.points = "gauss"
    yg = op.apply(x)
    op.points = "gll"
    assert torch.equal(op.apply(x), y0)
    assert float((yg - y0).norm() / y0.norm()) >= 1e-9   # deformed: a different operator


def test_symmetric_and_transpose(P):
    """The Gauss operator stays symmetric (both quadratures are applied to the
    symmetric form), so the transpose apply is the apply."""
    m = synth.small_mesh(3, 3, ("random", 1, 5), seed=80, rotate=True, lam=0.8)
    op = P.SipdgOperator(m)
    op.points = "gauss"
    rng = np.random.default_rng(81)
    x = torch.tensor(rng.standard_normal(op.n_dofs), device="cuda")
    z = torch.tensor(rng.standard_normal(op.n_dofs), device="cuda")
    a, b = float(torch.dot(z, op.apply(x))), float(torch.dot(x, op.apply(z)))
    assert abs(a - b) <= 1e-12 * (abs(a) + abs(b))
    assert torch.equal(op.apply_transpose(x), op.apply(x))
    # stage by stage equals the whole application
    y = torch.empty_like(x)
    op.apply_stage(x, 1, out=y)
    op.apply_stage(x, 2, out=y)
    assert torch.equal(y, op.apply(x))


def test_lambda_and_penalty_changes(P, orc):
    """set_lambda and set_penalty_scale act on the Gauss apply as on the GLL one."""
    m = synth.small_mesh(3, 3, ("random", 2, 4), seed=82, rotate=True, lam=1.0)
    op = P.SipdgOperator(m)
    op.points = "gauss"
    lam = np.random.default_rng(83).uniform(0.0, 5.0, m.n_elems)
    op.set_lambda(torch.tensor(lam, device="cuda"))
    op.set_penalty_scale(2.5)
    m.lam = lam.copy()
    m.sigma = 2.5
    om = orc.prepare(m, points="gl")
    x = synth.random_coefficients(m, 7106)
    y = op.apply(torch.tensor(x, device="cuda")).cpu().numpy()
    assert rel(y, om.apply(x)) <= 1e-12


def test_affine_equals_gll(P):
    """Both point sets integrate an affine element's terms exactly."""
    m = _affine(3, (1, 6), 72, rotate=True)
    op = P.SipdgOperator(m)
    x = torch.tensor(synth.random_coefficients(m, 7103), device="cuda")
    y0 = op.apply(x)
    op.points = "gauss"
    y1 = op.apply(x)
    assert float((y1 - y0).norm() / y0.norm()) <= 1e-13


def test_solvers(P, orc):
    m = synth.small_mesh(3, 3, ("random", 2, 5), seed=73, rotate=True, lam=1.0)
    om = orc.prepare(m, points="gl")
    x_true = synth.random_coefficients(m, 7104)
    b = om.apply(x_true)
    op = P.SipdgOperator(m)
    bt = torch.tensor(b, device="cuda")
    xs_gll, _ = op.cg_solve(bt, tol=1e-10)
    op.points = "gauss"
    for mode in ("f64", "f32_ir"):
        xs, info = op.cg_solve(bt, tol=1e-10, mode=mode)
        xs = xs.cpu().numpy()
        print(f"cg {mode}: {info}")
        assert info["converged"]
        assert np.linalg.norm(b - om.apply(xs)) <= 1e-9 * np.linalg.norm(b)
        assert rel2(xs, x_true) <= 1e-6
    # the graph cache follows the point set: a GLL solve after the Gauss ones
    op.points = "gll"
    xs2, _ = op.cg_solve(bt, tol=1e-10)
    assert torch.equal(xs2, xs_gll)
    op.points = "gauss"
    xg, info = op.gmres_solve(bt, tol=1e-10, restart=30)
    assert info["converged"]
    assert rel2(xg.cpu().numpy(), x_true) <= 1e-6


def test_refusals(P):
    m = synth.small_mesh(3, 2, ("random", 2, 4), seed=74, lam=1.0)
    op = P.SipdgOperator(m)
    x = torch.tensor(synth.random_coefficients(m, 7105), device="cuda")
    op.points = "gauss"
    for call in (op.diagonal, lambda: op.param_grad(x, x), op.autotune,
                 lambda: setattr(op, "variant", "gather"), lambda: setattr(op, "flux", "p2p")):
        with pytest.raises(P.SipdgError):
            call()
    assert op.points == "gauss" and op.variant == "gather_fold" and op.flux == "shared"
    op.points = "gll"
    op.flux = "p2p"
    with pytest.raises(P.SipdgError):
        op.points = "gauss"
    op.flux = "shared"
    with pytest.raises(P.SipdgError):
        P.SipdgOperator(synth.small_mesh(2, 3, 2, seed=75)).points = "gauss"
    # an order-6 element next to an order-8 one: that group runs on the general kernels
    m2 = synth.small_mesh(3, 2, 6, seed=76, lam=1.0)
    m2.order[0] = 8
    with pytest.raises(P.SipdgError):
        P.SipdgOperator(m2).points = "gauss"


def test_batch_equals_singles(P):
    ms = [synth.small_mesh(3, 2, ("random", 2, 5), seed=77, rotate=True, lam=1.0),
          _affine(3, (1, 4), 78, deform=0.3)]
    bop = P.SipdgOperator.batch(ms)
    singles = [P.SipdgOperator(m) for m in ms]
    off = bop.problem_dof_offsets
    x = torch.tensor(np.random.default_rng(79).standard_normal(bop.n_dofs), device="cuda")
    bop.points = "gauss"
    y = bop.apply(x)
    for i, op in enumerate(singles):
        op.points = "gauss"
        yi = op.apply(x[off[i]:off[i + 1]].contiguous())
        assert float((y[off[i]:off[i + 1]] - yi).norm() / yi.norm()) <= 1e-14, i


def test_autograd_wrt_inputs(P):
    """Under Gauss points the autograd Functions differentiate with respect to
    x and b (transpose apply, adjoint CG); lambda and sigma need the GLL
    parameter-gradient kernels."""
    from paper_2504_03573_amd import autograd as AG
    m = synth.small_mesh(3, 3, ("random", 2, 4), seed=84, rotate=True, lam=1.0)
    op = P.SipdgOperator(m)
    op.points = "gauss"
    rng = np.random.default_rng(85)
    lam = torch.tensor(m.lam, device="cuda")
    w = torch.tensor(rng.standard_normal(op.n_dofs), device="cuda")
    x = torch.tensor(rng.standard_normal(op.n_dofs), device="cuda", requires_grad=True)
    (w * AG.apply(op, x, lam, 1.0)).sum().backward()
    assert torch.equal(x.grad, op.apply(w))
    b = torch.tensor(rng.standard_normal(op.n_dofs), device="cuda", requires_grad=True)
    (w * AG.solve(op, b, lam, 1.0)).sum().backward()
    # db = A^{-1} w: A db = w
    r = op.apply(b.grad) - w
    assert float(r.norm() / w.norm()) <= 1e-9

