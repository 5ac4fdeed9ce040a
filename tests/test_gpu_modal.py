"""Modified C0 modal basis (Table 1 "Modal") through the C ABI against the
oracle's modal operator (pinned by the change of basis in
test_oracle_modal.py): apply FP64 within 1e-12 and FP32 within 1e-5, the
Jacobi diagonal, CG, and the point-to-point flux; switching back restores
the Legendre operator and the default kernel structure."""

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


CASES = {
    "2d_random_p1to8_rot": lambda: synth.small_mesh(2, 5, ("random", 1, 8), seed=3, rotate=True, lam=2.0),
    "3d_random_p1to4_rot": lambda: synth.small_mesh(3, 3, ("random", 1, 4), seed=5, rotate=True, lam=1.5),
    "w3_p3to6_n4": lambda: synth.workload(3, N=4),
    "3d_p5to8_n2_rot": lambda: synth.small_mesh(3, 2, ("random", 5, 8), seed=9, rotate=True, lam=0.5),
}




@pytest.fixture(scope="module", params=list(CASES))
def case(request, P, orc):
    print(f"[modal case {request.param}]", flush=True)
    mesh = CASES[request.param]()
    op = P.SipdgOperator(mesh)
    op.basis = "modal"
    return request.param, mesh, op, orc.prepare(mesh, "modal")


def test_apply_and_diagonal(case, P):
    name, mesh, op, om = case
    assert op.basis == "modal" and op.variant == "gather_fold"
    x = synth.random_coefficients(mesh, 7101)
    y_ref = om.apply(x)
    xt = torch.tensor(x, device="cuda")
    y = op.apply(xt).cpu().numpy()
    y32 = op.apply(xt.float()).double().cpu().numpy()
    print(f"{name}: modal fp64 {rel(y, y_ref):.2e} fp32 {rel(y32, y_ref):.2e}")
    assert rel(y, y_ref) <= 1e-12 and rel(y32, y_ref) <= 1e-5
    assert rel(op.diagonal().cpu().numpy(), om.diagonal()) <= 1e-12
    if mesh.dim == 3:
        # the general kernels agree; the structures with Legendre endpoint
        # values in closed form refuse the modal basis
        op.variant = "gather"
        try:
            yg = op.apply(xt).cpu().numpy()
            assert rel(yg, y_ref) <= 1e-12 and rel(yg, y) <= 1e-13
        finally:
            op.variant = "gather_fold"
        for v in ("gather_fold_persistent", "gather_fold_fused", "two_stage", "fused"):
            with pytest.raises(P.SipdgError):
                op.variant = v
        assert op.variant == "gather_fold"


def test_cg(case):
    name, mesh, op, om = case
    x_true = synth.random_coefficients(mesh, 7102)
    b = om.apply(x_true)
    xs, info = op.cg_solve(torch.tensor(b, device="cuda"), tol=1e-10)
    assert info["converged"] and info["rel_resid"] <= 1e-10
    # the GPU solution solves the oracle's system too
    xg = xs.cpu().numpy()
    assert np.linalg.norm(b - om.apply(xg)) <= 1e-8 * np.linalg.norm(b)
    if op.n_dofs <= 5000:
        # the modal basis is far worse conditioned than the orthogonal one
        # (hundreds to thousands of iterations here), so finite-precision CG
        # drifts by a few per cent with the summation order and restarts
        _, it_o, _ = om.cg(b, tol=1e-10)
        assert abs(info["iters"] - it_o) <= max(2, 0.05 * it_o), (info["iters"], it_o)


def test_point_to_point(case):
    name, mesh, op, om = case
    if mesh.dim != 3:
        pytest.skip("the point-to-point flux is 3-D")
    x = synth.random_coefficients(mesh, 7103)
    op.flux = "p2p"
    try:
        y = op.apply(torch.tensor(x, device="cuda")).cpu().numpy()
    finally:
        op.flux = "shared"
    assert rel(y, om.apply_p2p(x)) <= 1e-12


def test_switch_back_to_legendre(P, orc):
    m = synth.small_mesh(3, 2, ("random", 2, 5), seed=21, rotate=True, lam=0.8)
    op = P.SipdgOperator(m)
    default = op.variant
    x = torch.tensor(synth.random_coefficients(m, 7104), device="cuda")
    y0 = op.apply(x)
    d0 = op.diagonal()
    # captured CG iterations before and after a switch: the graphs are
    # captured again for the other basis (same kernel structure)
    xs0, _ = op.cg_solve(y0, tol=1e-10, graph_k=5)
    op.basis = "modal"
    om = orc.prepare(m, "modal")
    b = om.apply(synth.random_coefficients(m, 7105))
    xs1, info = op.cg_solve(torch.tensor(b, device="cuda"), tol=1e-10, graph_k=5)
    assert info["converged"]
    assert np.linalg.norm(b - om.apply(xs1.cpu().numpy())) <= 1e-8 * np.linalg.norm(b)
    op.basis = "legendre"
    assert op.variant == default
    assert torch.equal(op.apply(x), y0)
    assert torch.equal(op.diagonal(), d0)
    xs2, _ = op.cg_solve(y0, tol=1e-10, graph_k=5)
    assert torch.equal(xs2, xs0)
