"""Parity of the HIP path (through the C ABI) with the oracle.

Tolerances: FP64 relative 2-norm error <= 1e-12, FP32 <= 1e-5 (the
operator's stated bar); integer/topology outputs exact."""

from __future__ import annotations

import math

import numpy as np
import pytest

import synth
from tests.parity import rel, rel2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2504_03573_amd as P
    return P


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


def P_error():
    import paper_2504_03573_amd as P
    return P.SipdgError




CASES = {
    "w1_2d_4x4_p3": lambda: synth.workload(1),
    "2d_checker45_6x6": lambda: synth.small_mesh(2, 6, ("checker", 4, 5), seed=1002),
    "2d_random_p1to8_rot": lambda: synth.small_mesh(2, 5, ("random", 1, 8), seed=3, rotate=True, lam=2.0),
    "3d_random_p1to4_rot": lambda: synth.small_mesh(3, 3, ("random", 1, 4), seed=5, rotate=True, lam=1.5),
    "3d_random_p3to6_n4": lambda: synth.workload(3, N=4),
    "3d_p5to8_n2": lambda: synth.small_mesh(3, 2, ("random", 5, 8), seed=9, rotate=True, lam=0.5),
    "3d_p7_n2_rot": lambda: synth.small_mesh(3, 2, 7, seed=13, rotate=True, lam=2.0),
    "3d_checker78_n3": lambda: synth.small_mesh(3, 3, ("checker", 7, 8), seed=17, lam=1.0),
    "3d_single_elem_p2": lambda: synth.small_mesh(3, 1, 2, seed=1, lam=3.0),
    "3d_lam0_p2to5_n2_rot": lambda: synth.small_mesh(3, 2, ("random", 2, 5), seed=21, rotate=True, lam=0.0),
    "w5_lamfield_n3": lambda: synth.workload(5, N=3),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request, lib, orc):
    print(f"[case {request.param}]", flush=True)
    mesh = CASES[request.param]()
    op = lib.SipdgOperator(mesh)
    om = orc.prepare(mesh)
    return request.param, mesh, op, om


def test_apply_f64(case):
    name, mesh, op, om = case
    x = synth.random_coefficients(mesh, 4001)
    y_ref = om.apply(x)
    y = op.apply(torch.tensor(x, device="cuda")).cpu().numpy()
    e = rel(y, y_ref)
    print(f"{name}: fp64 rel err {e:.2e}")
    assert e <= 1e-12


def test_apply_f32(case):
    name, mesh, op, om = case
    x = synth.random_coefficients(mesh, 4002)
    y_ref = om.apply(x)
    y = op.apply(torch.tensor(x, device="cuda", dtype=torch.float32)).double().cpu().numpy()
    e = rel(y, y_ref)
    print(f"{name}: fp32 rel err {e:.2e}")
    assert e <= 1e-5


def test_transpose_symmetry_determinism(case):
    name, mesh, op, om = case
    rng = np.random.default_rng(7)
    x = torch.tensor(rng.standard_normal(op.n_dofs), device="cuda")
    z = torch.tensor(rng.standard_normal(op.n_dofs), device="cuda")
    y1 = op.apply(x)
    y2 = op.apply(x)
    assert torch.equal(y1, y2), "two applies differ bitwise"
    yt = op.apply_transpose(x)
    assert torch.equal(yt, y1)
    a = float(torch.dot(z, op.apply(x)))
    b = float(torch.dot(x, op.apply(z)))
    assert abs(a - b) <= 1e-12 * (abs(a) + abs(b) + 1e-300) * 10


def test_diagonal(case):
    name, mesh, op, om = case
    d = op.diagonal().cpu().numpy()
    assert rel(d, om.diagonal()) <= 1e-12


def test_points_and_load_vector(case):
    name, mesh, op, om = case
    xq, xb = op.quad_points()
    oq, ob = om.points()
    assert np.abs(xq.cpu().numpy() - oq).max() <= 1e-14
    assert np.abs(xb.cpu().numpy() - ob).max() <= 1e-14
    src = lambda X: np.sin(3 * X[:, 0]) + X[:, 1] ** 2 + 0.5
    gd = lambda X: np.cos(2 * X[:, 0]) - X[:, 1]
    b_ref = om.rhs(src(oq), gd(ob))
    s = torch.tensor(src(xq.cpu().numpy()), device="cuda")
    g = torch.tensor(gd(xb.cpu().numpy()) if len(ob) else np.zeros(1), device="cuda")
    b = op.load_vector(s, g).cpu().numpy()
    assert rel(b, b_ref) <= 1e-12


def test_param_grad(case):
    name, mesh, op, om = case
    rng = np.random.default_rng(11)
    a = rng.standard_normal(op.n_dofs)
    b = rng.standard_normal(op.n_dofs)
    dl_ref, ds_ref = om.param_grad(a, b)
    dl, ds = op.param_grad(torch.tensor(a, device="cuda"), torch.tensor(b, device="cuda"))
    assert rel(dl.cpu().numpy(), dl_ref) <= 1e-12
    assert abs(float(ds[0]) - ds_ref) <= 1e-12 * abs(ds_ref)


def test_cg_f64_matches_oracle(case):
    name, mesh, op, om = case
    if op.n_dofs > 5000:
        pytest.skip("oracle CG too slow for this case")
    x_true = synth.random_coefficients(mesh, 4003)
    b = om.apply(x_true)
    xo, it_o, rel_o = om.cg(b, tol=1e-10)
    xs, info = op.cg_solve(torch.tensor(b, device="cuda"), tol=1e-10)
    assert info["converged"] and info["rel_resid"] <= 1e-10
    assert abs(info["iters"] - it_o) <= 2, (info["iters"], it_o)
    assert rel2(xs.cpu().numpy(), x_true) <= 1e-6


def test_cg_f32_ir(case):
    name, mesh, op, om = case
    x_true = synth.random_coefficients(mesh, 4004)
    b = op.apply(torch.tensor(x_true, device="cuda"))
    for mode in ("f32_ir", "f32_ru"):
        xs, info = op.cg_solve(b, tol=1e-10, mode=mode)
        print(f"{name}: {mode} {info}")
        assert info["converged"] and info["rel_resid"] <= 1e-10, mode
    xg, info_g = op.cg_solve(b, tol=1e-10, graph_k=0)
    xh, info_h = op.cg_solve(b, tol=1e-10, graph_k=7)
    # captured iterations replay the stream's kernels in the same order:
    # the same iterates, bit for bit
    assert info_g["iters"] == info_h["iters"], (info_g, info_h)
    assert torch.equal(xg, xh)


def test_geometry_map(case):
    """Geometric factors derived at every point from the element's trilinear
    map give the operator of the stored per-point factors (Sec. 5.1: data
    traded for arithmetic), FP64 and FP32, and CG with captured iterations."""
    name, mesh, op, om = case
    if mesh.dim != 3:
        with pytest.raises(P_error()):
            op.geometry = "map"
        return
    x = synth.random_coefficients(mesh, 4006)
    y_ref = om.apply(x)
    xt = torch.tensor(x, device="cuda")
    keep = op.variant
    op.variant = "gather_fold"
    try:
        y_st = op.apply(xt).cpu().numpy()
        op.geometry = "map"
        assert op.geometry == "map"
        y = op.apply(xt).cpu().numpy()
        y32 = op.apply(xt.float()).double().cpu().numpy()
        print(f"{name}: map fp64 {rel(y, y_ref):.2e} fp32 {rel(y32, y_ref):.2e}")
        assert rel(y, y_ref) <= 1e-12 and rel(y32, y_ref) <= 1e-5
        assert rel(y, y_st) <= 1e-13
        xs, info = op.cg_solve(torch.tensor(y_ref, device="cuda"), tol=1e-10, graph_k=5)
        assert info["converged"] and rel2(xs.cpu().numpy(), x) <= 1e-6
    finally:
        op.geometry = "stored"
        op.variant = keep


def test_variants_agree(case):
    """Gather-and-interpolate and direct trace evaluation give the same
    operator (Sec. 3.2: equivalent when the trace order is at least the
    element's); the fused, two-stage and gather-fold launch structures are
    identical up to rounding."""
    name, mesh, op, om = case
    x = synth.random_coefficients(mesh, 4005)
    y_ref = om.apply(x)
    xt = torch.tensor(x, device="cuda")
    ys = {}
    keep = op.variant
    if mesh.dim == 2:
        # the general kernels, the wavefront kernels (trace launch + apply
        # launch) and, when every element fits the 8-point lane grid, the fused
        # wavefront launch (neighbour traces from their coefficients)
        small = int(mesh.order.max()) <= 6
        try:
            for v in ("gather", "gather_fold") + (("gather_fold_fused",) if small else ()):
                op.variant = v
                ys[v] = op.apply(xt).cpu().numpy()
                assert rel(ys[v], y_ref) <= 1e-12, v
                y32 = op.apply(xt.float()).double().cpu().numpy()
                assert rel(y32, y_ref) <= 1e-5, v
            assert rel(ys["gather_fold"], ys["gather"]) <= 1e-13
            if small:
                assert rel(ys["gather_fold_fused"], ys["gather_fold"]) <= 1e-14
            else:
                with pytest.raises(P_error()):
                    op.variant = "gather_fold_fused"
            with pytest.raises(P_error()):
                op.variant = "two_stage"
        finally:
            op.variant = keep
        return
    if int(mesh.order.max()) > 6:
        # orders 7-8 present: only the structures that support them
        try:
            for v in ("gather", "gather_fold", "gather_fold_persistent"):
                op.variant = v
                ys[v] = op.apply(xt).cpu().numpy()
                assert rel(ys[v], y_ref) <= 1e-12, v
            assert rel(ys["gather_fold"], ys["gather"]) <= 1e-13
            assert rel(ys["gather_fold_persistent"], ys["gather_fold"]) <= 1e-14
            with pytest.raises(P_error()):
                op.variant = "two_stage"
        finally:
            op.variant = keep
        return
    try:
        for v in ("gather", "two_stage", "fused", "gather_fold", "gather_fold_fused", "gather_fold_persistent"):
            op.variant = v
            ys[v] = op.apply(xt).cpu().numpy()
            assert rel(ys[v], y_ref) <= 1e-12, v
            y32 = op.apply(xt.float()).double().cpu().numpy()
            assert rel(y32, y_ref) <= 1e-5, v
        assert rel(ys["fused"], ys["gather"]) <= 1e-13
        assert rel(ys["two_stage"], ys["fused"]) <= 1e-14
        assert rel(ys["gather_fold"], ys["gather"]) <= 1e-13
        assert rel(ys["gather_fold_fused"], ys["gather_fold"]) <= 1e-14
        assert rel(ys["gather_fold_persistent"], ys["gather_fold"]) <= 1e-14
    finally:
        op.variant = keep
