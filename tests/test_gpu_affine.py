"""Affine (regular) elements, Sec. 5.1: where an element's map is affine its
geometric factors are constant, and the default apply reads seven values per
element instead of seven per quadrature point.

Checked here, through the C ABI:
* the number of elements the library treats as affine equals a direct check
  of the corners in the test (parallelepiped: X_v = X_0 + sum_k v_k (X_{2^k} - X_0));
* parity with the oracle (FP64 <= 1e-12, FP32 <= 1e-5) on all-affine and
  partly deformed meshes, rotated faces, orders 1..8;
* agreement with the per-point path of the same mesh (detection switched off),
  and with the structures that always read per-point factors;
* order groups all affine (one launch), at least half affine (affine and
  deformed launches side by side) and less than half (per-point only)."""

from __future__ import annotations

import os

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


def _mesh(N, orders, seed, deform=0.0, rotate=False, lam=2.0):
    m = synth.affine_mesh(3, N, seed=seed, order=1, lam=lam, deform_frac=deform)
    rng = np.random.default_rng(seed + 7)
    if orders[0] == "checker":
        e = np.arange(m.n_elems)
        ex, ey, ez = e % N, (e // N) % N, e // (N * N)
        m.order = np.where((ex + ey + ez) % 2 == 0, orders[1], orders[2]).astype(np.int32)
    else:
        m.order = rng.integers(orders[0], orders[1] + 1, size=m.n_elems).astype(np.int32)
    if rotate:
        m = synth.rotate_elements(m, seed + 11)
    return m


CASES = {
    "affine_p3to6_n3_rot": lambda: _mesh(3, (3, 6), 61, rotate=True),
    "partly_p2to5_n4": lambda: _mesh(4, (2, 5), 62, deform=0.35),
    "affine_checker78_n2": lambda: _mesh(2, ("checker", 7, 8), 63),
    "partly_p1to8_n3_rot": lambda: _mesh(3, (1, 8), 64, deform=0.5, rotate=True, lam=0.5),
    # groups of orders 3 and 5 mostly affine (split launches), order 4 all affine
    "mostly_p3to5_n4_rot": lambda: _mesh(4, (3, 5), 68, deform=0.05, rotate=True),
}


def _n_affine_direct(mesh):
    X = mesh.coords[mesh.elem_vertices]          # [ne][8][3]
    E = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 4] - X[:, 0]], axis=1)
    bits = np.array([[(v >> k) & 1 for k in range(3)] for v in range(8)], dtype=np.float64)
    pred = X[:, :1] + np.einsum("vk,ekd->evd", bits, E)
    dev = np.abs(X - pred).max(axis=(1, 2))
    size = np.linalg.norm(E, axis=2).max(axis=1)
    return int((dev <= 1e-10 * size).sum())




@pytest.fixture(scope="module", params=list(CASES))
def case(request, P, orc):
    print(f"[affine case {request.param}]", flush=True)
    mesh = CASES[request.param]()
    op = P.SipdgOperator(mesh)
    os.environ["SIPDG_NO_AFFINE"] = "1"
    try:
        op_pp = P.SipdgOperator(mesh)
    finally:
        del os.environ["SIPDG_NO_AFFINE"]
    return request.param, mesh, op, op_pp, orc.prepare(mesh)


def test_detected_count(case):
    name, mesh, op, op_pp, om = case
    n = _n_affine_direct(mesh)
    assert op.n_affine == n, (op.n_affine, n)
    assert op_pp.n_affine == 0
    if name.startswith("affine"):
        assert n == mesh.n_elems
    else:
        assert 0 < n < mesh.n_elems


def test_apply_parity(case):
    name, mesh, op, op_pp, om = case
    x = synth.random_coefficients(mesh, 5101)
    y_ref = om.apply(x)
    xt = torch.tensor(x, device="cuda")
    y = op.apply(xt).cpu().numpy()
    e64 = rel(y, y_ref)
    y32 = op.apply(xt.float()).double().cpu().numpy()
    e32 = rel(y32, y_ref)
    y_pp = op_pp.apply(xt).cpu().numpy()
    print(f"{name}: fp64 {e64:.2e} fp32 {e32:.2e} vs per-point {rel(y, y_pp):.2e}")
    assert e64 <= 1e-12 and e32 <= 1e-5
    assert rel(y, y_pp) <= 1e-13
    # symmetric and deterministic with the split launches
    z = torch.tensor(synth.random_coefficients(mesh, 5102), device="cuda")
    assert torch.equal(op.apply(xt), op.apply(xt))
    a, b = float(torch.dot(z, op.apply(xt))), float(torch.dot(xt, op.apply(z)))
    assert abs(a - b) <= 1e-12 * (abs(a) + abs(b))
    # deformed part from the trilinear map, affine part from its constants
    op.geometry = "map"
    try:
        ym = op.apply(xt).cpu().numpy()
        ym32 = op.apply(xt.float()).double().cpu().numpy()
        assert rel(ym, y_ref) <= 1e-12 and rel(ym32, y_ref) <= 1e-5 and rel(ym, y) <= 1e-13
    finally:
        op.geometry = "stored"
    # point-to-point flux on the same (split) launches
    op.flux = "p2p"
    try:
        yp = op.apply(xt).cpu().numpy()
        assert rel(yp, om.apply_p2p(x)) <= 1e-12
    finally:
        op.flux = "shared"


def test_variants_read_per_point(case):
    """The persistent and general structures read the per-point factors of
    every element; they agree with the split gather-fold launches."""
    name, mesh, op, op_pp, om = case
    xt = torch.tensor(synth.random_coefficients(mesh, 5103), device="cuda")
    y = op.apply(xt).cpu().numpy()
    keep = op.variant
    try:
        for v in ("gather", "gather_fold_persistent"):
            op.variant = v
            assert rel(op.apply(xt).cpu().numpy(), y) <= 1e-13, v
    finally:
        op.variant = keep


def test_cg_and_param_grad(case):
    name, mesh, op, op_pp, om = case
    x_true = synth.random_coefficients(mesh, 5104)
    b = op.apply(torch.tensor(x_true, device="cuda"))
    for mode in ("f64", "f32_ir"):
        xs, info = op.cg_solve(b, tol=1e-10, mode=mode)
        assert info["converged"] and info["rel_resid"] <= 1e-10, (mode, info)
    # captured iterations (the affine launch forks to a side stream and joins
    # back inside the graph) against plain launches, replayed several times
    xg, info_g = op.cg_solve(b, tol=1e-10, graph_k=0)
    x0, info0 = op.cg_solve(b, tol=1e-10, graph_k=5)
    assert info0["converged"] and rel2(x0.cpu().numpy(), xg.cpu().numpy()) <= 1e-8
    for _ in range(2):
        xh, info_h = op.cg_solve(b, tol=1e-10, graph_k=5)
        assert info_h["iters"] == info0["iters"] and torch.equal(xh, x0)
    rng = np.random.default_rng(5105)
    a = rng.standard_normal(op.n_dofs)
    c = rng.standard_normal(op.n_dofs)
    dl_ref, ds_ref = om.param_grad(a, c)
    dl, ds = op.param_grad(torch.tensor(a, device="cuda"), torch.tensor(c, device="cuda"))
    assert rel(dl.cpu().numpy(), dl_ref) <= 1e-12
    assert abs(float(ds[0]) - ds_ref) <= 1e-12 * abs(ds_ref)
