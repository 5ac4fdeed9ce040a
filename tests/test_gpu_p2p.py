"""Point-to-point interpolation flux (Sec. 3.3, ScatrInterp) through the C ABI
against the oracle's point-to-point operator (pinned in test_oracle_p2p.py):
FP64 within 1e-12 and FP32 within 1e-5 (relative 2-norm); conforming meshes
equal the shared-trace path; the asymmetry of the nonsymmetric case matches
the oracle's; the entry points that need a symmetric operator refuse it."""

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


def _checker_affine(N, a, b, seed):
    m = synth.affine_mesh(3, N, seed=seed, order=1, lam=0.9)
    e = np.arange(m.n_elems)
    m.order = np.where((e % N + (e // N) % N + e // (N * N)) % 2 == 0, a, b).astype(np.int32)
    return synth.rotate_elements(m, seed + 1)


CASES = {
    "random_p1to4_n3_rot": lambda: synth.small_mesh(3, 3, ("random", 1, 4), seed=5, rotate=True, lam=1.5),
    "w3_p3to6_n4": lambda: synth.workload(3, N=4),
    "random_p5to8_n2_rot": lambda: synth.small_mesh(3, 2, ("random", 5, 8), seed=9, rotate=True, lam=0.5),
    "checker24_affine_n3_rot": lambda: _checker_affine(3, 2, 4, 81),
    "single_elem_p3": lambda: synth.small_mesh(3, 1, 3, seed=1, lam=2.0),
}




@pytest.fixture(scope="module", params=list(CASES))
def case(request, P, orc):
    print(f"[p2p case {request.param}]", flush=True)
    mesh = CASES[request.param]()
    op = P.SipdgOperator(mesh)
    op.flux = "p2p"
    return request.param, mesh, op, orc.prepare(mesh)


def test_apply_parity(case):
    name, mesh, op, om = case
    x = synth.random_coefficients(mesh, 6101)
    y_ref = om.apply_p2p(x)
    xt = torch.tensor(x, device="cuda")
    y = op.apply(xt).cpu().numpy()
    y32 = op.apply(xt.float()).double().cpu().numpy()
    print(f"{name}: p2p fp64 {rel(y, y_ref):.2e} fp32 {rel(y32, y_ref):.2e}")
    assert rel(y, y_ref) <= 1e-12
    assert rel(y32, y_ref) <= 1e-5
    assert torch.equal(op.apply(xt), op.apply(xt))


def test_structures_agree(case):
    """The gather-fold path (every face side on its own point set, the
    neighbour's trace interpolated by its own trace stage) and the general
    kernels (interpolation inside the apply) give the same operator."""
    name, mesh, op, om = case
    xt = torch.tensor(synth.random_coefficients(mesh, 6106), device="cuda")
    keep = op.variant
    ys = {}
    try:
        for v in ("gather", "gather_fold"):
            op.variant = v
            ys[v] = op.apply(xt).cpu().numpy()
            y32 = op.apply(xt.float()).double().cpu().numpy()
            assert rel(y32, ys[v]) <= 1e-5, v
        op.geometry = "map"
        ys["map"] = op.apply(xt).cpu().numpy()
        op.geometry = "stored"
    finally:
        op.variant = keep
    assert rel(ys["gather_fold"], ys["gather"]) <= 1e-13
    assert rel(ys["map"], ys["gather"]) <= 1e-13


def test_asymmetry_matches_oracle(case):
    """z^T A x - x^T A z over |z^T A x| + |x^T A z|, GPU against oracle."""
    name, mesh, op, om = case
    x = synth.random_coefficients(mesh, 6102)
    z = synth.random_coefficients(mesh, 6103)
    xt, zt = torch.tensor(x, device="cuda"), torch.tensor(z, device="cuda")
    a = float(torch.dot(zt, op.apply(xt)))
    b = float(torch.dot(xt, op.apply(zt)))
    ao, bo = float(z @ om.apply_p2p(x)), float(x @ om.apply_p2p(z))
    d, do = (a - b) / (abs(a) + abs(b)), (ao - bo) / (abs(ao) + abs(bo))
    print(f"{name}: asymmetry gpu {d:.3e} oracle {do:.3e}")
    assert abs(d - do) <= 1e-11
    if name.startswith("checker24"):
        assert abs(d) >= 1e-4


def test_conforming_equals_shared(P):
    m = synth.small_mesh(3, 3, 4, seed=82, rotate=True, lam=1.1)
    op = P.SipdgOperator(m)
    x = torch.tensor(synth.random_coefficients(m, 6104), device="cuda")
    y0 = op.apply(x)
    op.flux = "p2p"
    y1 = op.apply(x)
    op.flux = "shared"
    assert float((y1 - y0).norm() / y0.norm()) <= 1e-13
    assert torch.equal(op.apply(x), y0)


def test_entry_points_refuse_nonsymmetric(P):
    m = synth.small_mesh(3, 2, ("random", 2, 4), seed=83, lam=1.0)
    op = P.SipdgOperator(m)
    op.flux = "p2p"
    assert op.flux == "p2p"
    x = torch.tensor(synth.random_coefficients(m, 6105), device="cuda")
    for call in (lambda: op.cg_solve(x, tol=1e-8), lambda: op.apply_transpose(x), op.diagonal,
                 lambda: op.param_grad(x, x), op.autotune):
        with pytest.raises(P.SipdgError):
            call()
    op.flux = "shared"
    xs, info = op.cg_solve(op.apply(x), tol=1e-10)
    assert info["converged"]
    m2 = synth.small_mesh(2, 3, 2, seed=84)
    with pytest.raises(P.SipdgError):
        P.SipdgOperator(m2).flux = "p2p"


def test_batch_equals_singles(P):
    """A batched handle under the point-to-point flux (and the modal basis)
    gives each problem's rows of its own handle."""
    ms = [synth.small_mesh(3, 2, ("random", 2, 5), seed=89, rotate=True, lam=1.0),
          synth.small_mesh(3, 3, ("random", 1, 3), seed=90, lam=2.0)]
    bop = P.SipdgOperator.batch(ms)
    singles = [P.SipdgOperator(m) for m in ms]
    off = bop.problem_dof_offsets
    x = torch.tensor(np.random.default_rng(91).standard_normal(bop.n_dofs), device="cuda")
    for basis in ("legendre", "modal"):
        bop.basis = basis
        bop.flux = "p2p"
        y = bop.apply(x)
        for i, op in enumerate(singles):
            op.basis = basis
            op.flux = "p2p"
            yi = op.apply(x[off[i]:off[i + 1]].contiguous())
            assert float((y[off[i]:off[i + 1]] - yi).norm() / yi.norm()) <= 1e-14, (basis, i)
            op.flux = "shared"
        bop.flux = "shared"
