"""Parity over seeded random meshes: each case draws its dimension, size,
order range (1..8), rotations, per-element lambda and penalty scale from its
seed, and every kernel structure that accepts the mesh, the modified C0 modal
basis and the Gauss volume points are compared with the oracle element-wise
(FP64 within 1e-12, FP32 within 1e-5, `rel` of tests/parity.py).  The fixed
cases elsewhere cover chosen structures; these cover combinations of orders,
orientations and sizes nobody picked."""

from __future__ import annotations

import numpy as np
import pytest

import synth
from tests.parity import rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SEEDS = list(range(48))


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


def _mesh(seed):
    rng = np.random.default_rng(9000 + seed)
    dim = 3 if seed % 4 else 2
    N = int(rng.integers(2, 4)) if dim == 3 else int(rng.integers(3, 6))
    lo = int(rng.integers(1, 5))
    hi = int(rng.integers(lo, 9))
    m = synth.small_mesh(dim, N, ("random", lo, hi), seed=9100 + seed, rotate=bool(rng.integers(0, 2)),
                         rot_seed=9200 + seed, sigma=float(rng.choice([0.5, 1.0, 2.0])))
    m.lam = rng.uniform(0.0, 20.0, size=m.n_elems)
    return m


def _structures(mesh):
    """The kernel structures the library accepts for this mesh."""
    pmax = int(mesh.order.max())
    if mesh.dim == 2:
        return ("gather", "gather_fold") + (("gather_fold_fused",) if pmax <= 6 else ())
    if pmax > 6:
        return ("gather", "gather_fold", "gather_fold_persistent")
    return ("gather", "two_stage", "fused", "gather_fold", "gather_fold_fused", "gather_fold_persistent")


@pytest.mark.parametrize("seed", SEEDS)
def test_random_mesh_parity(P, orc, seed):
    mesh = _mesh(seed)
    print(f"[random mesh {seed}: dim {mesh.dim}, {mesh.n_elems} elements, orders "
          f"{int(mesh.order.min())}..{int(mesh.order.max())}]", flush=True)
    op = P.SipdgOperator(mesh)
    x = synth.random_coefficients(mesh, 9300 + seed)
    xt = torch.tensor(x, device="cuda")
    y_ref = orc.prepare(mesh).apply(x)
    for v in _structures(mesh):
        op.variant = v
        e = rel(op.apply(xt).cpu().numpy(), y_ref)
        assert e <= 1e-12, (v, e)
        e32 = rel(op.apply(xt.float()).double().cpu().numpy(), y_ref)
        assert e32 <= 1e-5, (v, e32)
    op.variant = "gather_fold"
    # the allocation-free entry point gives the same bits
    y = op.apply(xt)
    assert torch.equal(op.apply_noalloc(xt, torch.empty_like(xt)), y)
    # the modified C0 modal basis on the default structure
    op.basis = "modal"
    e = rel(op.apply(xt).cpu().numpy(), orc.prepare(mesh, basis="modal").apply(x))
    assert e <= 1e-12, ("modal", e)
    op.basis = "legendre"
    # Gauss volume points: 3-D meshes whose order groups all run the wavefront
    # kernels (refused in 2-D and where an element of order <= 6 meets one of
    # order 7 or 8)
    try:
        op.points = "gauss"
    except P.SipdgError:
        assert mesh.dim == 2 or int(mesh.order.max()) > 6
    else:
        e = rel(op.apply(xt).cpu().numpy(), orc.prepare(mesh, points="gl").apply(x))
        assert e <= 1e-12, ("gauss", e)
        op.points = "gll"
    # a batch of two copies of the mesh gives the same rows for both
    bop = P.SipdgOperator.batch([mesh, mesh])
    yb = bop.apply(torch.cat([xt, xt])).cpu().numpy()
    n = op.n_dofs
    assert rel(yb[:n], y_ref) <= 1e-12 and rel(yb[n:], y_ref) <= 1e-12


@pytest.mark.parametrize("seed", SEEDS)
def test_random_mesh_diagonal_gradients_p2p(P, orc, seed):
    """On the same meshes: the Jacobi diagonal, the transpose application
    (the operator is symmetric), the lambda and penalty-scale gradients of
    a^T A b, and the point-to-point flux (3-D meshes)."""
    mesh = _mesh(seed)
    print(f"[random mesh {seed}: diagonal, transpose, gradients, p2p]", flush=True)
    op = P.SipdgOperator(mesh)
    om = orc.prepare(mesh)
    assert rel(op.diagonal().cpu().numpy(), om.diagonal()) <= 1e-12
    a = synth.random_coefficients(mesh, 9400 + seed)
    b = synth.random_coefficients(mesh, 9500 + seed)
    at, bt = torch.tensor(a, device="cuda"), torch.tensor(b, device="cuda")
    y = op.apply(at).cpu().numpy()
    assert rel(op.apply_transpose(at).cpu().numpy(), y) <= 1e-13
    dl, ds = op.param_grad(at, bt)
    dl_ref, ds_ref = om.param_grad(a, b)
    assert rel(dl.cpu().numpy(), dl_ref) <= 1e-12
    assert abs(float(ds.sum()) - ds_ref) <= 1e-12 * max(abs(ds_ref), 1.0)
    try:
        op.flux = "p2p"
    except P.SipdgError:
        assert mesh.dim == 2   # the point-to-point flux is built for 3-D meshes
        return
    assert rel(op.apply(at).cpu().numpy(), om.apply_p2p(a)) <= 1e-12


@pytest.mark.parametrize("seed", list(range(12)))
def test_random_batch_solves(P, orc, seed):
    """Batches of two to four random meshes of one dimension solved to 1e-10
    in FP64 and in FP32 inside FP64 refinement: every problem's residual,
    recomputed with the oracle's operator, meets the tolerance."""
    rng = np.random.default_rng(9600 + seed)
    # one dimension per batch (3-D for most seeds, 2-D for every fourth)
    pool = [s for s in SEEDS if (s % 4 == 0) == (seed % 4 == 0)]
    meshes = [_mesh(int(s)) for s in rng.choice(pool, size=int(rng.integers(2, 5)), replace=False)]
    print(f"[random batch {seed}: {len(meshes)} problems]", flush=True)
    bop = P.SipdgOperator.batch(meshes)
    off = bop.problem_dof_offsets
    b = rng.standard_normal(bop.n_dofs)
    bt = torch.tensor(b, device="cuda")
    for mode in ("f64", "f32_ir"):
        xs, info = bop.cg_solve(bt, tol=1e-10, mode=mode)
        assert info["converged"], (mode, info)
        x = xs.cpu().numpy()
        for i, m in enumerate(meshes):
            s = slice(int(off[i]), int(off[i + 1]))
            r = b[s] - orc.prepare(m).apply(x[s])
            assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(b[s]), (mode, i)
