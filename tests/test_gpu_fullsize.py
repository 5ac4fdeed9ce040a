"""Parity at the workloads' full sizes, in the launch configuration the
benchmark times: the whole 2-D 64^2 workload against the full oracle, and
sampled element rows of the 3-D workloads (the oracle evaluates the rows of
a random subset of elements one by one), also with geometry from the maps,
the point-to-point flux and Gauss volume points."""

from __future__ import annotations

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import oracle
    import paper_2504_03573_amd as P
    oracle.build(force=False)
    return P, oracle


def _rows(om, off, elems):
    return np.concatenate([np.arange(off[e], off[e + 1]) for e in elems])


def test_workload2_full(env):
    P, oracle = env
    print("[workload 2 full]", flush=True)
    m = synth.workload(2)
    op = P.SipdgOperator(m)
    om = oracle.prepare(m)
    x = synth.random_coefficients(m, 4002)
    y_ref = om.apply(x)
    y = op.apply(torch.tensor(x, device="cuda")).cpu().numpy()
    assert np.linalg.norm(y - y_ref) <= 1e-12 * np.linalg.norm(y_ref)
    y32 = op.apply(torch.tensor(x, device="cuda", dtype=torch.float32)).double().cpu().numpy()
    assert np.linalg.norm(y32 - y_ref) <= 1e-5 * np.linalg.norm(y_ref)


@pytest.mark.parametrize("k", [3, 5])
def test_workload_sampled_rows(env, k):
    P, oracle = env
    print(f"[workload {k} sampled]", flush=True)
    m = synth.workload(k)
    op = P.SipdgOperator(m)
    om = oracle.prepare(m)
    x = synth.random_coefficients(m, 4000 + k)
    rng = np.random.default_rng(10 + k)
    elems = np.sort(rng.choice(m.n_elems, size=300, replace=False))
    y_ref = om.apply(x, elems=elems)
    rows = _rows(om, om.dof_off, elems)
    for v in (["gather", "two_stage", "fused", "gather_fold", "gather_fold_fused", "gather_fold_persistent"] if op.variant != "gather" else ["gather"]):
        op.variant = v
        y = op.apply(torch.tensor(x, device="cuda")).cpu().numpy()
        assert np.linalg.norm(y[rows] - y_ref[rows]) <= 1e-12 * np.linalg.norm(y_ref[rows]), v
    y32 = op.apply(torch.tensor(x, device="cuda", dtype=torch.float32)).double().cpu().numpy()
    assert np.linalg.norm(y32[rows] - y_ref[rows]) <= 1e-5 * np.linalg.norm(y_ref[rows])
    # geometry from the element maps, same rows
    op.variant = "gather_fold"
    op.geometry = "map"
    try:
        y = op.apply(torch.tensor(x, device="cuda")).cpu().numpy()
        assert np.linalg.norm(y[rows] - y_ref[rows]) <= 1e-12 * np.linalg.norm(y_ref[rows])
    finally:
        op.geometry = "stored"
    # point-to-point flux against the oracle's, same rows
    yp_ref = om.apply_p2p(x, elems=elems)
    op.flux = "p2p"
    try:
        y = op.apply(torch.tensor(x, device="cuda")).cpu().numpy()
        assert np.linalg.norm(y[rows] - yp_ref[rows]) <= 1e-12 * np.linalg.norm(yp_ref[rows])
        y32 = op.apply(torch.tensor(x, device="cuda", dtype=torch.float32)).double().cpu().numpy()
        assert np.linalg.norm(y32[rows] - yp_ref[rows]) <= 1e-5 * np.linalg.norm(yp_ref[rows])
    finally:
        op.flux = "shared"
    # Gauss volume points against the oracle's Gauss operator, same rows
    yg_ref = oracle.prepare(m, points="gl").apply(x, elems=elems)
    op.points = "gauss"
    try:
        y = op.apply(torch.tensor(x, device="cuda")).cpu().numpy()
        assert np.linalg.norm(y[rows] - yg_ref[rows]) <= 1e-12 * np.linalg.norm(yg_ref[rows])
        y32 = op.apply(torch.tensor(x, device="cuda", dtype=torch.float32)).double().cpu().numpy()
        assert np.linalg.norm(y32[rows] - yg_ref[rows]) <= 1e-5 * np.linalg.norm(yg_ref[rows])
    finally:
        op.points = "gll"
    # properties at full size: symmetry and determinism
    rng2 = np.random.default_rng(20 + k)
    a = torch.tensor(rng2.standard_normal(op.n_dofs), device="cuda")
    xa = torch.tensor(x, device="cuda")
    s1 = float(torch.dot(a, op.apply(xa)))
    s2 = float(torch.dot(xa, op.apply(a)))
    assert abs(s1 - s2) <= 1e-12 * (abs(s1) + abs(s2))


def test_workload4_batched_sampled(env):
    P, oracle = env
    print("[workload 4 batched sampled]", flush=True)
    meshes = synth.workload(4)
    bop = P.SipdgOperator.batch(meshes)
    rng = np.random.default_rng(44)
    x = rng.standard_normal(bop.n_dofs)
    y = bop.apply(torch.tensor(x, device="cuda")).cpu().numpy()
    y32 = bop.apply(torch.tensor(x, device="cuda", dtype=torch.float32)).double().cpu().numpy()
    off = bop.problem_dof_offsets
    for i in rng.choice(len(meshes), size=3, replace=False):
        m = meshes[i]
        om = oracle.prepare(m)
        xi = x[off[i]:off[i + 1]]
        elems = np.sort(rng.choice(m.n_elems, size=min(60, m.n_elems), replace=False))
        y_ref = om.apply(xi, elems=elems)
        rows = _rows(om, om.dof_off, elems)
        yi = y[off[i]:off[i + 1]]
        assert np.linalg.norm(yi[rows] - y_ref[rows]) <= 1e-12 * np.linalg.norm(y_ref[rows]), i
        yi32 = y32[off[i]:off[i + 1]]
        assert np.linalg.norm(yi32[rows] - y_ref[rows]) <= 1e-5 * np.linalg.norm(y_ref[rows]), i


def test_workload3_cg_full(env):
    """The solves the benchmark times, at full size: both modes reach a true
    relative residual of 1e-10 (recomputed here with an FP64 apply)."""
    P, oracle = env
    print("[workload 3 cg]", flush=True)
    import math
    m = synth.workload(3)
    op = P.SipdgOperator(m)
    k = math.pi
    b = op.rhs(lambda X: (10 + 3 * k * k) * torch.sin(k * X[:, 0]) * torch.sin(k * X[:, 1]) * torch.sin(k * X[:, 2]),
               lambda X: torch.zeros(X.shape[0], dtype=torch.float64, device=X.device))
    for mode in ("f64", "f32_ir"):
        xs, info = op.cg_solve(b, tol=1e-10, mode=mode)
        r = float((b - op.apply(xs)).norm() / b.norm())
        print(f"workload 3 {mode}: {info}, recomputed residual {r:.3e}", flush=True)
        assert info["converged"] and r <= 1e-10 * (1 + 1e-6), (mode, r)
