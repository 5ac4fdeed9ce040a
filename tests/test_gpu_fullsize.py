"""Parity at the workloads' full sizes, in the launch configuration the
benchmark times: the whole 2-D 64^2, 3-D 32^3 and 3-D 24^3 workloads
against the full oracle (every element), also with geometry from the maps,
the point-to-point flux and Gauss volume points, and the 64-problem batch
(every element of 12 problems, sampled element rows of 12 more).  Each comparison checks the relative 2-norm and the element-wise
max-abs error (``tests.parity.rel``)."""

from __future__ import annotations

import numpy as np
import pytest

import synth
from tests.parity import rel, rows_of, worst_element

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


def _check(tag, y, y_ref, tol, off):
    e = rel(y, y_ref)
    we, wv = worst_element(y, y_ref, off)
    print(f"{tag}: err {e:.2e} (worst element {we}: {wv:.2e})", flush=True)
    assert e <= tol, (tag, e, we)


def test_workload2_full(env):
    P, oracle = env
    print("[workload 2 full]", flush=True)
    m = synth.workload(2)
    op = P.SipdgOperator(m)
    om = oracle.prepare(m)
    x = synth.random_coefficients(m, 4002)
    y_ref = om.apply(x)
    y = op.apply(torch.tensor(x, device="cuda")).cpu().numpy()
    _check("w2 fp64", y, y_ref, 1e-12, om.dof_off)
    y32 = op.apply(torch.tensor(x, device="cuda", dtype=torch.float32)).double().cpu().numpy()
    _check("w2 fp32", y32, y_ref, 1e-5, om.dof_off)


@pytest.mark.parametrize("k", [3, 5])
def test_workload_all_elements(env, k):
    P, oracle = env
    print(f"[workload {k} all elements]", flush=True)
    m = synth.workload(k)
    op = P.SipdgOperator(m)
    om = oracle.prepare(m)
    off = om.dof_off
    x = synth.random_coefficients(m, 4000 + k)
    xt = torch.tensor(x, device="cuda")
    y_ref = om.apply(x)
    default = op.variant
    for v in ["gather", "two_stage", "fused", "gather_fold", "gather_fold_fused", "gather_fold_persistent"]:
        op.variant = v
        y = op.apply(xt).cpu().numpy()
        _check(f"w{k} {v} fp64", y, y_ref, 1e-12, off)
    op.variant = default
    y32 = op.apply(xt.float()).double().cpu().numpy()
    _check(f"w{k} {default} fp32", y32, y_ref, 1e-5, off)
    # geometry from the element maps
    op.variant = "gather_fold"
    op.geometry = "map"
    try:
        _check(f"w{k} map fp64", op.apply(xt).cpu().numpy(), y_ref, 1e-12, off)
        _check(f"w{k} map fp32", op.apply(xt.float()).double().cpu().numpy(), y_ref, 1e-5, off)
    finally:
        op.geometry = "stored"
        op.variant = default
    # point-to-point flux against the oracle's point-to-point operator
    yp_ref = om.apply_p2p(x)
    op.flux = "p2p"
    try:
        _check(f"w{k} p2p fp64", op.apply(xt).cpu().numpy(), yp_ref, 1e-12, off)
        _check(f"w{k} p2p fp32", op.apply(xt.float()).double().cpu().numpy(), yp_ref, 1e-5, off)
    finally:
        op.flux = "shared"
    # Gauss volume points against the oracle's Gauss operator
    yg_ref = oracle.prepare(m, points="gl").apply(x)
    op.points = "gauss"
    try:
        _check(f"w{k} gauss fp64", op.apply(xt).cpu().numpy(), yg_ref, 1e-12, off)
        _check(f"w{k} gauss fp32", op.apply(xt.float()).double().cpu().numpy(), yg_ref, 1e-5, off)
    finally:
        op.points = "gll"
    # properties at full size: symmetry and determinism
    rng2 = np.random.default_rng(20 + k)
    a = torch.tensor(rng2.standard_normal(op.n_dofs), device="cuda")
    s1 = float(torch.dot(a, op.apply(xt)))
    s2 = float(torch.dot(xt, op.apply(a)))
    assert abs(s1 - s2) <= 1e-12 * (abs(s1) + abs(s2))
    assert torch.equal(op.apply(xt), op.apply(xt))


def test_workload4_batched(env):
    P, oracle = env
    print("[workload 4 batched]", flush=True)
    meshes = synth.workload(4)
    bop = P.SipdgOperator.batch(meshes)
    rng = np.random.default_rng(44)
    x = rng.standard_normal(bop.n_dofs)
    y = bop.apply(torch.tensor(x, device="cuda")).cpu().numpy()
    y32 = bop.apply(torch.tensor(x, device="cuda", dtype=torch.float32)).double().cpu().numpy()
    off = bop.problem_dof_offsets
    # every element of 12 problems drawn from the cheaper half for the dense
    # oracle (cost ~ elements x (p+1)^3 (p+2)^3), sampled rows of 12 others
    cost = np.array([m.n_elems * (int(m.order[0]) + 1) ** 3 * (int(m.order[0]) + 2) ** 3 for m in meshes])
    cheap = np.flatnonzero(cost <= np.median(cost))
    full = set(rng.choice(cheap, size=12, replace=False).tolist())
    rest = [i for i in range(len(meshes)) if i not in full]
    picked = sorted(full | set(rng.choice(rest, size=12, replace=False).tolist()))
    for i in picked:
        m = meshes[i]
        om = oracle.prepare(m)
        xi = x[off[i]:off[i + 1]]
        if i in full:
            y_ref = om.apply(xi)
            rows = np.arange(om.n_dofs)
        else:
            elems = np.sort(rng.choice(m.n_elems, size=min(40, m.n_elems), replace=False))
            y_ref = om.apply(xi, elems=elems)
            rows = rows_of(om.dof_off, elems)
        yi = y[off[i]:off[i + 1]]
        yi32 = y32[off[i]:off[i + 1]]
        e64, e32 = rel(yi[rows], y_ref[rows]), rel(yi32[rows], y_ref[rows])
        print(f"problem {i} (p={int(m.order[0])}, {m.n_elems} elements, {'all' if i in full else 'sampled'}): "
              f"fp64 {e64:.2e} fp32 {e32:.2e}", flush=True)
        assert e64 <= 1e-12, i
        assert e32 <= 1e-5, i


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
