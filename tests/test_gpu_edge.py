"""Edge cases of the C ABI on the GPU: an empty mesh, and a batch that holds
an empty problem between two others (ragged problem sizes)."""

from __future__ import annotations

import copy

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2504_03573_amd as P
    return P


def _empty(dim=3):
    m = copy.deepcopy(synth.small_mesh(dim, 1, 2, seed=1))
    m.elem_vertices = m.elem_vertices[:0].copy()
    m.order = m.order[:0].copy()
    m.lam = m.lam[:0].copy()
    return m


def test_empty_mesh(P):
    print("[empty mesh]", flush=True)
    op = P.SipdgOperator(_empty())
    assert op.n_dofs == 0 and op.n_elems == 0
    for dt in (torch.float64, torch.float32):
        x = torch.empty(0, dtype=dt, device="cuda")
        assert op.apply(x).numel() == 0
    x = torch.empty(0, dtype=torch.float64, device="cuda")
    assert op.apply_transpose(x).numel() == 0
    for mode in ("f64", "f32_ir", "f32_ru"):
        xs, info = op.cg_solve(x, tol=1e-10, mode=mode)
        assert xs.numel() == 0 and info["converged"] and info["iters"] == 0 and info["rel_resid"] == 0.0
    dl, ds = op.param_grad(x, x)
    assert dl.numel() == 0 and float(ds[0]) == 0.0


def test_batch_with_empty_problem(P):
    print("[batch with an empty problem]", flush=True)
    ms = [synth.small_mesh(3, 2, ("random", 2, 5), seed=31, rotate=True, lam=1.0), _empty(),
          synth.small_mesh(3, 3, 3, seed=32, lam=4.0)]
    bop = P.SipdgOperator.batch(ms)
    singles = [P.SipdgOperator(m) for m in (ms[0], ms[2])]
    for op in singles:
        op.variant = bop.variant
    off = bop.problem_dof_offsets
    assert off[1] == off[2]
    rng = np.random.default_rng(5)
    x = torch.tensor(rng.standard_normal(bop.n_dofs), device="cuda")
    y = bop.apply(x)
    for op, i in zip(singles, (0, 2)):
        assert torch.equal(op.apply(x[off[i]:off[i + 1]].contiguous()), y[off[i]:off[i + 1]]), i
    for mode in ("f64", "f32_ir", "f32_ru"):
        xs, info = bop.cg_solve(y, tol=1e-10, mode=mode)
        assert info["converged"] and info["rel_resid"] <= 1e-10, (mode, info)
        r = y - bop.apply(xs)
        for i in (0, 2):
            assert float(r[off[i]:off[i + 1]].norm() / y[off[i]:off[i + 1]].norm()) <= 1e-10, (mode, i)
    dl, ds = bop.param_grad(x, x)
    assert float(ds[1]) == 0.0
    for op, i in zip(singles, (0, 2)):
        _, dsi = op.param_grad(x[off[i]:off[i + 1]].contiguous(), x[off[i]:off[i + 1]].contiguous())
        assert abs(float(ds[i]) - float(dsi[0])) <= 1e-13 * abs(float(dsi[0])), i
