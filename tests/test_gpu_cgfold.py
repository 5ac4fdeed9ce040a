"""The folded CG iteration (x and p updated inside the next application's
trace stage, r alone in the vector update) against the separate vector
kernels (SIPDG_NO_FOLD=1): the same arithmetic in the same order, so the
solutions, iteration counts and checkpoints are equal bit for bit, in every
solver mode, on single and batched handles (a batch where one problem stops
long before the others)."""

from __future__ import annotations

import os

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


def _solve(op, b, mode, fold, **kw):
    if fold:
        os.environ.pop("SIPDG_NO_FOLD", None)
    else:
        os.environ["SIPDG_NO_FOLD"] = "1"
    try:
        xs, info = op.cg_solve(b, tol=1e-10, mode=mode, **kw)
        torch.cuda.synchronize()
        return xs.clone(), info
    finally:
        os.environ.pop("SIPDG_NO_FOLD", None)


CASES = {
    "3d_p1to6_n4_rot": lambda: [synth.small_mesh(3, 4, ("random", 1, 6), seed=61, rotate=True, lam=2.0)],
    "w5_recipe_6cubed": lambda: [synth.workload(5, N=6)],
    "batch3_uneven": lambda: [synth.small_mesh(3, 3, ("random", 2, 4), seed=62, lam=50.0),
                              synth.small_mesh(3, 5, ("random", 3, 6), seed=63, lam=0.3),
                              synth.small_mesh(3, 2, 5, seed=64, lam=5.0)],
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("mode", ["f64", "f32_ir", "f32_ru"])
def test_fold_equals_separate(P, name, mode):
    print(f"[cg fold {name} {mode}]", flush=True)
    meshes = CASES[name]()
    op = P.SipdgOperator(meshes[0]) if len(meshes) == 1 else P.SipdgOperator.batch(meshes)
    rng = np.random.default_rng(65)
    b = torch.tensor(rng.standard_normal(op.n_dofs), device="cuda")
    x1, i1 = _solve(op, b, mode, True)
    x0, i0 = _solve(op, b, mode, False)
    print(f"{name} {mode}: {i1['iters']} / {i0['iters']} its, resid {i1['rel_resid']:.2e}", flush=True)
    assert i1["converged"] and i0["converged"]
    assert i1["iters"] == i0["iters"] and i1["outer_iters"] == i0["outer_iters"]
    assert torch.equal(x1, x0)


def test_fold_checkpoints_equal(P):
    """Checkpointed iterates (x brought up to date before each callback) and
    a resume from one of them match the separate kernels."""
    m = synth.small_mesh(3, 4, ("random", 2, 5), seed=66, lam=1.0)
    op = P.SipdgOperator(m)
    b = torch.tensor(np.random.default_rng(67).standard_normal(op.n_dofs), device="cuda")
    snaps = {True: [], False: []}
    for fold in (True, False):
        def cb(x, r, it, fold=fold):
            snaps[fold].append((it, x.clone(), r.clone()))
        _solve(op, b, "f64", fold, checkpoint=cb, checkpoint_every=20)
    assert len(snaps[True]) == len(snaps[False]) > 2
    for (ia, xa, ra), (ib, xb, rb) in zip(snaps[True], snaps[False]):
        assert ia == ib
        assert torch.equal(xa, xb) and torch.equal(ra, rb)
    it, xk, _ = snaps[True][1]
    xr1, ir1 = _solve(op, b, "f64", True, x0=xk)
    xr0, ir0 = _solve(op, b, "f64", False, x0=xk)
    assert ir1["iters"] == ir0["iters"] and torch.equal(xr1, xr0)
