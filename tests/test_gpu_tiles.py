"""Multi-element tiles of the gather-fold apply: every tile shape the library
is built with, on meshes whose order groups end in a partial tile, gives the
one-element kernel's result bit for bit (the same arithmetic per element in
the same order) and the oracle's within the parity bar, in FP64 and FP32,
with stored and map geometry, and inside CG with captured iterations."""

from __future__ import annotations

import numpy as np
import pytest

import synth
from tests.parity import rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# the shapes of tile_shapes.hpp (order, elements per workgroup, budget)
SHAPES = [(1, 7, 2), (1, 7, 4), (2, 4, 2), (2, 4, 4), (3, 2, 2), (3, 2, 3), (3, 5, 2),
          (4, 3, 2), (4, 3, 3), (4, 7, 2), (5, 5, 2)]


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import oracle
    import paper_2504_03573_amd as P
    oracle.build(force=False)
    return P, oracle


MESHES = {
    # orders 1..6 mixed: every low-order group meets finer neighbours (lifted
    # faces) and ends in a partial tile for most shapes
    "3d_random_p1to6_n4_rot": lambda: synth.small_mesh(3, 4, ("random", 1, 6), seed=71, rotate=True, lam=1.3),
    "w3_recipe_n5": lambda: synth.workload(3, N=5),
}


@pytest.fixture(scope="module", params=list(MESHES))
def case(request, env):
    P, oracle = env
    print(f"[tiles {request.param}]", flush=True)
    m = MESHES[request.param]()
    op = P.SipdgOperator(m)
    om = oracle.prepare(m)
    x = synth.random_coefficients(m, 4011)
    return request.param, m, op, om, x


def test_shapes_match_one_element_kernel(case):
    name, m, op, om, x = case
    y_ref = om.apply(x)
    xt = torch.tensor(x, device="cuda")
    present = set(m.order.tolist())
    for geo in ("stored", "map"):
        op.geometry = geo
        base64 = op.apply(xt)
        base32 = op.apply(xt.float())
        for (p, e, b) in SHAPES:
            if p not in present:
                continue
            op.set_tile(p, e, b)
            y64 = op.apply(xt)
            y32 = op.apply(xt.float())
            same = torch.equal(y64, base64) and torch.equal(y32, base32)
            e64 = rel(y64.cpu().numpy(), y_ref)
            e32 = rel(y32.double().cpu().numpy(), y_ref)
            print(f"{name} {geo} p={p} tile={e} budget={b}: bitwise {same}, fp64 {e64:.2e} fp32 {e32:.2e}",
                  flush=True)
            assert e64 <= 1e-12 and e32 <= 1e-5, (p, e, b, geo)
            assert same, (p, e, b, geo)
            op.set_tile(p, 1, 2)
        op.geometry = "stored"


def test_all_orders_tiled_and_cg(case):
    """Every order on its largest tile at once, then a CG solve with captured
    iterations: the same iterates as with one element per wavefront."""
    name, m, op, om, x = case
    xt = torch.tensor(x, device="cuda")
    b = op.apply(xt)
    x_base, info_base = op.cg_solve(b, tol=1e-10, graph_k=5)
    y_base = op.apply(xt)
    best = {}
    for (p, e, bud) in SHAPES:
        if e > best.get(p, (0, 0))[0]:
            best[p] = (e, bud)
    for p, (e, bud) in best.items():
        op.set_tile(p, e, bud)
    try:
        assert torch.equal(op.apply(xt), y_base)
        xs, info = op.cg_solve(b, tol=1e-10, graph_k=5)
        assert info["iters"] == info_base["iters"] and torch.equal(xs, x_base)
    finally:
        for p in best:
            op.set_tile(p, 1, 2)


def test_refuses_unbuilt_shapes(env):
    P, _ = env
    op = P.SipdgOperator(synth.small_mesh(3, 2, 3, seed=5))
    for args in [(3, 3, 2), (6, 2, 2), (0, 1, 2), (9, 1, 2), (3, 2, 5)]:
        with pytest.raises(P.SipdgError):
            op.set_tile(*args)
    op.set_tile(3, 1, 2)
    assert op.tuning()["tile"][3] == 1
