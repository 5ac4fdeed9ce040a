"""The per-launch measurement entry point: launch structure, the algorithmic
byte shares per launch (they must add up to the algorithmic traffic of one
application) and unchanged results."""

from __future__ import annotations

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


def _alg_bytes(st, dim, word):
    words = (2 * st["n_dofs"] + st["n_volume_points"] * (dim * (dim + 1) // 2 + 1)
             + st["n_interior_trace_points"] * (2 * dim + 1) + st["n_boundary_trace_points"] * (dim + 1)
             + st["n_elems"])
    return word * words + 32 * (st["n_interior_faces"] + st["n_boundary_faces"])


@pytest.mark.parametrize("variant", ["gather_fold", "two_stage", "gather", "gather_fold_persistent"])
def test_apply_timed(P, variant):
    print(f"[apply_timed {variant}]", flush=True)
    m = synth.workload(3, N=6)
    st = P.inspect_mesh(m)
    op = P.SipdgOperator(m)
    op.variant = variant
    groups = len(set(m.order.tolist()))
    x = torch.tensor(synth.random_coefficients(m, 4006), device="cuda")
    y_ref = op.apply(x)
    for dt, word in ((torch.float64, 8), (torch.float32, 4)):
        xx = x.to(dt)
        y = torch.empty_like(xx)
        launches = op.apply_timed(xx, y, reps=3)
        if variant == "gather_fold_persistent":
            # one launch per stage for every order
            assert [(L["stage"], L["order"], L["elements"]) for L in launches] == [(1, 0, m.n_elems), (2, 0, m.n_elems)]
            assert sum(L["alg_bytes"] for L in launches) == pytest.approx(_alg_bytes(st, 3, word), rel=1e-12)
            if dt == torch.float64:
                assert torch.equal(y, y_ref)
            continue
        if variant == "gather_fold":
            # orders <= 6: one trace launch for every order, then one apply per order
            assert [(L["stage"], L["order"], L["elements"]) for L in launches[:1]] == [(1, 0, m.n_elems)]
            launches_t = launches[:1]
        else:
            launches_t = launches[:groups]
            assert [L["stage"] for L in launches_t] == [1] * groups
        nt = len(launches_t)
        assert len(launches) == nt + groups
        assert [L["stage"] for L in launches[nt:]] == [2] * groups
        assert sorted(L["order"] for L in launches[nt:]) == sorted(set(m.order.tolist()))
        assert sum(L["elements"] for L in launches[nt:]) == m.n_elems
        assert all(L["ms"] > 0 for L in launches)
        assert sum(L["alg_bytes"] for L in launches) == pytest.approx(_alg_bytes(st, 3, word), rel=1e-12)
        if dt == torch.float64:
            assert torch.equal(y, y_ref)
        else:
            assert torch.allclose(y.double(), y_ref, rtol=0, atol=1e-5 * float(y_ref.abs().max()))


def test_autotune_cache_round_trip(P, tmp_path):
    """The autotuner writes its result to the JSON cache (key: mesh signature,
    library source hash, GPU); a second handle on the same mesh takes the
    cached tuning without timing; a different mesh adds a second record; the
    applies agree bitwise whichever structure was kept."""
    import json
    print("[autotune cache]", flush=True)
    path = tmp_path / "tune.json"
    m = synth.workload(3, N=6)
    op1 = P.SipdgOperator(m)
    ms1 = op1.autotune(3, cache_path=path)
    t1 = op1.tuning()
    assert not t1["from_cache"] and ms1[t1["variant"]] == min(ms1.values())
    rec = json.load(open(path))
    assert len(rec) == 1
    key = next(iter(rec))
    assert key.startswith(t1["signature"])
    assert rec[key]["variant"] == P._capi.VARIANTS[t1["variant"]]
    op2 = P.SipdgOperator(m)
    ms2 = op2.autotune(3, cache_path=path)
    t2 = op2.tuning()
    assert t2["from_cache"] and t2["variant"] == t1["variant"] and t2["tile"] == t1["tile"]
    assert t2["budget"] == t1["budget"] and t2["signature"] == t1["signature"]
    assert ms2 == pytest.approx(ms1, rel=1e-5)
    x = torch.tensor(synth.random_coefficients(m, 4007), device="cuda")
    assert torch.equal(op1.apply(x), op2.apply(x))
    # another mesh: another key, the first record kept
    m3 = synth.workload(5, N=4)
    op3 = P.SipdgOperator(m3)
    op3.autotune(3, cache_path=path)
    assert op3.tuning()["signature"] != t1["signature"]
    rec = json.load(open(path))
    assert len(rec) == 2 and key in rec
