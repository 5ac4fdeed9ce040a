"""The allocation-free application sipdg_apply_noalloc against sipdg_apply,
through the C ABI: two calls in a row on the library's per-GPU scratch
array, the second with a smaller mesh (so it runs on the stale contents the
first one left), FP64 and FP32, results equal bit for bit (same kernels),
and the FP64 result within the parity tolerance of the oracle."""

from __future__ import annotations

import ctypes

import numpy as np
import pytest

import synth
from tests.parity import rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import oracle
    import paper_2504_03573_amd as P
    from paper_2504_03573_amd import _capi as C
    oracle.build(force=False)
    return P, C, oracle


def _call(C, op, x, y):
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    prec = C.SIPDG_F64 if x.dtype == torch.float64 else C.SIPDG_F32
    rc = C.load().sipdg_apply_noalloc(op._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                      prec, stream)
    return rc


def test_noalloc_apply_matches_apply_twice(env):
    P, C, oracle = env
    cases = [
        ("3-D 7^3, orders 3..6, rotated", synth.small_mesh(3, 7, ("random", 3, 6), seed=31, lam=2.0, rotate=True)),
        ("3-D 3^3, orders 1..4", synth.small_mesh(3, 3, ("random", 1, 4), seed=32, lam=0.5)),
    ]
    sizes = []
    for name, m in cases:
        print(f"[noalloc {name}]", flush=True)
        op = P.SipdgOperator(m)
        sizes.append(op.n_dofs)
        x = torch.tensor(synth.random_coefficients(m, 4101), device="cuda")
        y_ref = op.apply(x)
        y = torch.full_like(x, float("nan"))
        assert _call(C, op, x, y) == 0, C.load().sipdg_last_error()
        torch.cuda.synchronize()
        assert torch.equal(y, y_ref), float((y - y_ref).abs().max())
        y_np = y.cpu().numpy()
        e64 = rel(y_np, oracle.prepare(m).apply(x.cpu().numpy()))
        x32 = x.float()
        y32_ref = op.apply(x32)
        y32 = torch.full_like(x32, float("nan"))
        assert _call(C, op, x32, y32) == 0, C.load().sipdg_last_error()
        torch.cuda.synchronize()
        assert torch.equal(y32, y32_ref), float((y32 - y32_ref).abs().max())
        print(f"{name}: {op.n_dofs} dofs, FP64 vs oracle {e64:.2e}, equal to sipdg_apply bit for bit", flush=True)
        assert e64 <= 1e-12
    assert sizes[1] < sizes[0]


def test_noalloc_rejects(env):
    P, C, _ = env
    m = synth.small_mesh(3, 2, ("random", 2, 3), seed=33)
    op = P.SipdgOperator(m)
    x = torch.zeros(op.n_dofs, dtype=torch.float64, device="cuda")
    assert _call(C, op, x, x) == -1   # aliasing
    assert C.load().sipdg_apply_noalloc(None, None, None, C.SIPDG_F64, None) == -1
    op.flux = "p2p"
    y = torch.empty_like(x)
    assert _call(C, op, x, y) == -1
