"""C ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and the host-side mesh preprocessing (face matching,
orientation codes, validation errors) behaves as documented."""

from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sipdg.h")


@pytest.fixture(scope="module")
def capi():
    from paper_2504_03573_amd import _capi
    return _capi


def header_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sipdg_[a-z_0-9]+)\s*\(", txt)))


def test_exports_every_declared_symbol(capi):
    lib = capi.load()
    names = header_symbols()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(capi.SIGNATURES)


def test_inspect_workload3_counts():
    from paper_2504_03573_amd import inspect_mesh
    st = inspect_mesh(synth.workload(3))
    N = 32
    assert st["n_elems"] == N ** 3
    assert st["n_interior_faces"] == 3 * N * N * (N - 1)
    assert st["n_boundary_faces"] == 6 * N * N
    order = synth.workload(3).order
    assert st["n_dofs"] == int(((order.astype(np.int64) + 1) ** 3).sum())
    assert sum(st["elems_per_order"]) == N ** 3


def test_inspect_orientations_and_nonconforming():
    from paper_2504_03573_amd import inspect_mesh
    m = synth.small_mesh(3, 4, ("checker", 2, 3), seed=3, rotate=True, rot_seed=5)
    st = inspect_mesh(m)
    assert st["n_nonconforming_faces"] == st["n_interior_faces"]
    assert all(c > 0 for c in st["orientation_count"])
    m2 = synth.small_mesh(2, 5, 3, seed=3)
    st2 = inspect_mesh(m2)
    assert st2["orientation_count"][0] == st2["n_interior_faces"] == 2 * 5 * 4
    assert st2["n_nonconforming_faces"] == 0


def _expect(capi, mesh, code):
    from paper_2504_03573_amd import inspect_mesh
    with pytest.raises(capi.SipdgError) as ei:
        inspect_mesh(mesh)
    assert ei.value.code == code, str(ei.value)


def test_validation_errors(capi):
    m = synth.small_mesh(2, 2, 3, seed=1)
    bad = synth.small_mesh(2, 2, 3, seed=1)
    bad.order = bad.order.copy()
    bad.order[1] = 9
    _expect(capi, bad, -1)
    bad = synth.small_mesh(2, 2, 3, seed=1)
    bad.elem_vertices = bad.elem_vertices.copy()
    bad.elem_vertices[0, 0] = 10 ** 6
    _expect(capi, bad, -1)
    # inverted element: swap two corners along x
    bad = synth.small_mesh(2, 2, 3, seed=1)
    ev = bad.elem_vertices.copy()
    ev[0, [0, 1]] = ev[0, [1, 0]]
    ev[0, [2, 3]] = ev[0, [3, 2]]
    bad.elem_vertices = ev
    _expect(capi, bad, -2)
    # face shared by three elements: duplicate an element
    bad = synth.small_mesh(2, 2, 3, seed=1)
    bad.elem_vertices = np.concatenate([bad.elem_vertices, bad.elem_vertices[:1]])
    bad.order = np.concatenate([bad.order, bad.order[:1]])
    bad.lam = np.concatenate([bad.lam, bad.lam[:1]])
    _expect(capi, bad, -2)
    # non-positive h
    bad = synth.small_mesh(2, 2, 3, seed=1)
    bad.h = 0.0
    _expect(capi, bad, -1)
    from paper_2504_03573_amd import inspect_mesh
    assert inspect_mesh(m)["n_elems"] == 4


def test_create_without_device_reports_error(capi):
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    from paper_2504_03573_amd import SipdgOperator
    with pytest.raises(capi.SipdgError) as ei:
        SipdgOperator(synth.small_mesh(2, 2, 3, seed=1))
    assert ei.value.code == -4


def test_cg_default_opts_layout(capi):
    """The ctypes mirror of sipdg_cg_opts matches the C struct: the library's
    defaults land in the right fields (no device needed)."""
    lib = capi.load()
    o = capi.CgOpts()
    lib.sipdg_cg_default_opts(ctypes.byref(o))
    assert o.tol == 1e-10 and o.maxit == 20000 and o.mode == capi.SIPDG_CG_F64
    assert o.inner_tol == 1e-4 and o.precond == 1 and o.graph_k == 10 and o.max_outer == 50
    assert o.checkpoint_every == 0 and o.x0_given == 0 and o.ru_delta == 0.1
    assert capi.SIPDG_CG_F32_RU == 2


def test_quad_extra_and_basis_fields(capi):
    """quad_extra: 2 (p + 2 GLL points, what the kernels are built for) or 0
    for that default; anything else is EINVAL.  basis: 0 or 1."""
    from paper_2504_03573_amd import inspect_mesh
    m = synth.small_mesh(3, 2, ("random", 1, 4), seed=2)
    ref = inspect_mesh(m)
    assert inspect_mesh(m, quad_extra=0) == ref
    assert inspect_mesh(m, quad_extra=2) == ref
    assert inspect_mesh(m, basis="modal") == ref
    for q in (-1, 1, 3, 4):
        with pytest.raises(capi.SipdgError) as ei:
            inspect_mesh(m, quad_extra=q)
        assert ei.value.code == -1
    d = capi.MeshDesc()
    from paper_2504_03573_amd.operator import _desc_from
    keep = _desc_from(m)
    d = keep.desc
    d.basis = 2
    st = capi.MeshStats()
    assert capi.load().sipdg_mesh_inspect(ctypes.byref(d), ctypes.byref(st)) == -1


def test_struct_layouts_match_header(capi, tmp_path):
    """The ctypes mirrors of the ABI structs have the C compiler's sizes and
    field offsets (a C program built against include/sipdg.h prints them)."""
    import subprocess
    src = tmp_path / "layout.c"
    src.write_text(r"""
#include <stdio.h>
#include <stddef.h>
#include "sipdg.h"
int main(void) {
    printf("%zu %zu %zu %zu\n", sizeof(sipdg_mesh_desc), offsetof(sipdg_mesh_desc, penalty_scale),
           offsetof(sipdg_mesh_desc, basis), offsetof(sipdg_mesh_desc, quad_extra));
    printf("%zu %zu %zu %zu\n", sizeof(sipdg_tuning), offsetof(sipdg_tuning, signature),
           offsetof(sipdg_tuning, tile), offsetof(sipdg_tuning, budget));
    printf("%zu %zu %zu\n", sizeof(sipdg_cg_opts), offsetof(sipdg_cg_opts, checkpoint),
           offsetof(sipdg_cg_opts, ru_delta));
    printf("%zu %zu\n", sizeof(sipdg_launch_info), offsetof(sipdg_launch_info, alg_bytes));
    return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    rows = [list(map(int, r.split())) for r in subprocess.check_output([str(exe)]).decode().split("\n") if r]
    M, T, O, L = capi.MeshDesc, capi.Tuning, capi.CgOpts, capi.LaunchInfo
    assert rows[0] == [ctypes.sizeof(M), M.penalty_scale.offset, M.basis.offset, M.quad_extra.offset]
    assert rows[1] == [ctypes.sizeof(T), T.signature.offset, T.tile.offset, T.budget.offset]
    assert rows[2] == [ctypes.sizeof(O), O.checkpoint.offset, O.ru_delta.offset]
    assert rows[3] == [ctypes.sizeof(L), L.alg_bytes.offset]


def test_tuning_calls_reject_null(capi):
    lib = capi.load()
    ms = (ctypes.c_double * 6)()
    assert lib.sipdg_autotune(None, b"/nonexistent/cache.json", 5, ms, None) == -1
    t = capi.Tuning()
    assert lib.sipdg_get_tuning(None, ctypes.byref(t)) == -1
