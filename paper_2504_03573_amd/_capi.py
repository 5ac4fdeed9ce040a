"""ctypes declarations of the C ABI in ``include/sipdg.h``.

Argument marshalling only: every computation runs in the HIP library.  If
``libsipdg.so`` is missing the import fails loudly; there is no fallback."""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsipdg.so")

SIPDG_OK = 0
ERRORS = {
    -1: "SIPDG_EINVAL",
    -2: "SIPDG_EMESH",
    -3: "SIPDG_ENOMEM",
    -4: "SIPDG_EHIP",
    -5: "SIPDG_ENOCONV",
    -6: "SIPDG_EBREAKDOWN",
}
SIPDG_NOALLOC_SCRATCH_BYTES = 160 << 20
SIPDG_F64 = 0
SIPDG_F32 = 1
SIPDG_CG_F64 = 0
SIPDG_CG_F32_IR = 1
SIPDG_CG_F32_RU = 2
GEOMETRY = {"stored": 0, "map": 1}
FLUX = {"shared": 0, "p2p": 1}
BASIS = {"legendre": 0, "modal": 1}
POINTS = {"gll": 0, "gauss": 1}
MAX_ORDER = 8
VARIANTS = {"gather": 0, "two_stage": 1, "fused": 2, "gather_fold": 3, "gather_fold_fused": 4,
            "gather_fold_persistent": 5}

c_int64_p = ctypes.POINTER(ctypes.c_int64)


class MeshDesc(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("n_vertices", ctypes.c_int64),
        ("coords", ctypes.c_void_p),
        ("n_elems", ctypes.c_int64),
        ("elem_vertices", ctypes.c_void_p),
        ("order", ctypes.c_void_p),
        ("lambda_", ctypes.c_void_p),
        ("h", ctypes.c_double),
        ("penalty_scale", ctypes.c_double),
        ("basis", ctypes.c_int),
        ("quad_extra", ctypes.c_int),
    ]


class Tuning(ctypes.Structure):
    _fields_ = [
        ("variant", ctypes.c_int),
        ("blocks_per_cu", ctypes.c_int),
        ("from_cache", ctypes.c_int),
        ("signature", ctypes.c_uint64),
        ("tile", ctypes.c_int * (MAX_ORDER + 1)),
        ("budget", ctypes.c_int * (MAX_ORDER + 1)),
    ]


class MeshStats(ctypes.Structure):
    _fields_ = [
        ("n_elems", ctypes.c_int64),
        ("n_dofs", ctypes.c_int64),
        ("n_interior_faces", ctypes.c_int64),
        ("n_boundary_faces", ctypes.c_int64),
        ("n_nonconforming_faces", ctypes.c_int64),
        ("orientation_count", ctypes.c_int64 * 8),
        ("n_volume_points", ctypes.c_int64),
        ("n_trace_points", ctypes.c_int64),
        ("n_interior_trace_points", ctypes.c_int64),
        ("n_boundary_trace_points", ctypes.c_int64),
        ("elems_per_order", ctypes.c_int64 * (MAX_ORDER + 1)),
    ]


CKPT_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int)


class CgOpts(ctypes.Structure):
    _fields_ = [
        ("tol", ctypes.c_double),
        ("maxit", ctypes.c_int),
        ("mode", ctypes.c_int),
        ("inner_tol", ctypes.c_double),
        ("precond", ctypes.c_int),
        ("graph_k", ctypes.c_int),
        ("max_outer", ctypes.c_int),
        ("checkpoint", CKPT_FN),
        ("checkpoint_user", ctypes.c_void_p),
        ("checkpoint_every", ctypes.c_int),
        ("x0_given", ctypes.c_int),
        ("ru_delta", ctypes.c_double),
    ]


class CgInfo(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int),
        ("outer_iters", ctypes.c_int),
        ("converged", ctypes.c_int),
        ("rel_resid", ctypes.c_double),
        ("time_ms", ctypes.c_double),
    ]


class GmresOpts(ctypes.Structure):
    _fields_ = [
        ("tol", ctypes.c_double),
        ("restart", ctypes.c_int),
        ("maxit", ctypes.c_int),
        ("precond", ctypes.c_int),
    ]


class GmresInfo(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int),
        ("restarts", ctypes.c_int),
        ("converged", ctypes.c_int),
        ("rel_resid", ctypes.c_double),
        ("time_ms", ctypes.c_double),
    ]


class LaunchInfo(ctypes.Structure):
    _fields_ = [
        ("ms", ctypes.c_double),
        ("stage", ctypes.c_int),
        ("order", ctypes.c_int),
        ("elements", ctypes.c_int64),
        ("alg_bytes", ctypes.c_double),
    ]


# name -> (restype, argtypes)
_vp, _i, _d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
SIGNATURES = {
    "sipdg_create": (_i, [ctypes.POINTER(MeshDesc), ctypes.POINTER(_vp)]),
    "sipdg_create_batch": (_i, [_i, ctypes.POINTER(MeshDesc), ctypes.POINTER(_vp)]),
    "sipdg_destroy": (None, [_vp]),
    "sipdg_mesh_inspect": (_i, [ctypes.POINTER(MeshDesc), ctypes.POINTER(MeshStats)]),
    "sipdg_num_dofs": (_i, [_vp, c_int64_p]),
    "sipdg_num_elems": (_i, [_vp, c_int64_p]),
    "sipdg_num_problems": (_i, [_vp, ctypes.POINTER(_i)]),
    "sipdg_elem_offsets": (_i, [_vp, _vp]),
    "sipdg_problem_offsets": (_i, [_vp, _vp, _vp]),
    "sipdg_apply": (_i, [_vp, _vp, _vp, _i, _vp]),
    "sipdg_apply_noalloc": (_i, [_vp, _vp, _vp, _i, _vp]),
    "sipdg_apply_transpose": (_i, [_vp, _vp, _vp, _i, _vp]),
    "sipdg_apply_stage": (_i, [_vp, _vp, _vp, _i, _i, _vp]),
    "sipdg_apply_timed": (_i, [_vp, _vp, _vp, _i, _i, ctypes.POINTER(LaunchInfo), _i, ctypes.POINTER(_i), _vp]),
    "sipdg_diagonal": (_i, [_vp, _vp, _vp]),
    "sipdg_param_grad": (_i, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "sipdg_set_lambda": (_i, [_vp, _vp, _vp]),
    "sipdg_set_penalty_scale": (_i, [_vp, _i, _d]),
    "sipdg_num_points": (_i, [_vp, c_int64_p, c_int64_p]),
    "sipdg_num_affine": (_i, [_vp, c_int64_p]),
    "sipdg_quad_points": (_i, [_vp, _vp, _vp, _vp]),
    "sipdg_load_vector": (_i, [_vp, _vp, _vp, _vp, _vp]),
    "sipdg_cg_default_opts": (None, [ctypes.POINTER(CgOpts)]),
    "sipdg_cg_solve": (_i, [_vp, _vp, _vp, ctypes.POINTER(CgOpts), ctypes.POINTER(CgInfo), _vp]),
    "sipdg_gmres_default_opts": (None, [ctypes.POINTER(GmresOpts)]),
    "sipdg_gmres_solve": (_i, [_vp, _vp, _vp, ctypes.POINTER(GmresOpts), ctypes.POINTER(GmresInfo), _vp]),
    "sipdg_set_variant": (_i, [_vp, _i]),
    "sipdg_get_variant": (_i, [_vp, ctypes.POINTER(_i)]),
    "sipdg_set_geometry": (_i, [_vp, _i]),
    "sipdg_set_flux": (_i, [_vp, _i]),
    "sipdg_set_basis": (_i, [_vp, _i]),
    "sipdg_get_basis": (_i, [_vp, ctypes.POINTER(_i)]),
    "sipdg_set_points": (_i, [_vp, _i]),
    "sipdg_get_points": (_i, [_vp, ctypes.POINTER(_i)]),
    "sipdg_get_flux": (_i, [_vp, ctypes.POINTER(_i)]),
    "sipdg_get_geometry": (_i, [_vp, ctypes.POINTER(_i)]),
    "sipdg_autotune": (_i, [_vp, ctypes.c_char_p, _i, _vp, _vp]),
    "sipdg_get_tuning": (_i, [_vp, ctypes.POINTER(Tuning)]),
    "sipdg_set_tile": (_i, [_vp, _i, _i, _i]),
    "sipdg_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load(path: str | None = None):
    """Load the library (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"HIP library not built: {p} (run __graft_entry__.build() or "
                          f"python paper_2504_03573_amd/build.py)")
    lib = ctypes.CDLL(p)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


class SipdgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def check(code: int):
    if code != SIPDG_OK:
        msg = load().sipdg_last_error()
        raise SipdgError(code, msg.decode() if msg else "")
    return code
