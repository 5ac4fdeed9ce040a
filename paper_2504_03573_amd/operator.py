"""Python handle around the C ABI (device memory and streams from torch).

``SipdgOperator(mesh)`` builds one handle; ``SipdgOperator.batch(meshes)``
builds several independent problems in one handle.  Vectors are torch
tensors on the current HIP device in the library's natural layout
(element after element, modes lexicographic)."""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _capi as C


def _stream_ptr(stream=None, device_index=None):
    """The HIP stream handle to launch on: ``stream``'s, else the current
    stream of ``device_index`` (the current device if None)."""
    if stream is not None:
        return ctypes.c_void_p(stream.cuda_stream)
    if device_index is None:
        device_index = torch.cuda.current_device()
    return ctypes.c_void_p(torch._C._cuda_getCurrentRawStream(device_index))


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


_PREC = {torch.float64: C.SIPDG_F64, torch.float32: C.SIPDG_F32}


class _Desc:
    """Keeps the host arrays of one mesh alive while the library reads them."""

    def __init__(self, dim, coords, elem_vertices, order, lam, h, sigma, basis=0, quad_extra=2):
        self.coords = np.ascontiguousarray(coords, dtype=np.float64)
        self.ev = np.ascontiguousarray(elem_vertices, dtype=np.int64)
        self.order = np.ascontiguousarray(order, dtype=np.int32)
        self.lam = np.ascontiguousarray(np.broadcast_to(np.asarray(lam, dtype=np.float64), self.order.shape))
        self.desc = C.MeshDesc(
            dim=int(dim), n_vertices=self.coords.shape[0], coords=self.coords.ctypes.data,
            n_elems=self.ev.shape[0], elem_vertices=self.ev.ctypes.data,
            order=self.order.ctypes.data, lambda_=self.lam.ctypes.data, h=float(h),
            penalty_scale=float(sigma), basis=int(basis), quad_extra=int(quad_extra))


def _desc_from(mesh, basis: str = "legendre", quad_extra: int = 2) -> _Desc:
    return _Desc(mesh.dim, mesh.coords, mesh.elem_vertices, mesh.order, mesh.lam, mesh.h,
                 getattr(mesh, "sigma", 1.0), C.BASIS[basis], quad_extra)


def inspect_mesh(mesh, basis: str = "legendre", quad_extra: int = 2) -> dict:
    """Host-only statistics (face counts, orientations); needs no device."""
    lib = C.load()
    d = _desc_from(mesh, basis, quad_extra)
    st = C.MeshStats()
    C.check(lib.sipdg_mesh_inspect(ctypes.byref(d.desc), ctypes.byref(st)))
    return {
        "n_elems": st.n_elems, "n_dofs": st.n_dofs,
        "n_interior_faces": st.n_interior_faces, "n_boundary_faces": st.n_boundary_faces,
        "n_nonconforming_faces": st.n_nonconforming_faces,
        "orientation_count": list(st.orientation_count),
        "n_volume_points": st.n_volume_points, "n_trace_points": st.n_trace_points,
        "n_interior_trace_points": st.n_interior_trace_points,
        "n_boundary_trace_points": st.n_boundary_trace_points,
        "elems_per_order": list(st.elems_per_order),
    }


class SipdgOperator:
    def __init__(self, mesh=None, basis: str = "legendre", quad_extra: int = 2, _handle=None, _descs=None):
        self._lib = C.load()
        if _handle is None:
            d = _desc_from(mesh, basis, quad_extra)
            h = ctypes.c_void_p()
            C.check(self._lib.sipdg_create(ctypes.byref(d.desc), ctypes.byref(h)))
            _handle = h
            _descs = [d]
        self._h = _handle
        self.dim = _descs[0].desc.dim
        n = ctypes.c_int64()
        C.check(self._lib.sipdg_num_dofs(self._h, ctypes.byref(n)))
        self.n_dofs = n.value
        C.check(self._lib.sipdg_num_elems(self._h, ctypes.byref(n)))
        self.n_elems = n.value
        npb = ctypes.c_int()
        C.check(self._lib.sipdg_num_problems(self._h, ctypes.byref(npb)))
        self.n_problems = npb.value
        off = np.zeros(self.n_elems + 1, dtype=np.int64)
        C.check(self._lib.sipdg_elem_offsets(self._h, off.ctypes.data))
        self.elem_offsets = off
        po = np.zeros(self.n_problems + 1, dtype=np.int64)
        pe = np.zeros(self.n_problems + 1, dtype=np.int64)
        C.check(self._lib.sipdg_problem_offsets(self._h, po.ctypes.data, pe.ctypes.data))
        self.problem_dof_offsets = po
        self.problem_elem_offsets = pe
        nv, nb = ctypes.c_int64(), ctypes.c_int64()
        C.check(self._lib.sipdg_num_points(self._h, ctypes.byref(nv), ctypes.byref(nb)))
        self.n_volume_points, self.n_boundary_points = nv.value, nb.value
        C.check(self._lib.sipdg_num_affine(self._h, ctypes.byref(n)))
        self.n_affine = n.value   # elements whose apply uses per-element geometry
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._dev = self.device.index

    @classmethod
    def batch(cls, meshes, basis: str = "legendre"):
        lib = C.load()
        descs = [_desc_from(m, basis) for m in meshes]
        arr = (C.MeshDesc * len(descs))(*[d.desc for d in descs])
        h = ctypes.c_void_p()
        C.check(lib.sipdg_create_batch(len(descs), arr, ctypes.byref(h)))
        return cls(_handle=h, _descs=descs)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sipdg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ checks
    def _vec(self, t, dtype, n=None, name="vector"):
        n = self.n_dofs if n is None else n
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a device tensor")
        if t.dtype != dtype or t.numel() != n or not t.is_contiguous():
            raise ValueError(f"{name}: need contiguous {dtype} with {n} entries, got {t.dtype} {tuple(t.shape)}")
        return t

    # ------------------------------------------------------------------ operator
    def apply(self, x: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        prec = _PREC.get(x.dtype)
        if prec is None:
            raise TypeError("x must be float64 or float32")
        self._vec(x, x.dtype, name="x")
        y = torch.empty_like(x) if out is None else self._vec(out, x.dtype, name="out")
        C.check(self._lib.sipdg_apply(self._h, x.data_ptr(), y.data_ptr(), prec, _stream_ptr(stream, self._dev)))
        return y

    def apply_noalloc(self, x: torch.Tensor, out: torch.Tensor, stream=None) -> torch.Tensor:
        """y = A x through sipdg_apply_noalloc: the trace buffer is the
        library's fixed per-GPU scratch array, so the call allocates nothing
        (``out`` must be given).  Calls on one GPU must not overlap."""
        prec = _PREC.get(x.dtype)
        if prec is None:
            raise TypeError("x must be float64 or float32")
        self._vec(x, x.dtype, name="x")
        self._vec(out, x.dtype, name="out")
        C.check(self._lib.sipdg_apply_noalloc(self._h, _ptr(x), _ptr(out), prec, _stream_ptr(stream, self._dev)))
        return out

    def apply_stage(self, x: torch.Tensor, stage: int, out: torch.Tensor | None = None, stream=None):
        """Stage 1 (trace values into the handle's buffer) or stage 2 (fluxes,
        volume terms, inner products into ``out``) of one application."""
        prec = _PREC.get(x.dtype)
        if prec is None:
            raise TypeError("x must be float64 or float32")
        self._vec(x, x.dtype, name="x")
        if stage == 2:
            out = torch.empty_like(x) if out is None else self._vec(out, x.dtype, name="out")
        C.check(self._lib.sipdg_apply_stage(self._h, _ptr(x), _ptr(out) if out is not None else None,
                                            prec, int(stage), _stream_ptr(stream, self._dev)))
        return out

    def apply_timed(self, x: torch.Tensor, out: torch.Tensor, reps: int = 20, stream=None) -> list[dict]:
        """Run ``reps`` applications with a HIP event around every kernel
        launch; per launch of one application: mean ms, stage, order, element
        count and the algorithmic bytes of its elements (apply launches)."""
        prec = _PREC.get(x.dtype)
        if prec is None:
            raise TypeError("x must be float64 or float32")
        self._vec(x, x.dtype, name="x")
        self._vec(out, x.dtype, name="out")
        info = (C.LaunchInfo * 64)()
        n = ctypes.c_int()
        C.check(self._lib.sipdg_apply_timed(self._h, _ptr(x), _ptr(out), prec, int(reps), info, 64,
                                            ctypes.byref(n), _stream_ptr(stream, self._dev)))
        return [{"ms": info[i].ms, "stage": info[i].stage, "order": info[i].order,
                 "elements": int(info[i].elements), "alg_bytes": info[i].alg_bytes} for i in range(n.value)]

    def apply_transpose(self, g: torch.Tensor, out: torch.Tensor | None = None, stream=None):
        prec = _PREC.get(g.dtype)
        if prec is None:
            raise TypeError("g must be float64 or float32")
        self._vec(g, g.dtype, name="g")
        y = torch.empty_like(g) if out is None else self._vec(out, g.dtype, name="out")
        C.check(self._lib.sipdg_apply_transpose(self._h, _ptr(g), _ptr(y), prec, _stream_ptr(stream, self._dev)))
        return y

    @property
    def variant(self) -> str:
        v = ctypes.c_int()
        C.check(self._lib.sipdg_get_variant(self._h, ctypes.byref(v)))
        return {b: a for a, b in C.VARIANTS.items()}[v.value]

    @variant.setter
    def variant(self, name: str):
        C.check(self._lib.sipdg_set_variant(self._h, C.VARIANTS[name]))

    @property
    def geometry(self) -> str:
        """Where the default apply takes deformed elements' geometric factors:
        "stored" (per quadrature point, computed at create) or "map" (derived
        at every point from the element's trilinear map)."""
        v = ctypes.c_int()
        C.check(self._lib.sipdg_get_geometry(self._h, ctypes.byref(v)))
        return {b: a for a, b in C.GEOMETRY.items()}[v.value]

    @geometry.setter
    def geometry(self, name: str):
        C.check(self._lib.sipdg_set_geometry(self._h, C.GEOMETRY[name]))

    @property
    def basis(self) -> str:
        """Modal basis of the coefficients: "legendre" (orthogonal, the
        default) or "modal" (modified C0, Table 1)."""
        v = ctypes.c_int()
        C.check(self._lib.sipdg_get_basis(self._h, ctypes.byref(v)))
        return {b: a for a, b in C.BASIS.items()}[v.value]

    @basis.setter
    def basis(self, name: str):
        C.check(self._lib.sipdg_set_basis(self._h, C.BASIS[name]))

    @property
    def points(self) -> str:
        """Volume quadrature points: "gll" (p + 2 Gauss-Lobatto points per
        direction, the default) or "gauss" (p + 2 Gauss points; the faces
        keep the shared trace's GLL points, each side's trace evaluated from
        its coefficients).  Under "gauss": apply, cg_solve and gmres_solve."""
        v = ctypes.c_int()
        C.check(self._lib.sipdg_get_points(self._h, ctypes.byref(v)))
        return {b: a for a, b in C.POINTS.items()}[v.value]

    @points.setter
    def points(self, name: str):
        C.check(self._lib.sipdg_set_points(self._h, C.POINTS[name]))

    @property
    def flux(self) -> str:
        """Interior-face flux of apply: "shared" (shared trace space, the
        default) or "p2p" (point-to-point interpolation; nonsymmetric: the
        apply calls and gmres_solve accept it)."""
        v = ctypes.c_int()
        C.check(self._lib.sipdg_get_flux(self._h, ctypes.byref(v)))
        return {b: a for a, b in C.FLUX.items()}[v.value]

    @flux.setter
    def flux(self, name: str):
        C.check(self._lib.sipdg_set_flux(self._h, C.FLUX[name]))

    def autotune(self, reps: int = 20, cache_path: str | None = None, stream=None) -> dict:
        """Time every allowed kernel structure (and the tile shape of each
        order group's apply launch) and keep the fastest; with ``cache_path``
        a JSON file of earlier results is consulted first and updated."""
        ms = (ctypes.c_double * len(C.VARIANTS))()
        cp = None if cache_path is None else str(cache_path).encode()
        C.check(self._lib.sipdg_autotune(self._h, cp, int(reps), ms, _stream_ptr(stream, self._dev)))
        return {name: ms[i] for name, i in C.VARIANTS.items() if ms[i] > 0}

    def set_tile(self, order: int, tile: int, budget: int):
        """Tile shape of one order's gather-fold apply launch (elements per
        workgroup, register budget in waves per SIMD); (1, 2) is the default."""
        C.check(self._lib.sipdg_set_tile(self._h, int(order), int(tile), int(budget)))

    def tuning(self) -> dict:
        t = C.Tuning()
        C.check(self._lib.sipdg_get_tuning(self._h, ctypes.byref(t)))
        names = {b: a for a, b in C.VARIANTS.items()}
        return {"variant": names[t.variant], "blocks_per_cu": t.blocks_per_cu, "from_cache": bool(t.from_cache),
                "signature": "%016x" % t.signature, "tile": list(t.tile), "budget": list(t.budget)}

    def diagonal(self, stream=None) -> torch.Tensor:
        d = torch.empty(self.n_dofs, dtype=torch.float64, device=self.device)
        C.check(self._lib.sipdg_diagonal(self._h, _ptr(d), _stream_ptr(stream, self._dev)))
        return d

    def param_grad(self, a: torch.Tensor, b: torch.Tensor, stream=None):
        self._vec(a, torch.float64, name="a")
        self._vec(b, torch.float64, name="b")
        dl = torch.empty(self.n_elems, dtype=torch.float64, device=self.device)
        ds = torch.empty(self.n_problems, dtype=torch.float64, device=self.device)
        C.check(self._lib.sipdg_param_grad(self._h, _ptr(a), _ptr(b), _ptr(dl), _ptr(ds),
                                           _stream_ptr(stream, self._dev)))
        return dl, ds

    # Every change of lambda or sigma bumps ``param_generation``, so a cache of
    # the parameters the handle holds (the autograd Functions keep one) can
    # tell that they were set from elsewhere.
    param_generation = 0

    def set_lambda(self, lam: torch.Tensor, stream=None):
        self._vec(lam, torch.float64, n=self.n_elems, name="lambda")
        self.param_generation += 1
        C.check(self._lib.sipdg_set_lambda(self._h, _ptr(lam), _stream_ptr(stream, self._dev)))

    def set_penalty_scale(self, sigma: float, problem: int = -1):
        self.param_generation += 1
        C.check(self._lib.sipdg_set_penalty_scale(self._h, int(problem), float(sigma)))

    def quad_points(self, stream=None):
        xq = torch.empty((self.n_volume_points, self.dim), dtype=torch.float64, device=self.device)
        xb = torch.empty((max(self.n_boundary_points, 1), self.dim), dtype=torch.float64, device=self.device)
        C.check(self._lib.sipdg_quad_points(self._h, _ptr(xq), _ptr(xb), _stream_ptr(stream, self._dev)))
        return xq, xb[: self.n_boundary_points]

    def load_vector(self, s: torch.Tensor, g: torch.Tensor, stream=None) -> torch.Tensor:
        self._vec(s, torch.float64, n=self.n_volume_points, name="s")
        if self.n_boundary_points:
            self._vec(g, torch.float64, n=self.n_boundary_points, name="g")
        b = torch.empty(self.n_dofs, dtype=torch.float64, device=self.device)
        C.check(self._lib.sipdg_load_vector(self._h, _ptr(s), _ptr(g) if self.n_boundary_points else None,
                                            _ptr(b), _stream_ptr(stream, self._dev)))
        return b

    def rhs(self, source, dirichlet) -> torch.Tensor:
        """Load vector from callables of the physical coordinates."""
        xq, xb = self.quad_points()
        s = source(xq).contiguous()
        g = dirichlet(xb).contiguous() if self.n_boundary_points else torch.zeros(1, dtype=torch.float64, device=self.device)
        return self.load_vector(s, g)

    def gmres_solve(self, b: torch.Tensor, tol: float = 1e-10, restart: int = 30, maxit: int = 100000,
                    precond: bool = True, raise_on_fail: bool = True, stream=None):
        """Restarted GMRES for A x = b (FP64, x from zero) with the current
        interface flux; the point-to-point flux needs it (nonsymmetric A)."""
        self._vec(b, torch.float64, name="b")
        x = torch.empty_like(b)
        o = C.GmresOpts()
        self._lib.sipdg_gmres_default_opts(ctypes.byref(o))
        o.tol, o.restart, o.maxit, o.precond = float(tol), int(restart), int(maxit), int(bool(precond))
        info = C.GmresInfo()
        rc = self._lib.sipdg_gmres_solve(self._h, _ptr(b), _ptr(x), ctypes.byref(o), ctypes.byref(info),
                                         _stream_ptr(stream, self._dev))
        out = {"iters": info.iters, "restarts": info.restarts, "converged": bool(info.converged),
               "rel_resid": info.rel_resid, "time_ms": info.time_ms}
        if rc != 0 and not (rc == -5 and not raise_on_fail):
            C.check(rc)
        return x, out

    def cg_solve(self, b: torch.Tensor, x: torch.Tensor | None = None, tol: float = 1e-10,
                 maxit: int = 20000, mode: str = "f64", inner_tol: float = 1e-4, ru_delta: float = 0.1,
                 precond: bool = True, graph_k: int = 10, max_outer: int = 50,
                 checkpoint=None, checkpoint_every: int = 0, x0: torch.Tensor | None = None,
                 stream=None, raise_on_fail: bool = True):
        """Solve A x = b.  Returns (x, info dict).  ``checkpoint(x, r, iter)``
        receives device tensors (views valid only during the call)."""
        self._vec(b, torch.float64, name="b")
        if x is None:
            x = torch.empty_like(b)
        self._vec(x, torch.float64, name="x")
        o = C.CgOpts()
        self._lib.sipdg_cg_default_opts(ctypes.byref(o))
        o.tol, o.maxit, o.inner_tol, o.ru_delta = float(tol), int(maxit), float(inner_tol), float(ru_delta)
        o.mode = {"f64": C.SIPDG_CG_F64, "f32_ir": C.SIPDG_CG_F32_IR, "f32_ru": C.SIPDG_CG_F32_RU}[mode]
        o.precond, o.graph_k, o.max_outer = int(precond), int(graph_k), int(max_outer)
        cb_keep = None
        if checkpoint is not None and checkpoint_every > 0:
            n = self.n_dofs

            def _cb(user, xp, rp, it):
                xs = _wrap_device(xp, n, self.device)
                rs = _wrap_device(rp, n, self.device)
                checkpoint(xs, rs, int(it))

            cb_keep = C.CKPT_FN(_cb)
            o.checkpoint = cb_keep
            o.checkpoint_every = int(checkpoint_every)
        if x0 is not None:
            self._vec(x0, torch.float64, name="x0")
            x.copy_(x0)
            o.x0_given = 1
        info = C.CgInfo()
        rc = self._lib.sipdg_cg_solve(self._h, _ptr(b), _ptr(x), ctypes.byref(o), ctypes.byref(info),
                                      _stream_ptr(stream, self._dev))
        out = {"iters": info.iters, "outer_iters": info.outer_iters, "converged": bool(info.converged),
               "rel_resid": info.rel_resid, "time_ms": info.time_ms, "status": rc}
        if raise_on_fail:
            C.check(rc)
        del cb_keep
        return x, out


def _wrap_device(ptr, n, device):
    """A torch view of library-owned device memory (valid during a callback)."""
    # Copy to a fresh tensor: simplest safe way to expose the memory.
    out = torch.empty(n, dtype=torch.float64, device=device)
    rt = ctypes.CDLL("libamdhip64.so")
    rt.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    rt.hipMemcpy.restype = ctypes.c_int
    rc = rt.hipMemcpy(ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ptr), n * 8, 3)
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed ({rc})")
    return out
