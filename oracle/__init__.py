"""Oracle: plain FP64 CPU reference of the SIPG Helmholtz operator.

TEST INFRASTRUCTURE ONLY.  The product (the HIP library and its binding)
never imports this package; only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` do.  It shares no code, tables or
helpers with the HIP path: its quadrature nodes come from the Golub-Welsch
eigenvalue method, its face matching is a dictionary of sorted vertex ids
and its face maps are solved from matching corners.

The arithmetic lives in ``oracle.c`` (plain loops, physical gradients,
basis functions evaluated at every point).  This module adds:
  * GLL nodes/weights (Sec. 2.1 quadrature; nodes are the roots of P'_{n-1}
    plus the endpoints, weights 2 / (n (n-1) P_{n-1}(x)^2));
  * face matching and the owner-to-neighbour face-coordinate map of the
    shared trace (Sec. 3.3, shared trace space; Sec. 5.1, orientations);
  * Jacobi-preconditioned CG (the Krylov method the SIPG choice is made for,
    Sec. 2.2);
  * brute-force column assembly A[:, j] = A e_j for symmetry checks
    (Appendix A, the symmetry conditions on the face blocks).
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
OR_MAXN = 16
BASES = {"legendre": 0, "modal": 1}
_lib = None


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` (gcc, OpenMP); without
    ``force`` only when the library is missing or older than the source."""
    stale = (not os.path.exists(_LIB_PATH)
             or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC))
    if force or stale:
        cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c99", _SRC,
               "-o", _LIB_PATH + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class _OMesh(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("ne", ctypes.c_long),
        ("coords", ctypes.c_void_p),
        ("ev", ctypes.c_void_p),
        ("order", ctypes.c_void_p),
        ("lam", ctypes.c_void_p),
        ("dof_off", ctypes.c_void_p),
        ("h", ctypes.c_double),
        ("sigma", ctypes.c_double),
        ("nb", ctypes.c_void_p),
        ("nb_face", ctypes.c_void_p),
        ("owner", ctypes.c_void_p),
        ("amap", ctypes.c_void_p),
        ("gll_x", ctypes.c_void_p),
        ("gll_w", ctypes.c_void_p),
        ("basis", ctypes.c_int),
        ("vol_x", ctypes.c_void_p),
        ("vol_w", ctypes.c_void_p),
    ]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER(_OMesh)
        vp, lp = ctypes.c_void_p, ctypes.c_long
        lib.oracle_apply.argtypes = [P, vp, vp, vp, lp]
        lib.oracle_apply_p2p.argtypes = [P, vp, vp, vp, lp]
        lib.oracle_diagonal.argtypes = [P, vp]
        lib.oracle_points.argtypes = [P, vp, vp, vp, vp]
        lib.oracle_rhs.argtypes = [P, vp, vp, vp]
        lib.oracle_param_grad.argtypes = [P, vp, vp, vp, vp]
        lib.oracle_sample.argtypes = [P, vp, ctypes.c_int, vp, vp, vp, vp, vp]
        lib.oracle_min_detj.argtypes = [P, vp]
        lib.oracle_face_moments.argtypes = [P, vp, vp]
        lib.oracle_num_threads.argtypes = []
        lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
        for f in (lib.oracle_apply, lib.oracle_apply_p2p, lib.oracle_diagonal, lib.oracle_points, lib.oracle_rhs,
                  lib.oracle_param_grad, lib.oracle_sample, lib.oracle_min_detj,
                  lib.oracle_face_moments, lib.oracle_num_threads, lib.oracle_set_num_threads):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> int:
    """Threads of the oracle's OpenMP loops from now on; returns the new count."""
    return int(_load().oracle_set_num_threads(int(n)))


# ---------------------------------------------------------------- quadrature

def gll(n: int):
    """Gauss-Lobatto-Legendre nodes and weights with ``n >= 2`` points.

    Interior nodes are the eigenvalues of the symmetric tridiagonal Jacobi
    matrix of the Jacobi(1,1) polynomials (whose roots are those of
    P'_{n-1}), off-diagonal sqrt(k(k+2) / ((2k+1)(2k+3))), k = 1..n-3."""
    if n < 2:
        raise ValueError("GLL needs n >= 2")
    m = n - 2
    if m > 0:
        k = np.arange(1, m, dtype=np.float64)
        off = np.sqrt(k * (k + 2.0) / ((2.0 * k + 1.0) * (2.0 * k + 3.0)))
        T = np.diag(off, 1) + np.diag(off, -1)
        inner = np.linalg.eigvalsh(T) if m > 1 else np.zeros(1)
    else:
        inner = np.zeros(0)
    x = np.concatenate([[-1.0], np.sort(inner), [1.0]])
    # symmetrise the computed nodes exactly
    x = 0.5 * (x - x[::-1])
    Pn = np.polynomial.legendre.legval(x, np.eye(n)[n - 1])
    w = 2.0 / (n * (n - 1) * Pn * Pn)
    w = 0.5 * (w + w[::-1])
    return x, w


def gauss_legendre(n: int):
    """Gauss-Legendre nodes and weights (NumPy's Golub-Welsch routine)."""
    return np.polynomial.legendre.leggauss(n)


def _tables(rule):
    X = np.zeros((OR_MAXN + 1, OR_MAXN))
    W = np.zeros((OR_MAXN + 1, OR_MAXN))
    for n in range(2, OR_MAXN + 1):
        x, w = rule(n)
        X[n, :n] = x
        W[n, :n] = w
    return X, W


_GLL_X, _GLL_W = _tables(gll)
_GL_X, _GL_W = _tables(gauss_legendre)
POINTS = {"gll": (_GLL_X, _GLL_W), "gl": (_GL_X, _GL_W)}


# ---------------------------------------------------------------- topology

def _face_corner_ids(ev_e: np.ndarray, dim: int, f: int):
    """Global vertex ids of the corners of local face f = 2k + (s>0), in the
    lexicographic order of the face coordinates (remaining directions in
    increasing order), and those corners' face coordinates in {-1,+1}."""
    k, side = f // 2, f % 2
    others = [a for a in range(dim) if a != k]
    ids, coords = [], []
    for c in range(2 ** (dim - 1)):
        bits = [0] * dim
        bits[k] = side
        t = []
        for j, a in enumerate(others):
            b = (c >> j) & 1
            bits[a] = b
            t.append(2 * b - 1)
        v = sum(bits[a] << a for a in range(dim))
        ids.append(int(ev_e[v]))
        coords.append(t)
    return ids, np.array(coords, dtype=np.int64)


class OracleMesh:
    """A mesh prepared for the oracle (neighbours, owners, face maps)."""

    def __init__(self, mesh, basis: str = "legendre", points: str = "gll"):
        self.mesh = mesh
        self.basis = basis
        self.vol_points = points
        vx, vw = POINTS[points]
        d = mesh.dim
        ne = mesh.n_elems
        nf = 2 * d
        self.dim = d
        self.coords = np.ascontiguousarray(mesh.coords, dtype=np.float64)
        self.ev = np.ascontiguousarray(mesh.elem_vertices, dtype=np.int64)
        self.order = np.ascontiguousarray(mesh.order, dtype=np.int32)
        self.lam = np.ascontiguousarray(mesh.lam, dtype=np.float64)
        self.dof_off = np.zeros(ne + 1, dtype=np.int64)
        np.cumsum((self.order.astype(np.int64) + 1) ** d, out=self.dof_off[1:])
        self.n_dofs = int(self.dof_off[-1])
        self.nb = -np.ones((ne, nf), dtype=np.int64)
        self.nb_face = -np.ones((ne, nf), dtype=np.int32)
        self.owner = np.zeros((ne, nf), dtype=np.int32)
        self.amap = np.zeros((ne, nf, 4), dtype=np.int32)
        faces = {}
        corner_cache = {}
        for e in range(ne):
            for f in range(nf):
                ids, tc = _face_corner_ids(self.ev[e], d, f)
                corner_cache[(e, f)] = (ids, tc)
                faces.setdefault(tuple(sorted(ids)), []).append((e, f))
        n_int = 0
        for key, lst in faces.items():
            if len(lst) == 1:
                e, f = lst[0]
                self.owner[e, f] = 1
                self.amap[e, f, :] = [1, 0, 0, 1]
                continue
            if len(lst) != 2:
                raise ValueError(f"face {key} shared by {len(lst)} elements")
            (e0, f0), (e1, f1) = sorted(lst)
            if e0 == e1:
                raise ValueError("element meets itself")
            ids0, t0 = corner_cache[(e0, f0)]
            ids1, t1 = corner_cache[(e1, f1)]
            # owner e0: find A with A t0[c] = t1[c'] whenever ids agree
            tgt = np.array([t1[ids1.index(g)] for g in ids0], dtype=np.float64)
            T = t0.astype(np.float64).T            # [(d-1), corners]
            Tt = tgt.T
            A = Tt @ T.T @ np.linalg.inv(T @ T.T)
            Ai = np.rint(A).astype(np.int64)
            if not np.array_equal(Ai @ t0.T, tgt.T.astype(np.int64)):
                raise ValueError("faces do not match by a symmetry of the square")
            flat = np.zeros(4, dtype=np.int32)
            flat[: (d - 1) ** 2] = Ai.reshape(-1)
            for (e, f, o, en, fn) in ((e0, f0, 1, e1, f1), (e1, f1, 0, e0, f0)):
                self.nb[e, f] = en
                self.nb_face[e, f] = fn
                self.owner[e, f] = o
                self.amap[e, f, :] = flat
            n_int += 1
        self.n_interior_faces = n_int
        self.n_boundary_faces = sum(1 for v in faces.values() if len(v) == 1)
        self._s = _OMesh(
            dim=d, ne=ne,
            coords=self.coords.ctypes.data, ev=self.ev.ctypes.data,
            order=self.order.ctypes.data, lam=self.lam.ctypes.data,
            dof_off=self.dof_off.ctypes.data, h=float(mesh.h), sigma=float(mesh.sigma),
            nb=self.nb.ctypes.data, nb_face=self.nb_face.ctypes.data,
            owner=self.owner.ctypes.data, amap=self.amap.ctypes.data,
            gll_x=_GLL_X.ctypes.data, gll_w=_GLL_W.ctypes.data,
            basis=BASES[basis], vol_x=vx.ctypes.data, vol_w=vw.ctypes.data)

    def set_lambda(self, lam):
        self.lam[:] = np.asarray(lam, dtype=np.float64)

    def set_sigma(self, sigma: float):
        self._s.sigma = float(sigma)

    @property
    def sigma(self):
        return self._s.sigma

    # ------------------------------------------------------------ operators
    def apply(self, x: np.ndarray, elems=None) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        assert x.shape == (self.n_dofs,)
        y = np.zeros(self.n_dofs)
        if elems is None:
            rc = _load().oracle_apply(ctypes.byref(self._s), x.ctypes.data, y.ctypes.data, None, 0)
        else:
            el = np.ascontiguousarray(elems, dtype=np.int64)
            rc = _load().oracle_apply(ctypes.byref(self._s), x.ctypes.data, y.ctypes.data,
                                      el.ctypes.data, len(el))
        if rc:
            raise MemoryError("oracle_apply")
        return y

    def apply_p2p(self, x: np.ndarray, elems=None) -> np.ndarray:
        """y = A x with point-to-point interpolation on interior faces
        (Sec. 3.3): each side integrates on its own face quadrature with the
        other side's value and gradient interpolated to it."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        assert x.shape == (self.n_dofs,)
        y = np.zeros(self.n_dofs)
        el = None if elems is None else np.ascontiguousarray(elems, dtype=np.int64)
        rc = _load().oracle_apply_p2p(ctypes.byref(self._s), x.ctypes.data, y.ctypes.data,
                                      None if el is None else el.ctypes.data, 0 if el is None else len(el))
        if rc:
            raise MemoryError("oracle_apply_p2p")
        return y

    def diagonal(self) -> np.ndarray:
        y = np.zeros(self.n_dofs)
        if _load().oracle_diagonal(ctypes.byref(self._s), y.ctypes.data):
            raise MemoryError("oracle_diagonal")
        return y

    def points(self):
        lib = _load()
        nq, nb = ctypes.c_long(0), ctypes.c_long(0)
        lib.oracle_points(ctypes.byref(self._s), None, None, ctypes.byref(nq), ctypes.byref(nb))
        xq = np.zeros((nq.value, self.dim))
        xb = np.zeros((nb.value, self.dim))
        lib.oracle_points(ctypes.byref(self._s), xq.ctypes.data, xb.ctypes.data, None, None)
        return xq, xb

    def rhs(self, s_q: np.ndarray, g_b: np.ndarray) -> np.ndarray:
        s_q = np.ascontiguousarray(s_q, dtype=np.float64)
        g_b = np.ascontiguousarray(g_b, dtype=np.float64)
        b = np.zeros(self.n_dofs)
        if _load().oracle_rhs(ctypes.byref(self._s), s_q.ctypes.data, g_b.ctypes.data,
                              b.ctypes.data):
            raise MemoryError("oracle_rhs")
        return b

    def rhs_from(self, source, dirichlet) -> np.ndarray:
        xq, xb = self.points()
        return self.rhs(source(xq), dirichlet(xb) if len(xb) else np.zeros(0))

    def param_grad(self, a: np.ndarray, b: np.ndarray):
        a = np.ascontiguousarray(a, dtype=np.float64)
        b = np.ascontiguousarray(b, dtype=np.float64)
        ne = self.mesh.n_elems
        dl = np.zeros(ne)
        ds = np.zeros(ne)
        if _load().oracle_param_grad(ctypes.byref(self._s), a.ctypes.data, b.ctypes.data,
                                     dl.ctypes.data, ds.ctypes.data):
            raise MemoryError("oracle_param_grad")
        return dl, float(ds.sum())

    def sample(self, x: np.ndarray, extra: int = 4):
        """u_h, physical points and w|J| at Gauss-Legendre points with p+extra
        nodes per direction (for L2 errors)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        stride = OR_MAXN + 4
        pmax = int(self.order.max())
        RX = np.zeros((pmax + 1, stride))
        RW = np.zeros((pmax + 1, stride))
        for p in range(pmax + 1):
            gx, gw = gauss_legendre(p + extra)
            RX[p, : p + extra] = gx
            RW[p, : p + extra] = gw
        npts = int(((self.order.astype(np.int64) + extra) ** self.dim).sum())
        xyz = np.zeros((npts, self.dim))
        wd = np.zeros(npts)
        uv = np.zeros(npts)
        _load().oracle_sample(ctypes.byref(self._s), x.ctypes.data, extra, RX.ctypes.data,
                              RW.ctypes.data, xyz.ctypes.data, wd.ctypes.data, uv.ctypes.data)
        return xyz, wd, uv

    def l2_error(self, x: np.ndarray, exact) -> float:
        xyz, wd, uv = self.sample(x)
        return float(np.sqrt(np.sum(wd * (uv - exact(xyz)) ** 2)))

    def min_detj(self) -> np.ndarray:
        out = np.zeros(self.mesh.n_elems)
        _load().oracle_min_detj(ctypes.byref(self._s), out.ctypes.data)
        return out

    def face_moments(self):
        ne, d = self.mesh.n_elems, self.dim
        sn = np.zeros((ne, 2 * d, d))
        ar = np.zeros((ne, 2 * d))
        _load().oracle_face_moments(ctypes.byref(self._s), sn.ctypes.data, ar.ctypes.data)
        return sn, ar

    # ------------------------------------------------------------ assembly / solve
    def assemble(self, flux: str = "shared") -> np.ndarray:
        """Brute force: column j is A e_j (flux "shared" or "p2p")."""
        n = self.n_dofs
        A = np.zeros((n, n))
        e = np.zeros(n)
        f = self.apply if flux == "shared" else self.apply_p2p
        for j in range(n):
            e[j] = 1.0
            A[:, j] = f(e)
            e[j] = 0.0
        return A

    def cg(self, b: np.ndarray, tol: float = 1e-10, maxit: int = 100000, precond: bool = True):
        """Jacobi-preconditioned CG from x0 = 0, stop when ||r||/||b|| <= tol."""
        dinv = 1.0 / self.diagonal() if precond else np.ones(self.n_dofs)
        x = np.zeros(self.n_dofs)
        r = b.copy()
        z = dinv * r
        p = z.copy()
        rho = float(r @ z)
        nb = float(np.linalg.norm(b))
        it = 0
        if nb == 0.0:
            return x, 0, 0.0
        while it < maxit:
            q = self.apply(p)
            pq = float(p @ q)
            if pq <= 0.0:
                raise FloatingPointError("CG breakdown: p^T A p <= 0")
            alpha = rho / pq
            x += alpha * p
            r -= alpha * q
            it += 1
            rel = float(np.linalg.norm(r)) / nb
            if rel <= tol:
                break
            z = dinv * r
            rho_new = float(r @ z)
            p = z + (rho_new / rho) * p
            rho = rho_new
        return x, it, float(np.linalg.norm(b - self.apply(x))) / nb


def prepare(mesh, basis: str = "legendre", points: str = "gll") -> OracleMesh:
    """basis: "legendre" (orthogonal) or "modal" (modified C0, Table 1).
    points: the operator's volume quadrature, "gll" (p + 2 Gauss-Lobatto
    points per direction) or "gl" (p + 2 Gauss points, which leave out the
    element boundary, Sec. 3.2); the faces use the trace's GLL points
    either way."""
    return OracleMesh(mesh, basis, points)
