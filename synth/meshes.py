"""Structured quad/hex meshes treated as unstructured, with seeded perturbation.

Conventions (shared by every consumer, they are part of the input format):

* ``coords`` is ``[n_vertices, dim]`` float64; vertices of an ``(N+1)^dim``
  lattice on ``[0,1]^dim`` are numbered with x fastest.
* ``elem_vertices`` is ``[n_elems, 2^dim]`` int64; the corner with reference
  coordinates ``(c_1, .., c_d)`` in ``{-1,+1}^d`` is stored at position
  ``sum_k b_k 2^k`` with ``b_k = (c_k + 1) / 2`` (lexicographic, first
  reference direction fastest).  Elements of the lattice are numbered with x
  fastest.
* Orders ``p_e >= 1`` per element, Helmholtz coefficients ``lambda_e >= 0``.

The mesh is treated as a general unstructured mesh by every consumer: nothing
downstream may assume the lattice structure.
"""

from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Mesh:
    dim: int
    coords: np.ndarray          # [nv, dim] float64
    elem_vertices: np.ndarray   # [ne, 2^dim] int64
    order: np.ndarray           # [ne] int32
    lam: np.ndarray             # [ne] float64
    h: float                    # nominal mesh size used in the penalty
    sigma: float = 1.0          # penalty scale
    meta: dict = field(default_factory=dict)

    @property
    def n_elems(self) -> int:
        return int(self.elem_vertices.shape[0])

    @property
    def n_vertices(self) -> int:
        return int(self.coords.shape[0])

    def dofs_per_elem(self) -> np.ndarray:
        return (self.order.astype(np.int64) + 1) ** self.dim

    def dof_offsets(self) -> np.ndarray:
        """Natural layout: element after element, modes lexicographic."""
        off = np.zeros(self.n_elems + 1, dtype=np.int64)
        np.cumsum(self.dofs_per_elem(), out=off[1:])
        return off

    @property
    def n_dofs(self) -> int:
        return int(self.dofs_per_elem().sum())


def num_dofs(order: np.ndarray, dim: int) -> int:
    return int(((np.asarray(order, dtype=np.int64) + 1) ** dim).sum())


def structured_mesh(dim: int, N: int, perturb: float = 0.1, seed: int | None = None,
                    order=3, lam=1.0, sigma: float = 1.0) -> Mesh:
    """``N^dim`` lattice on ``[0,1]^dim``; interior vertices moved by
    ``U[-perturb*h, +perturb*h]`` per coordinate (numpy PCG64 ``seed``; the
    draw covers every vertex in lexicographic order times dims, boundary rows
    are then reset to zero so the boundary stays the unit square/cube)."""
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    h = 1.0 / N
    nv1 = N + 1
    axes = [np.arange(nv1, dtype=np.float64) * h for _ in range(dim)]
    grids = np.meshgrid(*axes, indexing="ij")
    # x fastest: vertex id = i + nv1*j (+ nv1^2*k)
    coords = np.stack([g.transpose().reshape(-1) for g in grids], axis=1)
    coords = np.ascontiguousarray(coords)
    if perturb != 0.0:
        rng = np.random.default_rng(seed)
        d = rng.uniform(-perturb * h, perturb * h, size=coords.shape)
        idx = np.stack(np.meshgrid(*[np.arange(nv1)] * dim, indexing="ij"), axis=-1)
        idx = idx.transpose(*reversed(range(dim)), dim).reshape(-1, dim)
        interior = np.all((idx > 0) & (idx < N), axis=1)
        coords = coords + d * interior[:, None]
        # snap exact lattice values on the boundary
    ne = N ** dim
    ev = np.zeros((ne, 2 ** dim), dtype=np.int64)
    e = 0
    if dim == 2:
        for ey in range(N):
            for ex in range(N):
                for c in range(4):
                    cx, cy = c & 1, (c >> 1) & 1
                    ev[e, c] = (ex + cx) + nv1 * (ey + cy)
                e += 1
    else:
        ex_, ey_, ez_ = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
        ex_ = ex_.transpose(2, 1, 0).reshape(-1)
        ey_ = ey_.transpose(2, 1, 0).reshape(-1)
        ez_ = ez_.transpose(2, 1, 0).reshape(-1)
        for c in range(8):
            cx, cy, cz = c & 1, (c >> 1) & 1, (c >> 2) & 1
            ev[:, c] = (ex_ + cx) + nv1 * (ey_ + cy) + nv1 * nv1 * (ez_ + cz)
    order_arr = np.broadcast_to(np.asarray(order, dtype=np.int32), (ne,)).copy()
    lam_arr = np.broadcast_to(np.asarray(lam, dtype=np.float64), (ne,)).copy()
    return Mesh(dim=dim, coords=coords, elem_vertices=ev, order=order_arr, lam=lam_arr,
                h=h, sigma=sigma, meta={"N": N, "perturb": perturb, "seed": seed})


def cube_rotations(dim: int) -> list[np.ndarray]:
    """Signed permutation matrices with determinant +1 (the rotations of the
    reference square, 4, or cube, 24), identity first."""
    mats = []
    for perm in itertools.permutations(range(dim)):
        for signs in itertools.product((1, -1), repeat=dim):
            R = np.zeros((dim, dim), dtype=np.int64)
            for r, (c, s) in enumerate(zip(perm, signs)):
                R[r, c] = s
            if round(np.linalg.det(R)) == 1:
                mats.append(R)
    mats.sort(key=lambda R: (not np.array_equal(R, np.eye(dim, dtype=np.int64)),))
    return mats


def rotate_elements(mesh: Mesh, seed: int, fraction: float = 1.0) -> Mesh:
    """Relabel each element's local corners by a random rotation of the
    reference element, so neighbouring faces meet in every orientation.
    The new map is ``F_new(xi) = F_old(R xi)``; ``det R = +1`` keeps the
    Jacobian positive.  Geometry and the discrete space are unchanged; only
    local numbering (hence face orientations) changes."""
    dim = mesh.dim
    rots = cube_rotations(dim)
    rng = np.random.default_rng(seed)
    pick = rng.integers(0, len(rots), size=mesh.n_elems)
    if fraction < 1.0:
        keep = rng.uniform(size=mesh.n_elems) >= fraction
        pick[keep] = 0
    corners = np.array([[2 * ((c >> k) & 1) - 1 for k in range(dim)]
                        for c in range(2 ** dim)], dtype=np.int64)

    def corner_index(xi):
        return int(sum(((int(xi[k]) + 1) // 2) << k for k in range(dim)))

    tables = []
    for R in rots:
        tables.append(np.array([corner_index(R @ corners[c]) for c in range(2 ** dim)],
                               dtype=np.int64))
    ev = mesh.elem_vertices
    new_ev = np.empty_like(ev)
    for e in range(mesh.n_elems):
        new_ev[e] = ev[e, tables[pick[e]]]
    out = Mesh(dim=dim, coords=mesh.coords.copy(), elem_vertices=new_ev,
               order=mesh.order.copy(), lam=mesh.lam.copy(), h=mesh.h,
               sigma=mesh.sigma, meta=dict(mesh.meta))
    out.meta["rotation_seed"] = seed
    return out


def random_coefficients(mesh: Mesh, seed: int) -> np.ndarray:
    """``N(0,1)`` i.i.d. float64 coefficients in the natural layout."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(mesh.n_dofs)


def affine_mesh(dim: int, N: int, seed: int, order=2, lam=1.0, sigma: float = 1.0,
                deform_frac: float = 0.0) -> Mesh:
    """Every element a parallelogram/parallelepiped: a tensor lattice with
    seeded non-uniform spacing per axis mapped by one global linear map with
    positive determinant.  Used where an exact polynomial reproduction is
    expected (constant Jacobian per element).  ``deform_frac`` > 0 moves that
    fraction of the interior vertices (drawn after the map, same generator) by
    ``U[-0.1h, 0.1h]`` per coordinate before the map, so that the elements
    around them are deformed and the rest stay affine."""
    rng = np.random.default_rng(seed)
    axes = []
    for _ in range(dim):
        w = rng.uniform(0.6, 1.4, size=N)
        axes.append(np.concatenate([[0.0], np.cumsum(w) / w.sum()]))
    base = structured_mesh(dim, N, 0.0, order=order, lam=lam, sigma=sigma)
    nv1 = N + 1
    ids = np.arange(base.n_vertices)
    lat = np.stack([(ids // nv1 ** k) % nv1 for k in range(dim)], axis=1)
    X = np.stack([axes[k][lat[:, k]] for k in range(dim)], axis=1)
    B = np.eye(dim) + rng.uniform(-0.25, 0.25, size=(dim, dim))
    if np.linalg.det(B) < 0:
        B[0] *= -1.0
    if deform_frac > 0.0:
        interior = np.all((lat > 0) & (lat < N), axis=1)
        moved = interior & (rng.uniform(size=len(ids)) < deform_frac)
        h = 1.0 / N
        X = X + rng.uniform(-0.1 * h, 0.1 * h, size=X.shape) * moved[:, None]
    base.coords = np.ascontiguousarray(X @ B.T)
    base.meta.update({"affine": deform_frac == 0.0, "seed": seed})
    return base
