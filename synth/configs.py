"""The five workloads of the operator, as seeded recipes.

Seeds are integers: mesh perturbation ``1000+k``, orders ``2000+k``, lambda
``3000+k``, coefficient vector ``4000+k`` for workload ``k`` (1-based).

1. 2-D ``[0,1]^2``, 4x4 quads, h=1/4, p=3 everywhere, lambda=1.
2. 2-D 64x64, checkerboard orders: p=4 where ``i+j`` is even, 5 where odd,
   so every interior face joins orders 4 and 5; lambda=1.
3. 3-D 32^3 hexes, p ~ U{3..6} per element, lambda=10.
4. 64 independent 3-D problems, problem i is an ``n_i^3`` hex mesh with
   ``n_i ~ U{8..24}``, one order ``p_i ~ U{2..7}`` and ``lambda_i`` log-uniform
   on ``[0.1, 100]`` per problem (drawn from seed 2004 in that order), mesh
   seed ``100400 + i``.
5. 3-D 24^3 hexes, p ~ U{3..5} per element, lambda_e log-uniform on [1, 10]
   per element, sigma=1.

All meshes perturb interior vertices by ``U[-0.1h, 0.1h]`` per coordinate.
"""

from __future__ import annotations

import numpy as np

from .meshes import Mesh, structured_mesh, rotate_elements

WORKLOADS = {
    1: "2-D 4x4 quads, p=3, lambda=1",
    2: "2-D 64x64 quads, checkerboard p in {4,5}, lambda=1",
    3: "3-D 32^3 hexes, p~U{3..6}, lambda=10",
    4: "64 3-D hex problems n~U{8..24}, p~U{2..7}, lambda log-U[0.1,100]",
    5: "3-D 24^3 hexes, p~U{3..5}, lambda_e log-U[1,10]",
}


def _checkerboard(N: int, even: int, odd: int) -> np.ndarray:
    i = np.arange(N)
    ii, jj = np.meshgrid(i, i, indexing="xy")  # jj rows (y), ii cols (x)
    par = (ii + jj) % 2
    return np.where(par == 0, even, odd).reshape(-1).astype(np.int32)


def workload(k: int, N: int | None = None):
    """Return the mesh (or list of meshes for workload 4) of workload ``k``.

    ``N`` overrides the lattice size (used to build the same recipe at a
    size the oracle finishes quickly)."""
    if k == 1:
        n = N or 4
        return structured_mesh(2, n, 0.1, seed=1001, order=3, lam=1.0)
    if k == 2:
        n = N or 64
        m = structured_mesh(2, n, 0.1, seed=1002, order=4, lam=1.0)
        m.order = _checkerboard(n, 4, 5)
        return m
    if k == 3:
        n = N or 32
        m = structured_mesh(3, n, 0.1, seed=1003, order=3, lam=10.0)
        rng = np.random.default_rng(2003)
        m.order = rng.integers(3, 7, size=m.n_elems).astype(np.int32)
        return m
    if k == 4:
        rng = np.random.default_rng(2004)
        nprob = 64
        ns = rng.integers(8, 25, size=nprob)
        ps = rng.integers(2, 8, size=nprob)
        lams = 10.0 ** rng.uniform(-1.0, 2.0, size=nprob)
        meshes = []
        for i in range(nprob):
            n = int(ns[i]) if N is None else min(int(ns[i]), N)
            m = structured_mesh(3, n, 0.1, seed=100400 + i, order=int(ps[i]),
                                lam=float(lams[i]))
            meshes.append(m)
        return meshes
    if k == 5:
        n = N or 24
        m = structured_mesh(3, n, 0.1, seed=1005, order=3, lam=1.0)
        rng = np.random.default_rng(2005)
        m.order = rng.integers(3, 6, size=m.n_elems).astype(np.int32)
        rl = np.random.default_rng(3005)
        m.lam = 10.0 ** rl.uniform(0.0, 1.0, size=m.n_elems)
        return m
    raise ValueError(f"unknown workload {k}")


def small_mesh(dim: int, N: int, orders, seed: int = 7, lam=1.0, perturb: float = 0.1,
               rotate: bool = False, rot_seed: int = 11, sigma: float = 1.0) -> Mesh:
    """A small perturbed mesh with given orders (scalar, array, or
    ``('random', lo, hi)`` drawn from ``seed+1``) for tests."""
    m = structured_mesh(dim, N, perturb, seed=seed, order=1, lam=lam, sigma=sigma)
    if isinstance(orders, tuple) and orders and orders[0] == "random":
        rng = np.random.default_rng(seed + 1)
        m.order = rng.integers(orders[1], orders[2] + 1, size=m.n_elems).astype(np.int32)
    elif isinstance(orders, tuple) and orders and orders[0] == "checker":
        if dim == 2:
            m.order = _checkerboard(N, orders[1], orders[2])
        else:
            e = np.arange(m.n_elems)
            ex, ey, ez = e % N, (e // N) % N, e // (N * N)
            m.order = np.where((ex + ey + ez) % 2 == 0, orders[1], orders[2]).astype(np.int32)
    else:
        m.order = np.broadcast_to(np.asarray(orders, dtype=np.int32), (m.n_elems,)).copy()
    if np.ndim(lam) == 0 and isinstance(lam, str):
        raise ValueError("lam must be numeric")
    if rotate:
        m = rotate_elements(m, rot_seed)
    return m
