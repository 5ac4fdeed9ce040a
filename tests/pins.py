"""Test-side constructions that pin the oracle to mathematics other than
itself: a hand-assembled 1-D SIPG matrix (for the tensor-product identity on
uniform meshes), L2 projection of a global function onto each element's
Legendre expansion (for patch and polynomial-exactness tests), and the
Kronecker index map.  Written independently of ``oracle/`` (numpy's own
Legendre and Gauss-Legendre routines, exact integration)."""

from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as L


def sipg_1d(N: int, p: int, h: float, sigma: float):
    """1-D SIPG on N equal elements of width h with Legendre modes of order p:
    returns (M1, K1) where M1 is the mass matrix and K1 the SIPG stiffness:
    volume (v', u') plus, at interior points, -{v'}[u] - [v]{u'} + tau [u][v]
    and, at the two boundary points (mirror exterior value),
    -v' n u - v u' n + 2 tau u v, with tau = sigma 2 (p+1)^2 / h."""
    NP = p + 1
    I = np.eye(NP)
    gx, gw = L.leggauss(p + 3)
    V = np.array([L.legval(gx, I[i]) for i in range(NP)])
    dV = np.array([L.legval(gx, L.legder(I[i])) for i in range(NP)])
    Mref = (V * gw) @ V.T
    Kref = (dV * gw) @ dV.T
    M1 = np.kron(np.eye(N), 0.5 * h * Mref)
    K = np.kron(np.eye(N), 2.0 / h * Kref)
    vp = np.array([L.legval(1.0, I[i]) for i in range(NP)])
    vm = np.array([L.legval(-1.0, I[i]) for i in range(NP)])
    dp = np.array([L.legval(1.0, L.legder(I[i])) for i in range(NP)]) * 2.0 / h
    dm = np.array([L.legval(-1.0, L.legder(I[i])) for i in range(NP)]) * 2.0 / h
    tau = sigma * 2.0 * (p + 1) ** 2 / h
    n = N * NP
    for f in range(N - 1):
        eL, eR = f, f + 1
        J = np.zeros(n)
        J[eL * NP:(eL + 1) * NP] = vp
        J[eR * NP:(eR + 1) * NP] = -vm
        Dv = np.zeros(n)
        Dv[eL * NP:(eL + 1) * NP] = 0.5 * dp
        Dv[eR * NP:(eR + 1) * NP] = 0.5 * dm
        K += -np.outer(Dv, J) - np.outer(J, Dv) + tau * np.outer(J, J)
    for (e, val, der, nrm) in ((0, vm, dm, -1.0), (N - 1, vp, dp, 1.0)):
        v = np.zeros(n)
        v[e * NP:(e + 1) * NP] = val
        dv = np.zeros(n)
        dv[e * NP:(e + 1) * NP] = der * nrm
        K += -np.outer(dv, v) - np.outer(v, dv) + 2.0 * tau * np.outer(v, v)
    return M1, K


def tensor_operator(dim: int, N: int, p: int, h: float, sigma: float, lam: float):
    """sum_k M1 x .. x K1 (k-th slot) x .. x M1 + lam M1^{x d}, slow index = last direction."""
    M1, K1 = sipg_1d(N, p, h, sigma)
    if dim == 2:
        return np.kron(M1, K1) + np.kron(K1, M1) + lam * np.kron(M1, M1)
    return (np.kron(M1, np.kron(M1, K1)) + np.kron(M1, np.kron(K1, M1))
            + np.kron(K1, np.kron(M1, M1)) + lam * np.kron(M1, np.kron(M1, M1)))


def kron_permutation(dim: int, N: int, p: int) -> np.ndarray:
    """Natural (element, mode) index -> Kronecker (x-index fastest) index on
    a lattice mesh with elements numbered x fastest."""
    NP = p + 1
    nm = NP ** dim
    perm = np.zeros(N ** dim * nm, dtype=np.int64)
    for e in range(N ** dim):
        ex, ey, ez = e % N, (e // N) % N, e // (N * N)
        for i in range(nm):
            i1, i2, i3 = i % NP, (i // NP) % NP, i // (NP * NP)
            gxi, gyi, gzi = ex * NP + i1, ey * NP + i2, ez * NP + i3
            if dim == 2:
                t = gyi * (N * NP) + gxi
            else:
                t = (gzi * (N * NP) + gyi) * (N * NP) + gxi
            perm[e * nm + i] = t
    return perm


def multilinear_map(X: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """x(xi) for corner coordinates X [2^d, d], reference points xi [m, d]."""
    d = X.shape[1]
    out = np.zeros((xi.shape[0], d))
    for v in range(2 ** d):
        w = np.ones(xi.shape[0])
        for k in range(d):
            b = (v >> k) & 1
            w = w * (0.5 * (1 + xi[:, k]) if b else 0.5 * (1 - xi[:, k]))
        out += w[:, None] * X[v][None, :]
    return out


def project(mesh, func, extra: int = 6) -> np.ndarray:
    """Legendre coefficients of the L2 projection (in reference coordinates,
    Gauss-Legendre with p+extra points) of func(x) on every element.  Exact
    when func composed with the element map lies in the element space."""
    d = mesh.dim
    out = []
    for e in range(mesh.n_elems):
        p = int(mesh.order[e])
        NP = p + 1
        gx, gw = L.leggauss(p + extra)
        grids = np.meshgrid(*([gx] * d), indexing="ij")
        xi = np.stack([g.reshape(-1) for g in grids], axis=1)
        wg = np.meshgrid(*([gw] * d), indexing="ij")
        w = np.prod(np.stack([g.reshape(-1) for g in wg], axis=1), axis=1)
        X = mesh.coords[mesh.elem_vertices[e]]
        f = func(multilinear_map(X, xi))
        Pv = [np.array([L.legval(xi[:, k], np.eye(NP)[i]) for i in range(NP)]) for k in range(d)]
        coef = np.zeros(NP ** d)
        for m in range(NP ** d):
            idx = [(m // NP ** k) % NP for k in range(d)]
            phi = np.ones(xi.shape[0])
            norm = 1.0
            for k in range(d):
                phi = phi * Pv[k][idx[k]]
                norm *= (2 * idx[k] + 1) / 2.0
            coef[m] = norm * np.sum(w * phi * f)
        out.append(coef)
    return np.concatenate(out)


def interior_elements(om) -> list[int]:
    return [e for e in range(om.mesh.n_elems) if (om.nb[e] >= 0).all()]
