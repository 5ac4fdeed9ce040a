"""Pins of the oracle's Gauss-Legendre volume quadrature (points="gl").

Gauss points leave out the element boundary (Sec. 3.2: such point sets take
their trace values from the coefficients, TracePhysEval), so only the volume
integrals change; the faces keep the shared trace's GLL points.  Pins that do
not rest on the oracle's own arithmetic:
  * the n-point table integrates x^k exactly for k <= 2n - 1 (closed form
    2 / (k + 1) for even k, 0 for odd k) and misses x^(2n);
  * affine elements: every volume integrand is a polynomial of degree <= 2p
    per direction, which both (p + 2)-point rules integrate exactly, so the
    Gauss and GLL operators agree to rounding;
  * trilinear (deformed) elements: lambda phi_i phi_j |J| has degree 2p + 2
    per direction, exact with p + 2 Gauss points (up to 2p + 3) but not with
    p + 2 GLL points (up to 2p + 1): the lambda part of the Gauss operator is
    the mass matrix computed here by brute force with a 20-point rule, the
    GLL operator's is not;
  * the Gauss operator is symmetric positive definite (brute-force assembly).
"""

from __future__ import annotations

import numpy as np
import pytest

import synth

oracle = pytest.importorskip("oracle")


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("n", list(range(3, 11)))
def test_gauss_table_exactness(n):
    X, W = oracle.POINTS["gl"]
    x, w = X[n, :n], W[n, :n]
    for k in range(2 * n):
        exact = 2.0 / (k + 1) if k % 2 == 0 else 0.0
        assert abs(float(w @ x ** k) - exact) <= 1e-14, (n, k)
    assert abs(float(w @ x ** (2 * n)) - 2.0 / (2 * n + 1)) >= 1e-6
    assert np.all(np.abs(x) < 1.0)   # no endpoint


def _ragged_affine(N, seed, lo, hi):
    m = synth.affine_mesh(3, N, seed=seed, order=1, lam=1.3)
    m.order = np.random.default_rng(seed).integers(lo, hi + 1, m.n_elems).astype(np.int32)
    return synth.rotate_elements(m, seed + 1)


@pytest.mark.parametrize("basis", ["legendre", "modal"])
def test_affine_gauss_equals_gll(basis):
    m = _ragged_affine(3, 4101, 1, 5)
    x = synth.random_coefficients(m, 4102)
    yl = oracle.prepare(m, basis).apply(x)
    yg = oracle.prepare(m, basis, points="gl").apply(x)
    assert rel(yg, yl) <= 1e-12


def _trilinear(corners, xi):
    """Map and Jacobian of a hexahedron with lexicographic corners at the
    reference points xi [..., 3]."""
    s = np.array([[(v >> a) & 1 for a in range(3)] for v in range(8)], dtype=np.float64) * 2 - 1
    f = 0.5 * (1 + s[None, :, :] * xi[:, None, :])          # [q, v, a]
    shape = f.prod(axis=2)                                    # [q, v]
    J = np.zeros((len(xi), 3, 3))
    for b in range(3):
        g = np.ones_like(shape)
        for a in range(3):
            g = g * (0.5 * s[None, :, a] if a == b else f[:, :, a])
        J[:, :, b] = g @ corners                              # dx_c / dxi_b
    return shape @ corners, J


def _mass_brute(corners, p, nq=20):
    z, wz = np.polynomial.legendre.leggauss(nq)
    Z = np.stack(np.meshgrid(z, z, z, indexing="ij"), axis=-1).reshape(-1, 3)
    Wq = np.einsum("i,j,k->ijk", wz, wz, wz).reshape(-1)
    _, J = _trilinear(corners, Z)
    det = np.linalg.det(J)
    L = [np.polynomial.legendre.legvander(Z[:, a], p) for a in range(3)]   # [q, p+1]
    # modes lexicographic, first direction fastest
    phi = np.einsum("qi,qj,qk->qkji", L[0], L[1], L[2]).reshape(len(Z), -1)
    return (phi * (Wq * det)[:, None]).T @ phi


def test_deformed_mass_exact_with_gauss_only():
    # 3 x 3 x 3: the middle element has all eight corners moved (an element
    # with one moved corner has a multilinear |J|, which GLL integrates too)
    m = synth.small_mesh(3, 3, ("random", 1, 3), seed=4103, rotate=True, lam=1.0)
    x = synth.random_coefficients(m, 4104)
    lam = np.random.default_rng(4105).uniform(0.5, 2.0, m.n_elems)
    diff = {}
    for pts in ("gl", "gll"):
        m.lam = lam.copy()   # the oracle keeps (and set_lambda writes) this array
        om = oracle.prepare(m, points=pts)
        y1 = om.apply(x)
        om.set_lambda(np.zeros(m.n_elems))
        diff[pts] = y1 - om.apply(x)
    off = np.concatenate([[0], np.cumsum((m.order.astype(np.int64) + 1) ** 3)])
    worst_gl, worst_gll = 0.0, 0.0
    for e in range(m.n_elems):
        corners = m.coords[m.elem_vertices[e]]
        M = _mass_brute(corners, int(m.order[e]))
        ref = lam[e] * (M @ x[off[e]:off[e + 1]])
        worst_gl = max(worst_gl, rel(diff["gl"][off[e]:off[e + 1]], ref))
        worst_gll = max(worst_gll, rel(diff["gll"][off[e]:off[e + 1]], ref))
    print(f"mass part: gauss {worst_gl:.2e}, gll {worst_gll:.2e}")
    assert worst_gl <= 5e-12
    assert worst_gll >= 1e-8


def test_gauss_operator_spd():
    m = synth.small_mesh(3, 2, ("random", 1, 3), seed=4106, rotate=True, lam=0.7)
    A = oracle.prepare(m, points="gl").assemble()
    assert np.abs(A - A.T).max() <= 1e-12 * np.abs(A).max()
    assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0.0
    Al = oracle.prepare(m).assemble()
    assert np.abs(A - Al).max() >= 1e-8 * np.abs(A).max()   # a different operator on deformed elements
