"""Pins of the oracle's modified C0 modal basis (Table 1 "Modal";
Karniadakis & Sherwin): psi_0 = (1-x)/2, psi_1 = (1+x)/2 and the bubbles
(1-x)/2 (1+x)/2 P^(1,1)_{i-2}(x).

The modal and Legendre bases span the same polynomials on every element, so
with T the block-diagonal change of basis (Legendre coefficients of each
modal function, tensor products per element) A_modal = T^T A_legendre T for
either interface flux.  T is built here from the definition with SciPy's
Jacobi polynomials and a least-squares Legendre fit, not from the oracle, and
A_legendre is pinned independently; a wrong mode, derivative or ordering in
the oracle's modal basis breaks the identity."""

from __future__ import annotations

import numpy as np
import pytest
from numpy.polynomial import legendre as L
from scipy.special import eval_jacobi

import synth


def _t1(p):
    """[p+1][p+1]: column i = Legendre coefficients of modal mode i."""
    x = np.cos(np.linspace(0.0, np.pi, 4 * (p + 2)))
    cols = []
    for i in range(p + 1):
        if i == 0:
            v = 0.5 * (1 - x)
        elif i == 1:
            v = 0.5 * (1 + x)
        else:
            v = 0.25 * (1 - x) * (1 + x) * eval_jacobi(i - 2, 1, 1, x)
        cols.append(L.legfit(x, v, p))
    return np.array(cols).T


def _T(mesh):
    blocks = []
    for p in mesh.order:
        t = _t1(int(p))
        blk = t
        for _ in range(mesh.dim - 1):
            blk = np.kron(t, blk)
        blocks.append(blk)
    n = sum(b.shape[0] for b in blocks)
    T = np.zeros((n, n))
    o = 0
    for b in blocks:
        k = b.shape[0]
        T[o:o + k, o:o + k] = b
        o += k
    return T


CASES = [
    (2, lambda: synth.small_mesh(2, 4, ("random", 1, 5), seed=91, rotate=True, lam=1.3)),
    (3, lambda: synth.small_mesh(3, 2, ("random", 1, 4), seed=92, rotate=True, lam=0.7)),
]


@pytest.mark.parametrize("dim,make", CASES)
def test_change_of_basis(oracle_lib, dim, make):
    m = make()
    T = _T(m)
    leg = oracle_lib.prepare(m, "legendre")
    mod = oracle_lib.prepare(m, "modal")
    rng = np.random.default_rng(93 + dim)
    c = rng.standard_normal(leg.n_dofs)
    for f_mod, f_leg in ((mod.apply, leg.apply), (mod.apply_p2p, leg.apply_p2p)):
        y = f_mod(c)
        y_ref = T.T @ f_leg(T @ c)
        assert np.linalg.norm(y - y_ref) <= 1e-12 * np.linalg.norm(y_ref)
    # the Jacobi diagonal is the diagonal of T^T A T
    A = leg.assemble()
    assert np.abs(mod.diagonal() - np.diag(T.T @ A @ T)).max() <= 1e-12 * np.abs(A).max()


def test_modal_operator_symmetric_positive_definite(oracle_lib):
    m = synth.small_mesh(3, 2, ("random", 2, 4), seed=94, rotate=True, lam=1.0)
    A = oracle_lib.prepare(m, "modal").assemble()
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
    np.linalg.cholesky(0.5 * (A + A.T))
