"""Pins of the oracle's point-to-point flux (Sec. 3.3, ScatrInterp): every
interior face is integrated once per side, on that side's own GLL face
quadrature, with the other side's value and physical gradient Lagrange-
interpolated to it.

Facts pinned here, none of them computed by the code under test:
* conforming faces (equal orders) have identical point sets, so the flux is
  the shared-trace flux, whose oracle is pinned independently;
* a global affine u is interpolated exactly, so both fluxes agree on it;
* the symmetry conditions of Sec. 3.3: with N_P coefficients and N_Q points
  per direction, N_Pl < N_Pr <= N_Ql < N_Qr and a lower-side quadrature exact
  for the integrand make A symmetric.  With Q = p + 2 this holds for orders
  3 | 4 (P4Q5-P5Q6) on affine elements, where every face integrand has degree
  7 per direction and both GLL rules are exact, so A equals the shared-trace
  operator.  It fails for orders 2 | 4 (P3Q4-P5Q6: degree 6 on 4 GLL points)
  and for 3 | 4 on deformed hexahedra (non-constant J, n); the asymmetry
  ||A - A^T||_1 / ||A||_1 is then clearly above rounding (Table 2 pattern)."""

from __future__ import annotations

import numpy as np
import pytest

import synth
from tests import pins


def _asym(A):
    return np.abs(A - A.T).sum(axis=0).max() / np.abs(A).sum(axis=0).max()


def _checker(m, N, dim, a, b):
    e = np.arange(m.n_elems)
    par = (e % N + (e // N) % N + ((e // (N * N)) if dim == 3 else 0)) % 2
    m.order = np.where(par == 0, a, b).astype(np.int32)
    return m


@pytest.mark.parametrize("dim,N,p,seed", [(2, 4, 3, 71), (3, 2, 2, 72), (3, 2, 4, 73)])
def test_conforming_faces_equal_shared_trace(oracle_lib, dim, N, p, seed):
    m = synth.small_mesh(dim, N, p, seed=seed, lam=1.2, rotate=True)
    om = oracle_lib.prepare(m)
    x = synth.random_coefficients(m, seed)
    y0, y1 = om.apply(x), om.apply_p2p(x)
    assert np.linalg.norm(y1 - y0) <= 1e-13 * np.linalg.norm(y0)


@pytest.mark.parametrize("dim,N,orders", [(2, 5, ("random", 1, 5)), (3, 3, ("random", 1, 4))])
def test_affine_field_agrees_with_shared_trace(oracle_lib, dim, N, orders):
    """Global affine u on perturbed, non-conforming, rotated meshes: the
    neighbour's u and grad u are interpolated exactly, both fluxes give the
    same rows, and with lambda = 0 the interior rows vanish (patch test)."""
    m = synth.small_mesh(dim, N, orders, seed=74, lam=0.0, rotate=True)
    om = oracle_lib.prepare(m)
    a = np.array([0.3, -1.1, 0.7][:dim])
    x = pins.project(m, lambda X: X @ a + 0.4)
    y0, y1 = om.apply(x), om.apply_p2p(x)
    assert np.abs(y1 - y0).max() <= 1e-12 * np.abs(y0).max()
    inner = pins.interior_elements(om)
    assert inner
    r = max(np.abs(y1[om.dof_off[e]:om.dof_off[e + 1]]).max() for e in inner)
    assert r <= 1e-12 * np.abs(y1).max()


def test_random_field_differs_on_nonconforming_faces(oracle_lib):
    """On non-conforming faces the two fluxes are different operators."""
    m = synth.small_mesh(3, 2, ("checker", 2, 4), seed=75, lam=1.0, rotate=True)
    om = oracle_lib.prepare(m)
    x = synth.random_coefficients(m, 75)
    y0, y1 = om.apply(x), om.apply_p2p(x)
    assert np.linalg.norm(y1 - y0) >= 1e-6 * np.linalg.norm(y0)


@pytest.mark.parametrize("dim", [2, 3])
def test_symmetric_case_p4q5_p5q6_affine(oracle_lib, dim):
    m = _checker(synth.affine_mesh(dim, 2 if dim == 3 else 4, seed=76, order=1, lam=0.9),
                 2 if dim == 3 else 4, dim, 3, 4)
    m = synth.rotate_elements(m, 77)
    om = oracle_lib.prepare(m)
    A1 = om.assemble("p2p")
    A0 = om.assemble("shared")
    assert _asym(A1) <= 1e-13
    assert np.abs(A1 - A0).max() <= 1e-12 * np.abs(A0).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_asymmetric_case_p3q4_p5q6(oracle_lib, dim):
    m = _checker(synth.affine_mesh(dim, 2 if dim == 3 else 4, seed=78, order=1, lam=0.9),
                 2 if dim == 3 else 4, dim, 2, 4)
    om = oracle_lib.prepare(m)
    A1 = om.assemble("p2p")
    assert _asym(A1) >= 1e-4
    assert _asym(om.assemble("shared")) <= 1e-13


def test_asymmetric_case_p4q5_p5q6_deformed(oracle_lib):
    m = synth.small_mesh(3, 2, ("checker", 3, 4), seed=79, lam=0.9)
    om = oracle_lib.prepare(m)
    a = _asym(om.assemble("p2p"))
    assert 1e-7 <= a <= 1e-1
