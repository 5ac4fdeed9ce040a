"""Pins of the oracle against facts other than itself.

Each test names the passage of Xia & Moxey (arXiv 2504.03573) or the
mathematical fact it checks.  Together they are chosen so that a dropped
term, a wrong sign, a wrong index or a transposed operand in the oracle fails
at least one of them."""

from __future__ import annotations

import math
import os

import numpy as np
import pytest

import synth
from tests import pins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_table(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append(line.split())
    return rows


# ----------------------------------------------------------------- quadrature

def test_gll_closed_forms(oracle_lib):
    """GLL nodes/weights (Sec. 2.1 quadrature) equal their closed forms."""
    env = {"sqrt": math.sqrt}
    for n, i, node, weight in _read_table("gll_closed_forms.txt"):
        n, i = int(n), int(i)
        x, w = oracle_lib.gll(n)
        assert abs(x[i] - eval(node, env)) < 1e-15
        assert abs(w[i] - eval(weight, env)) < 1e-15


@pytest.mark.parametrize("n", range(3, 14))
def test_gll_degree_of_exactness(oracle_lib, n):
    """Q-point GLL integrates degree 2Q-3 exactly and not 2Q-2 (Table 2,
    row 'actual quadrature degree')."""
    x, w = oracle_lib.gll(n)
    assert abs(w.sum() - 2.0) < 1e-14
    for deg in range(0, 2 * n - 2):
        exact = 0.0 if deg % 2 else 2.0 / (deg + 1)
        assert abs(np.sum(w * x ** deg) - exact) < 1e-13, deg
    deg = 2 * n - 2
    assert abs(np.sum(w * x ** deg) - 2.0 / (deg + 1)) > 1e-10


def test_quadrature_degree_table(oracle_lib):
    """Table 2 prints the GLL degree of exactness 2Q-3 for Q = 4, 5."""
    for Q, deg in _read_table("quadrature_degree.txt"):
        Q, deg = int(Q), int(deg)
        x, w = oracle_lib.gll(Q)
        for j in range(deg + 1):
            exact = 0.0 if j % 2 else 2.0 / (j + 1)
            assert abs(np.sum(w * x ** j) - exact) < 1e-13
        assert abs(np.sum(w * x ** (deg + 1)) - 2.0 / (deg + 2)) > 1e-6


# ----------------------------------------------------------------- geometry

@pytest.mark.parametrize("dim,N", [(2, 5), (3, 3)])
def test_geometry_invariants(oracle_lib, dim, N):
    """Sum of w|J| is the domain measure; each element's area-weighted
    outward normals close (sum n J_s w = 0); boundary faces cover 2d units
    of area; all Jacobians positive."""
    m = synth.small_mesh(dim, N, ("random", 1, 4), seed=21, rotate=True)
    om = oracle_lib.prepare(m)
    _, wd, _ = om.sample(np.zeros(om.n_dofs))
    assert abs(wd.sum() - 1.0) < 1e-13
    assert om.min_detj().min() > 0
    sn, area = om.face_moments()
    assert np.abs(sn.sum(axis=1)).max() < 1e-14
    bnd = om.nb < 0
    assert abs(area[bnd].sum() - 2 * dim) < 1e-12


# ----------------------------------------------------------------- operator

@pytest.mark.parametrize("dim,N,p,lam,sigma", [
    (2, 3, 2, 1.5, 1.3),
    (2, 2, 4, 0.0, 1.0),
    (3, 2, 2, 0.7, 1.0),
    (3, 2, 3, 2.0, 0.8),
])
def test_tensor_product_identity(oracle_lib, dim, N, p, lam, sigma):
    """On an unperturbed uniform mesh with one order the operator factorises
    into 1-D SIPG stiffness and mass matrices (eq. IP / eq. primal reduce to
    the textbook 1-D SIPG form in each direction, Arnold et al.)."""
    m = synth.structured_mesh(dim, N, 0.0, order=p, lam=lam, sigma=sigma)
    om = oracle_lib.prepare(m)
    A = om.assemble()
    T = pins.tensor_operator(dim, N, p, m.h, sigma, lam)
    perm = pins.kron_permutation(dim, N, p)
    Tp = T[np.ix_(perm, perm)]
    assert np.abs(A - Tp).max() <= 1e-13 * np.abs(A).max()


SYM_CASES = [
    # (dim, N, orders, rotate, seed) - cfg1 itself, a checkerboard 4/5,
    # random 3-D orders, rotated 3-D local orientations
    (2, 4, 3, False, 1001),
    (2, 4, ("checker", 4, 5), False, 1002),
    (2, 4, ("random", 1, 5), True, 5),
    (3, 2, ("random", 3, 5), False, 8),
    (3, 3, ("random", 1, 3), True, 9),
]


@pytest.mark.parametrize("dim,N,orders,rotate,seed", SYM_CASES)
def test_symmetric_positive_definite(oracle_lib, dim, N, orders, rotate, seed):
    """Shared-trace evaluation makes A symmetric (Appendix A: the face blocks
    satisfy M'_C = -M_C^T etc. when both sides use the same quadrature) and
    SPD for lambda > 0.  Metric of Table 2: ||A-A^T||_1 / ||A||_1."""
    m = synth.small_mesh(dim, N, orders, seed=seed, lam=1.0, rotate=rotate)
    om = oracle_lib.prepare(m)
    A = om.assemble()
    asym = np.abs(A - A.T).sum(axis=0).max() / np.abs(A).sum(axis=0).max()
    assert asym <= 1e-13
    np.linalg.cholesky(0.5 * (A + A.T))


def test_diagonal_matches_assembly(oracle_lib):
    m = synth.small_mesh(3, 2, ("random", 1, 3), seed=4, lam=0.5, rotate=True)
    om = oracle_lib.prepare(m)
    A = om.assemble()
    assert np.abs(np.diag(A) - om.diagonal()).max() <= 1e-13 * np.abs(A).max()


@pytest.mark.parametrize("dim,N,orders", [(2, 5, ("random", 1, 5)), (3, 3, ("random", 1, 3))])
def test_patch_test(oracle_lib, dim, N, orders):
    """lambda = 0 and a global affine u: (A u)_i = 0 on every element without
    a boundary face, on perturbed, non-conforming, rotated meshes (every
    integrand is polynomial within GLL exactness; consistency of eq. IP)."""
    m = synth.small_mesh(dim, N, orders, seed=31, lam=0.0, rotate=True)
    om = oracle_lib.prepare(m)
    a = np.array([0.3, -1.1, 0.7][:dim])
    x = pins.project(m, lambda X: X @ a + 0.4)
    y = om.apply(x)
    inner = pins.interior_elements(om)
    assert inner
    r = max(np.abs(y[om.dof_off[e]:om.dof_off[e + 1]]).max() for e in inner)
    assert r <= 1e-12 * np.abs(y).max()


def _poly2(dim):
    if dim == 2:
        u = lambda X: 1 + 2 * X[:, 0] - X[:, 1] + 0.5 * X[:, 0] ** 2 + 0.3 * X[:, 0] * X[:, 1] - 0.7 * X[:, 1] ** 2
        lap = 0.5 * 2 - 0.7 * 2
    else:
        u = lambda X: (1 + 2 * X[:, 0] - X[:, 1] + 0.4 * X[:, 2] + 0.5 * X[:, 0] ** 2
                       + 0.3 * X[:, 0] * X[:, 1] - 0.7 * X[:, 1] ** 2 + 0.2 * X[:, 1] * X[:, 2]
                       + 0.6 * X[:, 2] ** 2)
        lap = 0.5 * 2 - 0.7 * 2 + 0.6 * 2
    return u, lap


@pytest.mark.parametrize("dim,N", [(2, 4), (3, 2)])
def test_polynomial_exactness(oracle_lib, dim, N):
    """Global quadratic u on affine elements with mixed orders >= 2: the
    discrete equations hold exactly, A u = b with b from the source
    -lap u + lambda u and Dirichlet data u (eq. IP with the mirrored
    boundary value), and CG recovers u."""
    lam = 1.3
    m = synth.affine_mesh(dim, N, seed=41, order=2, lam=lam)
    rng = np.random.default_rng(42)
    m.order = rng.integers(2, 5, size=m.n_elems).astype(np.int32)
    m = synth.rotate_elements(m, 43)
    om = oracle_lib.prepare(m)
    u, lap = _poly2(dim)
    x = pins.project(m, u)
    b = om.rhs_from(lambda X: -lap + lam * u(X), u)
    y = om.apply(x)
    assert np.linalg.norm(y - b) <= 1e-12 * np.linalg.norm(b)
    xs, it, rel = om.cg(b, tol=1e-12)
    assert rel <= 1e-11
    assert np.abs(xs - x).max() <= 1e-8 * np.abs(x).max()


@pytest.mark.slow
def test_manufactured_convergence(oracle_lib):
    """sin(pi x) sin(pi y), CG solve, L2 error slope close to p+1 (Sec. 4.2:
    'around N_P order')."""
    k = math.pi
    lam = 1.0
    for p in (2, 3):
        errs = []
        for N in (4, 8, 16):
            m = synth.structured_mesh(2, N, 0.1, seed=1001, order=p, lam=lam)
            om = oracle_lib.prepare(m)
            ue = lambda X: np.sin(k * X[:, 0]) * np.sin(k * X[:, 1])
            b = om.rhs_from(lambda X: (lam + 2 * k * k) * ue(X), lambda X: np.zeros(len(X)))
            x, it, rel = om.cg(b, tol=1e-12)
            errs.append(om.l2_error(x, ue))
        slopes = [math.log(errs[i] / errs[i + 1], 2) for i in range(2)]
        assert abs(slopes[-1] - (p + 1)) < 0.35, (p, errs, slopes)


@pytest.mark.slow
@pytest.mark.parametrize("p,Ns", [(2, (2, 4, 6)), (3, (2, 3, 4))])
def test_manufactured_convergence_3d(oracle_lib, p, Ns):
    """Hexahedra (perturbed trilinear elements): sin(pi x) sin(pi y) sin(pi z),
    CG solve, L2 error slope close to p+1 over h = 1/N (Sec. 4.2, convergence
    under p-refinement: around N_P = p + 1)."""
    k = math.pi
    lam = 1.0
    ue = lambda X: np.sin(k * X[:, 0]) * np.sin(k * X[:, 1]) * np.sin(k * X[:, 2])
    errs = []
    for N in Ns:
        m = synth.structured_mesh(3, N, 0.1, seed=1003, order=p, lam=lam)
        om = oracle_lib.prepare(m)
        b = om.rhs_from(lambda X: (lam + 3 * k * k) * ue(X), lambda X: np.zeros(len(X)))
        x, it, rel = om.cg(b, tol=1e-12)
        errs.append(om.l2_error(x, ue))
    slopes = [math.log(errs[i] / errs[i + 1]) / math.log(Ns[i + 1] / Ns[i]) for i in range(len(Ns) - 1)]
    assert abs(slopes[-1] - (p + 1)) < 0.35, (p, errs, slopes)
    assert errs[-1] < errs[0]


@pytest.mark.parametrize("basis,points", [("legendre", "gll"), ("legendre", "gl"), ("modal", "gll"),
                                          ("modal", "gl")])
def test_param_grad_matches_finite_difference(oracle_lib, basis, points):
    """d(a^T A b)/d lambda_e and d/d sigma: the operator is affine in both,
    so a central difference of a^T A b is exact up to rounding.  With Gauss
    volume points the lambda derivative must come from the Gauss rule too:
    on these deformed elements the two rules' mass terms differ by ~1e-4
    relative, far above the tolerance."""
    # 3^3 lattice: the centre element has all eight corners moved, so its
    # |J| is not multilinear and the two volume rules differ on it
    m = synth.small_mesh(3, 3, ("random", 1, 3), seed=51, lam=1.0, rotate=True)
    m.lam = np.random.default_rng(52).uniform(0.5, 2.0, m.n_elems)
    om = oracle_lib.prepare(m, basis, points=points)
    rng = np.random.default_rng(53)
    a = rng.standard_normal(om.n_dofs)
    b = rng.standard_normal(om.n_dofs)
    dl, ds = om.param_grad(a, b)
    base = om.lam.copy()
    for e in (0, 3, 13):
        hstep = 1e-3
        om.lam[:] = base
        om.lam[e] += hstep
        fp = a @ om.apply(b)
        om.lam[e] -= 2 * hstep
        fm = a @ om.apply(b)
        fd = (fp - fm) / (2 * hstep)
        assert abs(fd - dl[e]) <= 1e-8 * max(1.0, abs(dl[e]))
    om.lam[:] = base
    s0 = om.sigma
    om.set_sigma(s0 + 1e-3)
    fp = a @ om.apply(b)
    om.set_sigma(s0 - 1e-3)
    fm = a @ om.apply(b)
    om.set_sigma(s0)
    fd = (fp - fm) / 2e-3
    assert abs(fd - ds) <= 1e-8 * max(1.0, abs(ds))


def test_orientation_invariance(oracle_lib):
    """Relabelling local corners (a rotation of each reference element) does
    not change the discrete space: A restricted to mode-permuted bases has
    the same spectrum."""
    m = synth.small_mesh(3, 2, ("random", 1, 2), seed=61, lam=0.8)
    A0 = oracle_lib.prepare(m).assemble()
    mr = synth.rotate_elements(m, 62)
    A1 = oracle_lib.prepare(mr).assemble()
    e0 = np.linalg.eigvalsh(A0)
    e1 = np.linalg.eigvalsh(0.5 * (A1 + A1.T))
    assert np.abs(e0 - e1).max() <= 1e-11 * np.abs(e0).max()
