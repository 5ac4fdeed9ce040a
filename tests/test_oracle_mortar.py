"""Pin of the oracle's shared-trace face terms by the mortar projection.

Sec. 3.3 (shared trace space) states that evaluating each side's solution at
the trace quadrature points is the L2 (mortar) projection onto the trace
space, coefficients (M^Xi)^-1 S u_hat, evaluated at those points, whenever
the trace space has at least the order of the side.  This test builds the
penalty part of the operator that way, with nothing from the oracle:

  * the trace space of a face is the tensor Legendre space of degree
    p_F = max(p_L, p_R) in the owner's face coordinates; its mass matrix M
    and the transfer matrix S (mortar basis against the side's basis
    functions restricted to the face) are integrated with NumPy's
    Gauss-Legendre rule, enough points to be exact;
  * the neighbour's face coordinates of a mortar point come from its
    physical position (Newton on the neighbour's face map), not from any
    orientation code;
  * the trace's GLL points are the roots of P'_{n-1} plus the end points
    (NumPy's Legendre root finder), weights 2 / (n (n-1) P_{n-1}^2);
  * a = w |dx/dz_1 x dx/dz_2| (3-D) or w |dx/dz| (2-D) on the owner's face.

The penalty matrix sum_F tau0_F sum_q a_q [phi_i][phi_j] (2 tau0 on the
boundary, the mirrored exterior value) must equal A(sigma = 1) - A(sigma = 0)
of the oracle, assembled column by column: the operator is affine in sigma
and only the penalty carries it.  Negative control: projecting onto a trace
space of the lower side's degree misses (the projection is then no longer
exact for the higher side)."""

from __future__ import annotations

import itertools

import numpy as np
import pytest

import synth

oracle = pytest.importorskip("oracle")
leg = np.polynomial.legendre


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def gll_points(n):
    c = np.zeros(n)
    c[n - 1] = 1.0
    inner = np.sort(np.real(leg.legroots(leg.legder(c)))) if n > 2 else np.zeros(0)
    x = np.concatenate([[-1.0], inner, [1.0]])
    w = 2.0 / (n * (n - 1) * leg.legval(x, c) ** 2)
    return x, w


def legendre_vals(p, t):
    """P_0..P_p at the points t: [p+1, len(t)]."""
    t = np.atleast_1d(t)
    return np.array([leg.legval(t, np.eye(p + 1)[i]) for i in range(p + 1)])


class Geom:
    def __init__(self, mesh):
        self.d = mesh.dim
        self.X = mesh.coords[mesh.elem_vertices]   # [ne, 2^d, d]
        self.order = mesh.order

    def map(self, e, xi):
        """Physical points of reference points xi [m, d]."""
        d = self.d
        out = np.zeros((xi.shape[0], d))
        for c in range(2 ** d):
            w = np.ones(xi.shape[0])
            for k in range(d):
                b = (c >> k) & 1
                w = w * ((1 + xi[:, k]) / 2 if b else (1 - xi[:, k]) / 2)
            out += w[:, None] * self.X[e, c][None, :]
        return out

    def embed(self, f, z):
        """Reference points of face f = 2k + s at face coordinates z [m, d-1]."""
        d, k, s = self.d, f // 2, f % 2
        xi = np.zeros((z.shape[0], d))
        xi[:, k] = 1.0 if s else -1.0
        others = [a for a in range(d) if a != k]
        for j, a in enumerate(others):
            xi[:, a] = z[:, j]
        return xi

    def face_map(self, e, f, z):
        return self.map(e, self.embed(f, z))

    def face_tangents(self, e, f, z, h=0.5):
        # the face map is linear in each face coordinate: a central
        # difference is exact for any step
        cols = []
        for j in range(self.d - 1):
            dz = np.zeros_like(z)
            dz[:, j] = h
            cols.append((self.face_map(e, f, z + dz) - self.face_map(e, f, z - dz)) / (2 * h))
        return cols

    def face_coords_of(self, e, f, x):
        """Face coordinates on (e, f) of physical points x (Newton)."""
        z = np.zeros((x.shape[0], self.d - 1))
        for _ in range(30):
            r = self.face_map(e, f, z) - x
            T = np.stack(self.face_tangents(e, f, z), axis=-1)   # [m, d, d-1]
            dz = np.array([np.linalg.lstsq(T[i], r[i], rcond=None)[0] for i in range(len(x))])
            z = z - dz
            if np.abs(dz).max() < 1e-15:
                break
        assert np.abs(self.face_map(e, f, z) - x).max() < 1e-12
        return z

    def basis_on_face(self, e, f, z):
        """phi_i of element e at the points z of its face f: [nm, m], modes
        lexicographic with the first reference direction fastest."""
        p, d = int(self.order[e]), self.d
        xi = self.embed(f, z)
        V = [legendre_vals(p, xi[:, k]) for k in range(d)]
        rows = []
        for idx in itertools.product(range(p + 1), repeat=d):
            i = idx[::-1]   # i[0] fastest
            v = np.ones(z.shape[0])
            for k in range(d):
                v = v * V[k][i[k]]
            rows.append(v)
        return np.array(rows)


def tensor_rule(n, dm1):
    x, w = leg.leggauss(n)
    if dm1 == 1:
        return x[:, None], w
    X = np.array([[a, b] for b in x for a in x])
    W = np.array([wa * wb for wb in w for wa in w])
    return X, W


def mortar_trace(geo, e, f, zq, pF, own_coords):
    """Values at the trace points zq (owner's face coordinates) of the L2
    projection of each basis function of (e, f) onto the degree-pF Legendre
    trace space: ((M^Xi)^-1 S)^T evaluated at zq, [nm, len(zq)]."""
    dm1 = geo.d - 1
    zg, wg = tensor_rule(pF + int(geo.order[e]) + 3, dm1)
    ce = [legendre_vals(pF, zg[:, j]) for j in range(dm1)]
    cq = [legendre_vals(pF, zq[:, j]) for j in range(dm1)]
    modes = list(itertools.product(range(pF + 1), repeat=dm1))
    Bg = np.array([np.prod([ce[j][m[::-1][j]] for j in range(dm1)], axis=0) for m in modes])
    Bq = np.array([np.prod([cq[j][m[::-1][j]] for j in range(dm1)], axis=0) for m in modes])
    M = (Bg * wg) @ Bg.T
    zs = own_coords(zg)                       # this side's face coordinates of the mortar points
    phi = geo.basis_on_face(e, f, zs)         # [nm, ng]
    S = (Bg * wg) @ phi.T                     # [modes, nm]
    coef = np.linalg.solve(M, S)
    return (Bq.T @ coef).T


def faces_of(mesh):
    d = mesh.dim
    table = {}
    for e in range(mesh.n_elems):
        for f in range(2 * d):
            k, s = f // 2, f % 2
            ids = [int(mesh.elem_vertices[e, c]) for c in range(2 ** d) if ((c >> k) & 1) == s]
            table.setdefault(tuple(sorted(ids)), []).append((e, f))
    return list(table.values())


def mortar_penalty(mesh, trace_degree=max):
    geo = Geom(mesh)
    d = mesh.dim
    off = mesh.dof_offsets()
    A = np.zeros((mesh.n_dofs, mesh.n_dofs))
    for sides in faces_of(mesh):
        sides = sorted(sides)
        eL, fL = sides[0]
        pL = int(mesh.order[eL])
        if len(sides) == 2:
            eR, fR = sides[1]
            pR = int(mesh.order[eR])
            pF = trace_degree(pL, pR)
            nF = max(pL, pR) + 2
        else:
            pF, nF = pL, pL + 2
        x1, w1 = gll_points(nF)
        if d == 2:
            zq, wq = x1[:, None], w1
        else:
            zq = np.array([[a, b] for b in x1 for a in x1])
            wq = np.array([wa * wb for wb in w1 for wa in w1])
        T = geo.face_tangents(eL, fL, zq)
        Js = np.linalg.norm(T[0], axis=1) if d == 2 else np.linalg.norm(np.cross(T[0], T[1]), axis=1)
        a = wq * Js
        tau0 = 2.0 * (max(pL, int(mesh.order[sides[-1][0]])) + 1) ** 2 / mesh.h
        VL = mortar_trace(geo, eL, fL, zq, pF, lambda z: z)
        rL = np.arange(off[eL], off[eL + 1])
        if len(sides) == 1:
            A[np.ix_(rL, rL)] += 2 * tau0 * (VL * a) @ VL.T
            continue
        own = lambda z: geo.face_coords_of(eR, fR, geo.face_map(eL, fL, z))
        VR = mortar_trace(geo, eR, fR, zq, pF, own)
        rR = np.arange(off[eR], off[eR + 1])
        J = np.concatenate([VL, -VR])          # jump of each basis function
        rows = np.concatenate([rL, rR])
        A[np.ix_(rows, rows)] += tau0 * (J * a) @ J.T
    return A


def oracle_penalty(mesh):
    om = oracle.prepare(mesh)
    om.set_sigma(1.0)
    A1 = om.assemble()
    om.set_sigma(0.0)
    A0 = om.assemble()
    return A1 - A0


CASES = {
    "2d_random_p1to5_rot": lambda: synth.small_mesh(2, 3, ("random", 1, 5), seed=61, rotate=True, lam=0.7),
    "2d_checker24": lambda: synth.small_mesh(2, 3, ("checker", 2, 4), seed=62, lam=1.0),
    "3d_random_p1to3_rot": lambda: synth.small_mesh(3, 2, ("random", 1, 3), seed=63, rotate=True, lam=1.0),
    "3d_affine_p1to3_rot": lambda: synth.rotate_elements(
        _with_orders(synth.affine_mesh(3, 2, seed=64, order=1, lam=1.0), 65, 1, 3), 66),
}


def _with_orders(m, seed, lo, hi):
    m.order = np.random.default_rng(seed).integers(lo, hi + 1, m.n_elems).astype(np.int32)
    return m


@pytest.mark.parametrize("name", list(CASES))
def test_penalty_equals_mortar_projection(name):
    mesh = CASES[name]()
    assert len(set(mesh.order.tolist())) > 1, "needs non-conforming faces"
    Ao = oracle_penalty(mesh)
    Am = mortar_penalty(mesh)
    scale = np.abs(Ao).max()
    err = np.abs(Ao - Am).max() / scale
    print(f"{name}: penalty vs mortar projection, max rel {err:.2e}")
    assert err <= 1e-11
    # negative control: a trace space of the lower side's degree is not exact
    Alo = mortar_penalty(mesh, trace_degree=min)
    assert np.abs(Ao - Alo).max() / scale > 1e-3
