"""Restarted GMRES through the C ABI, for the nonsymmetric point-to-point
operator (the paper solves it with GMRES, Table 2) and for the shared-trace
operator.  Reference: a plain NumPy GMRES(m) with the same right Jacobi
preconditioning written around the oracle's operators (modified Gram-Schmidt,
so its rounding differs); the solutions must solve the oracle's system and the
Arnoldi step counts agree within a few steps."""

from __future__ import annotations

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2504_03573_amd as P
    return P


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


def gmres_ref(apply, b, dinv, tol, m, maxit):
    """Right-preconditioned GMRES(m) from x = 0; returns x and Arnoldi steps."""
    n = len(b)
    x = np.zeros(n)
    bn = np.linalg.norm(b)
    steps = 0
    while True:
        r = b - apply(x)
        beta = np.linalg.norm(r)
        if beta / bn <= tol or steps >= maxit:
            return x, steps, beta / bn
        V = np.zeros((m + 1, n))
        H = np.zeros((m + 1, m))
        V[0] = r / beta
        k = 0
        for j in range(m):
            w = apply(dinv * V[j])
            for i in range(j + 1):
                H[i, j] = V[i] @ w
                w -= H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            steps += 1
            k = j + 1
            e1 = np.zeros(k + 1)
            e1[0] = beta
            y, *_ = np.linalg.lstsq(H[:k + 1, :k], e1, rcond=None)
            res = np.linalg.norm(H[:k + 1, :k] @ y - e1)
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            if res / bn <= tol or H[j + 1, j] == 0 or steps >= maxit:
                break
        x += dinv * (V[:k].T @ y)


def _checker_affine(N, a, b, seed):
    m = synth.affine_mesh(3, N, seed=seed, order=1, lam=0.9)
    e = np.arange(m.n_elems)
    m.order = np.where((e % N + (e // N) % N + e // (N * N)) % 2 == 0, a, b).astype(np.int32)
    return synth.rotate_elements(m, seed + 1)


CASES = {
    "p2p_checker24_affine_n3": (lambda: _checker_affine(3, 2, 4, 85), "p2p"),
    "p2p_random_p1to4_n3_rot": (lambda: synth.small_mesh(3, 3, ("random", 1, 4), seed=86, rotate=True, lam=1.0), "p2p"),
    "shared_random_p2to5_n2_rot": (lambda: synth.small_mesh(3, 2, ("random", 2, 5), seed=87, rotate=True, lam=1.0), "shared"),
}


@pytest.mark.parametrize("name", list(CASES))
def test_gmres_matches_reference(P, orc, name):
    print(f"[gmres case {name}]", flush=True)
    make, flux = CASES[name]
    mesh = make()
    op = P.SipdgOperator(mesh)
    om = orc.prepare(mesh)
    apply = om.apply_p2p if flux == "p2p" else om.apply
    dinv = 1.0 / om.diagonal()
    x_true = synth.random_coefficients(mesh, 8101)
    b = apply(x_true)
    op.flux = flux
    m = 20
    xg, info = op.gmres_solve(torch.tensor(b, device="cuda"), tol=1e-10, restart=m)
    xr, steps, rel_r = gmres_ref(apply, b, dinv, 1e-10, m, 100000)
    xg = xg.cpu().numpy()
    print(f"{name}: gpu {info} reference steps {steps}")
    assert info["converged"] and info["rel_resid"] <= 1e-10
    assert np.linalg.norm(b - apply(xg)) <= 1e-9 * np.linalg.norm(b)
    assert np.linalg.norm(xg - x_true) <= 1e-6 * np.linalg.norm(x_true)
    assert abs(info["iters"] - steps) <= max(3, 0.05 * steps), (info["iters"], steps)
    # deterministic
    xg2, info2 = op.gmres_solve(torch.tensor(b, device="cuda"), tol=1e-10, restart=m)
    assert info2["iters"] == info["iters"] and np.array_equal(xg2.cpu().numpy(), xg)


def test_gmres_options_and_limits(P):
    m = synth.small_mesh(3, 2, ("random", 2, 4), seed=88, lam=1.0)
    op = P.SipdgOperator(m)
    op.flux = "p2p"
    b = op.apply(torch.tensor(synth.random_coefficients(m, 8102), device="cuda"))
    with pytest.raises(P.SipdgError):
        op.gmres_solve(b, restart=0)
    x, info = op.gmres_solve(b, tol=1e-12, maxit=3, raise_on_fail=False)
    assert not info["converged"] and info["iters"] == 3
    x, info = op.gmres_solve(b, tol=1e-10, restart=5, precond=False)
    assert info["converged"] and info["restarts"] >= 2
    z = torch.zeros_like(b)
    x, info = op.gmres_solve(z)
    assert info["converged"] and info["iters"] == 0 and float(x.abs().max()) == 0.0
