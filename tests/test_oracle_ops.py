"""Pins of the oracle's per-iteration operators (eqs. (15)-(23))."""
import numpy as np
import pytest

from oracle import graph, ops, patches


def _cplx(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _unitary(rng, n):
    q, r = np.linalg.qr(_cplx(rng, n, n))
    return q * (np.diag(r) / np.abs(np.diag(r)))[None, :]


def test_svt_of_prescribed_spectrum():
    rng = np.random.default_rng(1)
    m, n = 6, 9
    U = _unitary(rng, m); V = _unitary(rng, n)[:, :m]
    sig = np.array([9.0, 7.0, 4.0, 2.5, 1.0, 0.5])
    P = U @ np.diag(sig) @ V.conj().T
    out, nuc = ops.svt(P, 2.0, 3)
    expect = U @ np.diag([7.0, 5.0, 2.0, 0, 0, 0]) @ V.conj().T
    np.testing.assert_allclose(out, expect, atol=1e-12)
    assert abs(nuc - sig.sum()) < 1e-12
    np.testing.assert_allclose(ops.svt(P, 0.0, m)[0], P, atol=1e-12)
    np.testing.assert_allclose(ops.svt(P, 9.0, m)[0], 0.0, atol=1e-12)


def test_svt_is_the_prox_of_the_nuclear_norm():
    """Without a cap, SVT_tau(P) minimises ||Y||_* + 1/(2 tau) ||Y - P||^2 (eq. (20))."""
    rng = np.random.default_rng(2)
    P = _cplx(rng, 5, 12)
    tau = 1.3
    Y, _ = ops.svt(P, tau, 5)

    def f(Y):
        return np.linalg.svd(Y, compute_uv=False).sum() + 0.5 / tau * np.linalg.norm(Y - P) ** 2
    f0 = f(Y)
    for _ in range(200):
        assert f(Y + 1e-3 * _cplx(rng, 5, 12)) >= f0 - 1e-12


def test_svd_route_equals_gram_eigh_route():
    rng = np.random.default_rng(3)
    P = _cplx(rng, 16, 40)
    tau, cap = 3.0, 6
    out, nuc = ops.svt(P, tau, cap)
    lam, U = np.linalg.eigh(P @ P.conj().T)
    lam, U = lam[::-1], U[:, ::-1]
    sig = np.sqrt(np.maximum(lam, 0))
    f = np.where(sig > tau, (sig - tau) / np.where(sig > 0, sig, 1), 0.0)
    f[cap:] = 0
    np.testing.assert_allclose(U @ np.diag(f) @ U.conj().T @ P, out, atol=1e-10)
    assert abs(sig.sum() - nuc) < 1e-10 * nuc


def test_projection_is_idempotent_and_eckart_young():
    rng = np.random.default_rng(4)
    D = _cplx(rng, 40, 12)
    D /= np.linalg.norm(D, axis=1, keepdims=True)
    _, s, vh = np.linalg.svd(D, full_matrices=False)
    r = 5
    V = vh[:r].conj().T
    assert np.allclose(V.conj().T @ V, np.eye(r), atol=1e-12)
    X = _cplx(rng, 12, 3, 3)
    PX = ops.project(X, V)
    np.testing.assert_allclose(ops.project(PX, V), PX, atol=1e-12)
    DV = ops.project(D.T.reshape(12, 40, 1), V).reshape(12, 40).T
    assert abs(np.linalg.norm(D - DV) ** 2 - np.sum(s[r:] ** 2)) < 1e-10


@pytest.mark.parametrize("N,p,s", [(12, 4, 2), (12, 4, 4)])
def test_x_update_minimises_eq21(N, p, s):
    rng = np.random.default_rng(5)
    L = 2
    mu, lam2, beta = 0.7, 0.3, 0.4
    Z = _cplx(rng, L, N, N)
    Np = len(patches.patch_origins(N, p, s))
    P = _cplx(rng, Np, p * p, L)
    X = ops.x_update(Z, patches.Qadj(P, N, p, s), mu, lam2, beta, p, s)
    grad = (X - Z) / mu + lam2 * beta * patches.Qadj(patches.Q(X, p, s) - P, N, p, s)
    assert np.max(np.abs(grad)) <= 1e-12
    if p == s:   # no overlap: the paper's scalar formula eq. (23)
        lit = (Z + mu * lam2 * beta * patches.Qadj(P, N, p, s)) / (1 + mu * lam2 * beta)
        np.testing.assert_allclose(X, lit, atol=1e-13)


def test_laplacian_apply_is_self_adjoint_and_kills_constants():
    rng = np.random.default_rng(6)
    N, p, s = 12, 4, 2
    maps = np.stack([rng.uniform(300, 2500, (N, N)), rng.uniform(40, 300, (N, N)), rng.uniform(0, 1, (N, N))])
    Lap = graph.knn_laplacian(maps, p, s, 4)["L"]
    X = _cplx(rng, 2, N, N); Y = _cplx(rng, 2, N, N)
    a = np.vdot(Y, ops.laplacian_apply(X, Lap, p, s))
    b = np.vdot(ops.laplacian_apply(Y, Lap, p, s), X)
    assert abs(a - b) <= 1e-12 * abs(a)
    const = np.full((2, N, N), 1.5 - 0.5j)
    assert np.max(np.abs(ops.laplacian_apply(const, Lap, p, s))) <= 1e-12


def test_llr_prox_with_one_patch_is_plain_svt():
    rng = np.random.default_rng(7)
    N, L = 4, 7
    X = _cplx(rng, L, N, N)
    out, nuc = ops.llr_prox(X, N, N, 0.8, 16)
    ref, nref = ops.svt(X.reshape(L, 16).T, 0.8, 16)
    np.testing.assert_allclose(out.reshape(L, 16).T, ref, atol=1e-12)
    assert abs(nuc - nref) < 1e-12
