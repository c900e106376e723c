"""Pins of the oracle's NUFFT (eq. (1)) against things other than itself."""
import math

import numpy as np
import pytest
import scipy.integrate
import scipy.special

from oracle import nufft


def _rand_img(rng, L, N):
    return rng.standard_normal((L, N, N)) + 1j * rng.standard_normal((L, N, N))


def test_i0_series_matches_scipy():
    z = np.linspace(0.0, 14.0, 57)
    np.testing.assert_allclose(nufft.bessel_i0(z), scipy.special.i0(z), rtol=1e-14)


def test_beatty_beta_value():
    # pi * sqrt((6/2)^2 (2 - 1/2)^2 - 0.8) for W = 6, sigma = 2
    assert abs(nufft.kb_beta(6, 2) - 13.855100) < 1e-5   # sqrt(19.45) = 4.4102154


@pytest.mark.parametrize("s", [0.0, 0.05, 0.13, 0.25, 0.4])
def test_kb_ft_closed_form_matches_quadrature(s):
    W, beta = 6, nufft.kb_beta(6, 2)
    val, _ = scipy.integrate.quad(lambda t: float(nufft.kb_kernel(t, W, beta)) * math.cos(2 * math.pi * s * t),
                                  -W / 2, W / 2, epsabs=1e-12, epsrel=1e-13, limit=200)
    assert abs(float(nufft.kb_ft(np.array([s]), W, beta)[0]) - val) <= 1e-9 * abs(val)


@pytest.mark.parametrize("N,Ns", [(8, 37), (12, 200), (16, 200), (32, 37)])
def test_gridding_matches_brute_force_nudft(N, Ns):
    rng = np.random.default_rng(N * 1000 + Ns)
    traj = rng.uniform(-math.pi, math.pi, (2, Ns, 2))
    X = _rand_img(rng, 2, N)
    b = nufft.nufft_fwd(X, traj)
    ref = nufft.nudft_fwd(X, traj)
    err = np.linalg.norm(b - ref) / np.linalg.norm(ref)
    assert err < 1e-4, err


def test_adjoint_identity():
    rng = np.random.default_rng(3)
    N, Ns, L = 16, 150, 3
    traj = rng.uniform(-math.pi, math.pi, (L, Ns, 2))
    x = _rand_img(rng, L, N)
    y = rng.standard_normal((L, Ns)) + 1j * rng.standard_normal((L, Ns))
    lhs = np.vdot(nufft.nufft_fwd(x, traj), y)
    rhs = np.vdot(x, nufft.nufft_adj(y, traj, N))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_full_cartesian_sampling_is_the_centred_unitary_dft():
    rng = np.random.default_rng(4)
    N = 16
    k = np.arange(N) - N // 2
    ky, kx = np.meshgrid(k, k, indexing="ij")
    traj = np.stack([2 * math.pi * kx.ravel() / N, 2 * math.pi * ky.ravel() / N], -1)[None]
    X = _rand_img(rng, 1, N)
    ref = np.fft.fft2(np.fft.ifftshift(X[0]), norm="ortho")[ky % N, kx % N].ravel()
    exact = nufft.nudft_fwd(X, traj)[0]
    assert np.linalg.norm(exact - ref) <= 1e-12 * np.linalg.norm(ref)
    grid = nufft.nufft_fwd(X, traj)[0]
    assert np.linalg.norm(grid - ref) <= 1e-4 * np.linalg.norm(ref)
    # and the adjoint inverts it on this unitary case
    back = nufft.nufft_adj(grid[None], traj, N)[0]
    assert np.linalg.norm(back - X[0]) <= 2e-4 * np.linalg.norm(X[0])


def test_power_iteration_bounds_the_dense_operator():
    rng = np.random.default_rng(5)
    N, Ns = 8, 90
    traj = rng.uniform(-math.pi, math.pi, (1, Ns, 2))
    A = np.stack([nufft.nufft_fwd(e.reshape(1, N, N), traj)[0] for e in np.eye(N * N)], axis=1)
    lam_true = np.linalg.eigvalsh(A.conj().T @ A).max()
    lam = nufft.operator_norm(traj, N, _rand_img(rng, 1, N), iters=200)
    assert abs(lam - lam_true) <= 1e-6 * lam_true


def _coil_maps(rng, Nc, N):
    S = rng.standard_normal((Nc, N, N)) + 1j * rng.standard_normal((Nc, N, N))
    return S / np.sqrt(np.sum(np.abs(S) ** 2, axis=0))[None]


@pytest.mark.parametrize("N,Nc,Ns", [(8, 3, 37), (12, 4, 150)])
def test_multicoil_matches_dense_stack_of_coil_blocks(N, Nc, Ns):
    """eq. (1) with coils: the dense operator [F diag(S_1); ...; F diag(S_Nc)] with F the exact
    NUDFT matrix, applied by hand, agrees with nufft_fwd_mc to the KB error (1e-4, as the
    single-coil pin)."""
    rng = np.random.default_rng(N * 10 + Nc)
    traj = rng.uniform(-math.pi, math.pi, (2, Ns, 2))
    X = _rand_img(rng, 2, N)
    S = _coil_maps(rng, Nc, N)
    b = nufft.nufft_fwd_mc(X, traj, S)
    assert b.shape == (Nc, 2, Ns)
    for l in range(2):
        F = nufft.nudft_matrix(traj[l], N)
        for c in range(Nc):
            ref = F @ (S[c].ravel() * X[l].ravel())
            assert np.linalg.norm(b[c, l] - ref) <= 1e-4 * np.linalg.norm(ref)
    # the adjoint against the dense conjugate transpose
    y = rng.standard_normal((Nc, 2, Ns)) + 1j * rng.standard_normal((Nc, 2, Ns))
    a = nufft.nufft_adj_mc(y, traj, N, S)
    for l in range(2):
        F = nufft.nudft_matrix(traj[l], N)
        ref = sum(np.conj(S[c].ravel()) * (F.conj().T @ y[c, l]) for c in range(Nc)).reshape(N, N)
        assert np.linalg.norm(a[l] - ref) <= 1e-4 * np.linalg.norm(ref)


def test_multicoil_adjoint_identity_and_single_coil_reduction():
    rng = np.random.default_rng(21)
    N, Nc, Ns, L = 16, 5, 120, 3
    traj = rng.uniform(-math.pi, math.pi, (L, Ns, 2))
    S = _coil_maps(rng, Nc, N)
    X = _rand_img(rng, L, N)
    y = rng.standard_normal((Nc, L, Ns)) + 1j * rng.standard_normal((Nc, L, Ns))
    lhs = np.vdot(nufft.nufft_fwd_mc(X, traj, S), y)
    rhs = np.vdot(X, nufft.nufft_adj_mc(y, traj, N, S))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    one = np.ones((1, N, N))
    np.testing.assert_allclose(nufft.nufft_fwd_mc(X, traj, one)[0], nufft.nufft_fwd(X, traj), rtol=0, atol=1e-13)
    np.testing.assert_allclose(nufft.nufft_adj_mc(y[:1], traj, N, one), nufft.nufft_adj(y[0], traj, N), rtol=0,
                               atol=1e-13)


def test_multicoil_full_cartesian_normal_operator_is_identity():
    """Full Cartesian sampling makes F_u unitary (to the KB error) and sum_c |S_c|^2 = 1 then makes
    A^H A = sum_c conj(S_c) S_c = I; the synthetic coil generator has that normalisation."""
    import mrfgen
    N, L, Nc = 16, 2, 4
    k = np.arange(N) - N // 2
    ky, kx = np.meshgrid(k, k, indexing="ij")
    traj = np.repeat(np.stack([2 * math.pi * kx.ravel() / N, 2 * math.pi * ky.ravel() / N], -1)[None], L, 0)
    S = mrfgen.coil_maps(N, Nc, seed=3).astype(np.complex128)
    np.testing.assert_allclose(np.sum(np.abs(S) ** 2, axis=0), 1.0, rtol=1e-6)
    X = _rand_img(np.random.default_rng(4), L, N)
    Y = nufft.nufft_adj_mc(nufft.nufft_fwd_mc(X, traj, S), traj, N, S)
    assert np.linalg.norm(Y - X) <= 2e-4 * np.linalg.norm(X)
