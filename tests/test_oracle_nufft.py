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
