"""Pins of the oracle's Toeplitz normal operator (A^H A of eq. (15) as a convolution)."""
import math

import numpy as np

from oracle import nufft, toeplitz


def _rand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_psf_kernel_is_the_defining_sum():
    rng = np.random.default_rng(0)
    N, L, Ns = 8, 2, 40
    traj = rng.uniform(-math.pi, math.pi, (L, Ns, 2))
    Kt = toeplitz.psf_circulant(traj, N)
    for l in range(L):
        ref = toeplitz.psf_exact(traj[l], N)
        assert np.linalg.norm(Kt[l] - ref) <= 1e-4 * np.linalg.norm(ref)
    # a single sample at the origin: K = 1/N^2 at every offset that occurs (|d| < N)
    K0 = toeplitz.psf_exact(np.zeros((1, 2)), N)
    want = np.full((2 * N, 2 * N), 1.0 / N ** 2)
    want[N, :] = 0.0
    want[:, N] = 0.0
    np.testing.assert_allclose(K0, want, rtol=0, atol=1e-15)


def test_toeplitz_equals_the_dense_normal_operator():
    """Against A^H A formed from the exact NUDFT matrix, with the exact kernel to 1e-12 and with
    the gridded kernel to the KB error."""
    rng = np.random.default_rng(1)
    N, L, Ns = 6, 2, 50
    traj = rng.uniform(-math.pi, math.pi, (L, Ns, 2))
    X = _rand(rng, L, N, N)
    exact = np.stack([toeplitz.psf_exact(traj[l], N) for l in range(L)])
    Y = toeplitz.toeplitz_normal(X, toeplitz.kernel_spectrum(exact))
    Yg = toeplitz.toeplitz_normal(X, toeplitz.kernel_spectrum(toeplitz.psf_circulant(traj, N)))
    for l in range(L):
        A = nufft.nudft_matrix(traj[l], N)
        ref = (A.conj().T @ (A @ X[l].ravel())).reshape(N, N)
        np.testing.assert_allclose(Y[l], ref, rtol=0, atol=1e-12 * np.abs(ref).max())
        assert np.linalg.norm(Yg[l] - ref) <= 1e-4 * np.linalg.norm(ref)


def test_toeplitz_matches_the_gridded_pair_and_is_hermitian_psd():
    rng = np.random.default_rng(2)
    N, L, Ns = 16, 3, 200
    traj = rng.uniform(-math.pi, math.pi, (L, Ns, 2))
    X, Z = _rand(rng, L, N, N), _rand(rng, L, N, N)
    Kh = toeplitz.kernel_spectrum(toeplitz.psf_circulant(traj, N))
    assert np.abs(Kh.imag).max() <= 1e-10 * np.abs(Kh.real).max()       # Hermitian kernel: real spectrum
    TX = toeplitz.toeplitz_normal(X, Kh)
    ref = nufft.nufft_adj(nufft.nufft_fwd(X, traj), traj, N)
    assert np.linalg.norm(TX - ref) <= 1e-4 * np.linalg.norm(ref)
    TZ = toeplitz.toeplitz_normal(Z, Kh)
    assert abs(np.vdot(Z, TX) - np.vdot(TZ, X)) <= 1e-10 * abs(np.vdot(Z, TX))
    assert np.vdot(X, TX).real > 0 and abs(np.vdot(X, TX).imag) <= 1e-10 * np.vdot(X, TX).real


def test_cost_identity():
    rng = np.random.default_rng(3)
    N, L, Ns = 8, 2, 60
    traj = rng.uniform(-math.pi, math.pi, (L, Ns, 2))
    X, b = _rand(rng, L, N, N), _rand(rng, L, Ns)
    exact = np.stack([toeplitz.psf_exact(traj[l], N) for l in range(L)])
    TX = toeplitz.toeplitz_normal(X, toeplitz.kernel_spectrum(exact))
    AHb = np.stack([(nufft.nudft_matrix(traj[l], N).conj().T @ b[l]).reshape(N, N) for l in range(L)])
    direct = 0.5 * np.linalg.norm(nufft.nudft_fwd(X, traj) - b) ** 2
    assert abs(toeplitz.data_term(X, TX, AHb, np.vdot(b, b).real) - direct) <= 1e-10 * direct
