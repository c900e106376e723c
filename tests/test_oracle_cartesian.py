"""Pins of the oracle's Cartesian acquisition (pseudo-radial Cartesian sampling, eq. (1))."""
import math

import numpy as np

import mrfgen
from oracle import cartesian as cart
from oracle import nufft


def _rand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_cartesian_operator_is_the_dft_definition():
    rng = np.random.default_rng(0)
    for N in (4, 6, 8):
        X = _rand(rng, 2, N, N)
        mask = (rng.uniform(size=(2, N, N)) < 0.4).astype(np.uint8)
        D = cart.dft_matrix(N)
        for l in range(2):
            want = mask[l].ravel() * (D @ X[l].ravel())
            np.testing.assert_allclose(cart.cart_fwd(X, mask)[l].ravel(), want, rtol=0, atol=1e-12)
            np.testing.assert_allclose(cart.cart_adj(X, mask)[l].ravel(), D.conj().T @ (mask[l].ravel() * X[l].ravel()),
                                       rtol=0, atol=1e-12)


def test_cartesian_operator_is_the_nufft_at_grid_frequencies():
    """The same frequencies through oracle.nufft (omega = 2 pi k / N): equal to its KB error."""
    rng = np.random.default_rng(1)
    N, L = 16, 2
    X = _rand(rng, L, N, N)
    mask = mrfgen.radial_cartesian_mask(N, L, 5)
    b = cart.cart_fwd(X, mask)
    for l in range(L):
        ky, kx = np.nonzero(mask[l])
        traj = np.stack([2 * math.pi * (kx - N // 2) / N, 2 * math.pi * (ky - N // 2) / N], -1)[None]
        ref = nufft.nufft_fwd(X[l:l + 1], traj)[0]
        got = b[l][ky, kx]
        assert np.linalg.norm(got - ref) <= 1e-4 * np.linalg.norm(ref)
        assert np.all(b[l][mask[l] == 0] == 0)


def test_cartesian_adjoint_identity_and_full_sampling():
    rng = np.random.default_rng(2)
    N, L = 32, 3
    X, Y = _rand(rng, L, N, N), _rand(rng, L, N, N)
    mask = mrfgen.radial_cartesian_mask(N, L, 6)
    lhs = np.vdot(cart.cart_fwd(X, mask), Y)
    rhs = np.vdot(X, cart.cart_adj(Y, mask))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    full = np.ones((L, N, N), np.uint8)
    np.testing.assert_allclose(cart.cart_adj(cart.cart_fwd(X, full), full), X, rtol=0, atol=1e-12)
    # energy is kept under full sampling (F unitary)
    assert abs(np.linalg.norm(cart.cart_fwd(X, full)) - np.linalg.norm(X)) <= 1e-12 * np.linalg.norm(X)


def test_cartesian_multicoil_stack():
    rng = np.random.default_rng(3)
    N, L, Nc = 16, 2, 3
    X = _rand(rng, L, N, N)
    S = mrfgen.coil_maps(N, Nc, seed=1)
    mask = mrfgen.radial_cartesian_mask(N, L, 4)
    b = cart.cart_fwd_mc(X, mask, S)
    for c in range(Nc):
        np.testing.assert_allclose(b[c], cart.cart_fwd(X * S[c][None].astype(np.complex128), mask), rtol=0, atol=1e-12)
    Y = _rand(rng, Nc, L, N, N)
    lhs = np.vdot(b, Y)
    rhs = np.vdot(X, cart.cart_adj_mc(Y, mask, S))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # full sampling with sum_c |S_c|^2 = 1: A^H A = I
    full = np.ones((L, N, N), np.uint8)
    np.testing.assert_allclose(cart.cart_adj_mc(cart.cart_fwd_mc(X, full, S), full, S), X, rtol=0, atol=1e-6)


def test_radial_mask_geometry():
    N, L = 64, 3
    m = mrfgen.radial_cartesian_mask(N, L, 8)
    assert m.dtype == np.uint8 and m.shape == (L, N, N)
    assert np.all(m[:, N // 2, N // 2] == 1)                        # every spoke passes the centre
    assert not np.array_equal(m[0], m[1])                           # frames rotate
    # each spoke covers a full diameter: at most 8 N points, at least N (one spoke)
    assert np.all(m.sum(axis=(1, 2)) <= 8 * N) and np.all(m.sum(axis=(1, 2)) >= N)
