"""Oracle: the normal operator A^H A of the gradient in eq. (15) as a convolution (Toeplitz form).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Definition. For frame l, (A^H A X)[v] = sum_{v'} K_l[v - v'] X[v'] with the point-spread kernel
    K_l[d] = (1/N^2) sum_j exp(i (omega_x d_x + omega_y d_y)),   d in (-N, N)^2,
since the centre offsets of A and A^H cancel. A linear convolution of an N x N image with a kernel
of extent 2N - 1 equals a circular one on a 2N x 2N grid once the image is zero-padded and the
kernel stored at (d mod 2N): no output inside the N x N window wraps. So
    A^H A X = crop( IFFT_2N( FFT_2N(K~) * FFT_2N(pad X) ) ).
The offsets d_x = -N or d_y = -N never occur (|d| <= N - 1) and are set to zero; K~ is then
Hermitian (K[-d] = conj K[d]) and FFT_2N(K~) real.

Method. K~ from the gridded adjoint on a 2N image of the same samples (oracle.nufft, the same KB
method the gradient's A^H uses): adjoint of all-ones data on a 2N x 2N image gives
(1/(2N)) sum_j exp(i omega . (v - N)) = (N/2) K[v - N]. With the cost of Algorithm 1 written
through it, 0.5 ||A X - b||^2 = 0.5 <X, A^H A X> - Re <X, A^H b> + 0.5 ||b||^2.

Pins (tests/test_oracle_toeplitz.py): the exact kernel written as the sum above; the dense A^H A
of the exact NUDFT matrix (to the KB error); oracle.nufft's own adjoint of its forward (to the KB
error); Hermitian and positive semidefinite; the cost identity.
"""
import numpy as np

from . import nufft


def psf_circulant(traj, N, osf=2, W=6):
    """K~ [L, 2N, 2N] with K~[d mod 2N] = K[d], from the gridded adjoint on a 2N image."""
    L, Ns, _ = traj.shape
    img = (2.0 / N) * nufft.nufft_adj(np.ones((L, Ns)), traj, 2 * N, osf, W)   # index v <-> d = v - N
    img[:, 0, :] = 0.0                                                   # d_y = -N
    img[:, :, 0] = 0.0                                                   # d_x = -N
    return np.roll(img, shift=(-N, -N), axis=(1, 2))                    # position d mod 2N


def psf_exact(traj_l, N):
    """K~ [2N, 2N] of one frame by the defining sum (small sizes)."""
    d = np.arange(2 * N) - N
    wx = np.asarray(traj_l[:, 0], np.float64)
    wy = np.asarray(traj_l[:, 1], np.float64)
    ex = np.exp(1j * np.outer(wx, d))                                    # [Ns, 2N] over d_x
    ey = np.exp(1j * np.outer(wy, d))
    K = (ey.T @ ex) / (N * N)                                           # [d_y, d_x]
    K[0, :] = 0.0
    K[:, 0] = 0.0
    return np.roll(K, shift=(-N, -N), axis=(0, 1))


def kernel_spectrum(Kt):
    """FFT_2N of K~ per frame (complex; its imaginary part is rounding)."""
    return np.fft.fft2(np.asarray(Kt, np.complex128), axes=(-2, -1))


def toeplitz_normal(X, Khat):
    """A^H A X [L, N, N] through the circulant embedding; Khat [L, 2N, 2N] from kernel_spectrum."""
    X = np.asarray(X, np.complex128)
    L, N, _ = X.shape
    P = np.zeros((L, 2 * N, 2 * N), np.complex128)
    P[:, :N, :N] = X
    Y = np.fft.ifft2(Khat * np.fft.fft2(P, axes=(-2, -1)), axes=(-2, -1))
    return Y[:, :N, :N]


def data_term(X, TX, AHb, bnorm2):
    """0.5 ||A X - b||^2 = 0.5 <X, A^H A X> - Re <X, A^H b> + 0.5 ||b||^2."""
    X = np.asarray(X, np.complex128)
    return 0.5 * float(np.vdot(X, TX).real) - float(np.vdot(X, AHb).real) + 0.5 * float(bnorm2)
