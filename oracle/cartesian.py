"""Oracle: the Cartesian acquisition of eq. (1) for pseudo-radial Cartesian sampling (Sec. IV,
the third sampling pattern), A_l X_l = M_l (F X_l), single- and multi-coil, and the adjoints.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Definition. F is the exact operator of oracle.nufft with every sample on the integer grid: the
k-space point at row ky + N/2, column kx + N/2 (kx, ky in [-N/2, N/2)) holds
    (F X)[ky + N/2, kx + N/2] = (1/N) sum_{y,x} X[y, x] exp(-2 pi i (kx (x - N/2) + ky (y - N/2)) / N),
the unitary centred 2D DFT. M_l keeps the frame's sampled grid points and zeroes the others, so the
measurements are a dense [L, N, N] array, zero where M_l is. The adjoint is F^H M_l.

Method: numpy's orthonormal FFT between two half-length circular shifts (a library primitive).

Pins (tests/test_oracle_cartesian.py): a dense DFT matrix written from the definition on tiny
grids; oracle.nufft's gridded operator at the same grid frequencies (to its KB error); the adjoint
identity; A^H A = I under full sampling; the multi-coil stack against the single-coil operator.
"""
import numpy as np


def _F(X):
    return np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(X, axes=(-2, -1)), norm="ortho"), axes=(-2, -1))


def _FH(K):
    return np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(K, axes=(-2, -1)), norm="ortho"), axes=(-2, -1))


def cart_fwd(X, mask):
    """b [L, N, N] = M_l F X_l; X [L, N, N], mask [L, N, N] (0/1)."""
    return np.asarray(mask, np.float64) * _F(np.asarray(X, np.complex128))


def cart_adj(b, mask):
    """X [L, N, N] = F^H (M_l b_l), the adjoint of cart_fwd."""
    return _FH(np.asarray(mask, np.float64) * np.asarray(b, np.complex128))


def cart_fwd_mc(X, mask, smaps):
    """b [Nc, L, N, N] with b_c = M F (S_c X)."""
    X = np.asarray(X, np.complex128)
    return np.stack([cart_fwd(X * np.asarray(S, np.complex128)[None], mask) for S in smaps])


def cart_adj_mc(b, mask, smaps):
    """X = sum_c conj(S_c) F^H M b_c, the adjoint of cart_fwd_mc."""
    out = None
    for c, S in enumerate(smaps):
        term = np.conj(np.asarray(S, np.complex128))[None] * cart_adj(b[c], mask)
        out = term if out is None else out + term
    return out


def dft_matrix(N):
    """Dense [N*N, N*N] matrix of F from the definition (row-major (ky, kx) and (y, x))."""
    k = np.arange(N) - N // 2
    x = np.arange(N) - N // 2
    E = np.exp(-2j * np.pi * np.outer(k, x) / N)            # [k, x]
    return np.kron(E, E) / N
