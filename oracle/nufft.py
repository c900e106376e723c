"""Oracle: the acquisition operator of eq. (1), single-coil A = F_u and multi-coil A = F_u C, and
their adjoints.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Definition (the exact operator). For frame l with image X_l in C^{N x N} (row y,
column x) and trajectory samples omega_{l,j} = (omega_x, omega_y) in rad/pixel,
    b_l[j] = (1/N) sum_{y,x} X_l[y, x] exp(-i (omega_x (x - N/2) + omega_y (y - N/2)))
(orthonormal 1/sqrt(N*N) scaling, centre at N/2). `nudft_fwd` writes this out.

Method (approximates it): Kaiser-Bessel gridding on the oversampled G x G grid,
G = osf * N, width W (Jackson et al. 1991; beta of Beatty et al. 2005):
  1. a = X / (phi_hat(y'/G) phi_hat(x'/G)), x' = x - N/2  (deapodisation)
  2. place a at grid index (y' mod G, x' mod G) and take the G x G DFT (numpy.fft.fft2)
  3. b[j] = (1/N) sum over the W x W taps k of phi(u_y - k_y) phi(u_x - k_x) grid[k mod G],
     u = omega G / (2 pi), taps k = floor(u) - W/2 + 1, ..., floor(u) + W/2
with phi(t) = I0(beta sqrt(1 - (2t/W)^2)) for |t| <= W/2 and its Fourier transform
phi_hat(s) = W sinh(sqrt(beta^2 - (pi W s)^2)) / sqrt(beta^2 - (pi W s)^2).
`nufft_adj` is the exact adjoint of `nufft_fwd` (spread with the same real weights,
inverse DFT times G^2, crop, deapodise, scale 1/N).

Pins: brute-force NUDFT on tiny grids, the adjoint identity, the full Cartesian
special case against numpy's orthonormal FFT, the I0 series against scipy, and the
closed-form phi_hat against numerical quadrature (tests/test_oracle_nufft.py); for the
multi-coil pair, a dense brute-force stack of NUDFT diag(S_c) blocks, its adjoint identity,
the single-coil reduction (one coil of sensitivity 1), and A^H A = I for full Cartesian
sampling with sum_c |S_c|^2 = 1.
"""
import math

import numpy as np


def kb_beta(W, osf):
    """Beatty et al. (2005) shape parameter for width W and oversampling osf."""
    return math.pi * math.sqrt((W / osf) ** 2 * (osf - 0.5) ** 2 - 0.8)


def bessel_i0(z):
    """Modified Bessel function I0 by its power series sum_k (z/2)^{2k} / (k!)^2."""
    z = np.asarray(z, np.float64)
    q = (z / 2.0) ** 2
    term = np.ones_like(z)
    total = np.ones_like(z)
    for k in range(1, 200):
        term = term * q / (k * k)
        total = total + term
        if np.all(term <= 1e-18 * total):
            break
    return total


def kb_kernel(t, W, beta):
    """phi(t) = I0(beta sqrt(1 - (2t/W)^2)) on |t| <= W/2, zero outside."""
    t = np.asarray(t, np.float64)
    arg = 1.0 - (2.0 * t / W) ** 2
    inside = arg >= 0.0
    val = bessel_i0(beta * np.sqrt(np.where(inside, arg, 0.0)))
    return np.where(inside, val, 0.0)


def kb_ft(s, W, beta):
    """Fourier transform of phi at frequency s (cycles per grid cell)."""
    s = np.asarray(s, np.float64)
    a = beta ** 2 - (math.pi * W * s) ** 2
    out = np.empty_like(s)
    pos = a > 0
    ra = np.sqrt(np.abs(a))
    out[pos] = W * np.sinh(ra[pos]) / ra[pos]
    neg = a < 0
    out[neg] = W * np.sin(ra[neg]) / ra[neg]
    out[a == 0] = W
    return out


def deapod(N, G, W, beta):
    """phi_hat((x - N/2) / G) for x = 0..N-1 (the same vector serves rows and columns)."""
    xc = np.arange(N) - N // 2
    return kb_ft(xc / G, W, beta)


def _taps(u, W):
    """Integer tap positions [n, W] (unwrapped) and kernel arguments u - k."""
    base = np.floor(u).astype(np.int64) - W // 2 + 1
    k = base[:, None] + np.arange(W)[None, :]
    return k, u[:, None] - k


def _weights(traj_l, G, W, beta):
    ux = traj_l[:, 0].astype(np.float64) * G / (2 * math.pi)
    uy = traj_l[:, 1].astype(np.float64) * G / (2 * math.pi)
    kx, dx = _taps(ux, W)
    ky, dy = _taps(uy, W)
    return np.mod(kx, G), kb_kernel(dx, W, beta), np.mod(ky, G), kb_kernel(dy, W, beta)


def nufft_fwd(X, traj, osf=2, W=6):
    """b = A X by KB gridding. X [L, N, N] complex, traj [L, Ns, 2] -> b [L, Ns] complex128."""
    X = np.asarray(X, np.complex128)
    L, N, _ = X.shape
    G = int(osf * N)
    beta = kb_beta(W, osf)
    d = deapod(N, G, W, beta)
    rows = np.mod(np.arange(N) - N // 2, G)
    Ns = traj.shape[1]
    b = np.empty((L, Ns), np.complex128)
    for l in range(L):
        grid = np.zeros((G, G), np.complex128)
        grid[np.ix_(rows, rows)] = X[l] / (d[:, None] * d[None, :])
        F = np.fft.fft2(grid)
        kx, wx, ky, wy = _weights(traj[l], G, W, beta)
        acc = np.zeros(Ns, np.complex128)
        for iy in range(W):
            for ix in range(W):
                acc += wy[:, iy] * wx[:, ix] * F[ky[:, iy], kx[:, ix]]
        b[l] = acc / N
    return b


def nufft_adj(b, traj, N, osf=2, W=6):
    """X = A^H b, the exact adjoint of nufft_fwd. b [L, Ns] -> X [L, N, N] complex128."""
    b = np.asarray(b, np.complex128)
    L, Ns = b.shape
    G = int(osf * N)
    beta = kb_beta(W, osf)
    d = deapod(N, G, W, beta)
    rows = np.mod(np.arange(N) - N // 2, G)
    X = np.empty((L, N, N), np.complex128)
    for l in range(L):
        kx, wx, ky, wy = _weights(traj[l], G, W, beta)
        H = np.zeros((G, G), np.complex128)
        for iy in range(W):
            for ix in range(W):
                np.add.at(H, (ky[:, iy], kx[:, ix]), wy[:, iy] * wx[:, ix] * b[l])
        a = np.fft.ifft2(H) * (G * G)
        X[l] = a[np.ix_(rows, rows)] / (d[:, None] * d[None, :]) / N
    return X


def nudft_matrix(traj_l, N):
    """Dense matrix of the exact operator for one frame: [Ns, N*N] (row-major y, x)."""
    yy, xx = np.mgrid[0:N, 0:N]
    xc = (xx - N // 2).ravel().astype(np.float64)
    yc = (yy - N // 2).ravel().astype(np.float64)
    wx = traj_l[:, 0].astype(np.float64)
    wy = traj_l[:, 1].astype(np.float64)
    return np.exp(-1j * (np.outer(wx, xc) + np.outer(wy, yc))) / N


def nudft_fwd(X, traj):
    """Exact A X by the dense definition (for small sizes)."""
    X = np.asarray(X, np.complex128)
    L, N, _ = X.shape
    return np.stack([nudft_matrix(traj[l], N) @ X[l].ravel() for l in range(L)])


def operator_norm(traj, N, x0, iters=30, osf=2, W=6):
    """lambda_max(A^H A) by power iteration from the given start x0 [L, N, N].

    The step-size rule needs this bound; the start vector is an input so that the
    oracle draws no random numbers of its own.
    """
    x = np.asarray(x0, np.complex128)
    x = x / np.linalg.norm(x)
    lam = 0.0
    for _ in range(iters):
        y = nufft_adj(nufft_fwd(x, traj, osf, W), traj, N, osf, W)
        lam = float(np.vdot(x, y).real)
        x = y / np.linalg.norm(y)
    return lam


# ---------------------------------------------------------------- multi-coil acquisition
# Eq. (1) with coil sensitivities: the acquisition is A = F_u C, where C stacks the coils'
# pixel-wise sensitivity maps S_c and F_u is the single-coil operator above applied to every
# coil image: b_c = F_u (S_c X). Its adjoint combines the coils: A^H b = sum_c conj(S_c) F_u^H b_c.

def nufft_fwd_mc(X, traj, smaps, osf=2, W=6):
    """b [Nc, L, Ns] with b_c = A (S_c X); smaps [Nc, N, N] complex."""
    X = np.asarray(X, np.complex128)
    return np.stack([nufft_fwd(X * np.asarray(S, np.complex128)[None], traj, osf, W) for S in smaps])


def nufft_adj_mc(b, traj, N, smaps, osf=2, W=6):
    """X = sum_c conj(S_c) A^H b_c, the exact adjoint of nufft_fwd_mc; b [Nc, L, Ns]."""
    b = np.asarray(b, np.complex128)
    out = None
    for c, S in enumerate(smaps):
        term = np.conj(np.asarray(S, np.complex128))[None] * nufft_adj(b[c], traj, N, osf, W)
        out = term if out is None else out + term
    return out


def operator_norm_mc(traj, N, smaps, x0, iters=30, osf=2, W=6):
    """lambda_max(A^H A) of the multi-coil operator by power iteration from x0 [L, N, N]."""
    x = np.asarray(x0, np.complex128)
    x = x / np.linalg.norm(x)
    lam = 0.0
    for _ in range(iters):
        y = nufft_adj_mc(nufft_fwd_mc(x, traj, smaps, osf, W), traj, N, smaps, osf, W)
        lam = float(np.vdot(x, y).real)
        x = y / np.linalg.norm(y)
    return lam
