"""Variable-density spiral sampling (Sec. IV-A; one interleave per frame).

k(tau) = k_max * tau^alpha * exp(i 2 pi n_t tau), tau in [0, 1), with n_t chosen so
that n_interleaves rotated copies meet Nyquist (2 pi / N rad/pixel) at k_max. Frame l
is rotated by l times the golden angle pi (3 - sqrt 5). Coordinates are in rad/pixel
and lie in [-pi, pi).
"""
import numpy as np

GOLDEN = np.pi * (3.0 - np.sqrt(5.0))


def vds_spiral(N, L, Ns, n_interleaves, alpha=1.5, interleaves_per_frame=1, frame0=0):
    """Return traj float32 [L, Ns * interleaves_per_frame, 2] with (omega_x, omega_y)."""
    kmax = np.pi * (1.0 - 1e-4)
    n_turns = alpha * N / (2.0 * n_interleaves)
    tau = np.arange(Ns, dtype=np.float64) / Ns
    base = kmax * tau ** alpha * np.exp(2j * np.pi * n_turns * tau)
    out = np.empty((L, Ns * interleaves_per_frame, 2), np.float32)
    for l in range(L):
        segs = []
        for i in range(interleaves_per_frame):
            ang = (frame0 + l) * GOLDEN + i * 2.0 * np.pi / n_interleaves
            segs.append(base * np.exp(1j * ang))
        k = np.concatenate(segs)
        out[l, :, 0] = k.real
        out[l, :, 1] = k.imag
    return out


def radial_cartesian_mask(N, L, n_spokes, frame0=0):
    """Pseudo-radial Cartesian sampling (Sec. IV, the third sampling pattern): per frame, n_spokes
    lines through the k-space centre at angles j pi / n_spokes plus the frame's golden-angle
    rotation, each traced at unit steps over [-N/2, N/2) and rounded to the nearest point of the
    N x N Cartesian grid. Returns uint8 [L, N, N]; entry [l, ky + N/2, kx + N/2] is 1 where
    frequency (kx, ky) (cycles per field of view) is sampled in frame l."""
    mask = np.zeros((L, N, N), np.uint8)
    t = np.arange(-N // 2, N // 2, dtype=np.float64)
    for l in range(L):
        for j in range(n_spokes):
            ang = j * np.pi / n_spokes + (frame0 + l) * GOLDEN
            kx = np.clip(np.rint(t * np.cos(ang)), -N // 2, N // 2 - 1).astype(np.int64)
            ky = np.clip(np.rint(t * np.sin(ang)), -N // 2, N // 2 - 1).astype(np.int64)
            mask[l, ky + N // 2, kx + N // 2] = 1
    return mask
