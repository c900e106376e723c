"""Synthetic receive-coil sensitivities for the multi-coil acquisition of eq. (1).

Nc coils sit on a ring around the field of view (radius 0.75 N from the centre, evenly spaced
from a seeded start angle). A coil's magnitude falls off smoothly with distance from it,
1 / (1 + (d / (0.5 N))^2), and its phase is a smooth seeded linear ramp plus a constant. The maps
are then normalised pixel by pixel so that sum_c |S_c|^2 = 1 (the usual normalisation of coil
sensitivities). An input of the method, like the trajectory: none of its arithmetic.
"""
import numpy as np


def coil_maps(N, ncoils, seed=0):
    """[ncoils, N, N] complex64 sensitivities with sum_c |S_c|^2 = 1 at every pixel."""
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:N, 0:N].astype(np.float64)
    yc, xc = yy - (N - 1) / 2.0, xx - (N - 1) / 2.0
    start = rng.uniform(0.0, 2.0 * np.pi)
    maps = []
    for c in range(ncoils):
        ang = start + 2.0 * np.pi * c / ncoils
        cy, cx = 0.75 * N * np.sin(ang), 0.75 * N * np.cos(ang)
        d2 = (yc - cy) ** 2 + (xc - cx) ** 2
        mag = 1.0 / (1.0 + d2 / (0.5 * N) ** 2)
        gy, gx = rng.uniform(-1.0, 1.0, 2) * np.pi / N
        phase = gy * yc + gx * xc + rng.uniform(0.0, 2.0 * np.pi)
        maps.append(mag * np.exp(1j * phase))
    S = np.stack(maps)
    S /= np.sqrt(np.sum(np.abs(S) ** 2, axis=0))[None]
    return S.astype(np.complex64)
