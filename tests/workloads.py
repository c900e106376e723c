"""Seeded synthetic workloads for the tests (inputs from mrfgen; measurements by the oracle's A)."""
import functools

import numpy as np

import mrfgen
from oracle import nufft as onufft


@functools.lru_cache(maxsize=4)
def c1_workload(seed=0, N=None, L=None, Ns=None, n_int=None):
    """C1 shapes (or a cropped variant): dictionary, basis, phantom, X_true, traj, noisy b, lamA."""
    over = {k: v for k, v in dict(N=N, L=L, Ns=Ns).items() if v is not None}
    cfg = mrfgen.get_config("C1", **over)
    atoms, grid = mrfgen.make_dictionary(cfg)
    V, _ = mrfgen.subspace_basis(atoms, cfg["r"])
    ph = mrfgen.make_phantom(cfg, seed)
    X = mrfgen.truth_fingerprints(cfg, ph)
    traj = mrfgen.vds_spiral(cfg["N"], cfg["L"], cfg["Ns"], n_int or cfg["n_interleaves"])
    b_clean = onufft.nufft_fwd(X, traj)
    sig2 = mrfgen.noise_sigma(np.mean(np.abs(b_clean) ** 2), cfg["snr_db"])
    b = (b_clean + mrfgen.complex_noise(b_clean.shape, sig2, seed + 101)).astype(np.complex64)
    x0 = mrfgen.complex_noise((cfg["L"], cfg["N"], cfg["N"]), 1.0, seed + 202)
    lamA = onufft.operator_norm(traj, cfg["N"], x0, iters=20)
    return dict(cfg=cfg, atoms=atoms, grid=grid, V=V, phantom=ph, X=X, traj=traj, b=b, lamA=lamA)


def random_maps(rng, N, zero_frac=0.0):
    maps = np.stack([rng.uniform(300, 2500, (N, N)), rng.uniform(40, 300, (N, N)), rng.uniform(0, 100, (N, N))])
    if zero_frac > 0:
        maps[:, rng.uniform(size=(N, N)) < zero_frac] = 0.0
    return maps.astype(np.float32)


def c2_workload(seed=0):
    """The 256 x 256, L = 1000 workload: C2 dictionary and basis, smooth phantom, truth series,
    VDS spiral (1 of 48 interleaves, 2048 samples), b = the oracle's A X + 40 dB noise."""
    cfg = mrfgen.get_config("C2")
    atoms, grid = mrfgen.make_dictionary(cfg)
    V, _ = mrfgen.subspace_basis(atoms, cfg["r"])
    ph = mrfgen.make_phantom(cfg, seed)
    X = mrfgen.truth_fingerprints(cfg, ph)
    traj = mrfgen.vds_spiral(cfg["N"], cfg["L"], cfg["Ns"], cfg["n_interleaves"])
    b_clean = onufft.nufft_fwd(X, traj)
    sig2 = mrfgen.noise_sigma(np.mean(np.abs(b_clean) ** 2), cfg["snr_db"])
    b = (b_clean + mrfgen.complex_noise(b_clean.shape, sig2, seed + 17)).astype(np.complex64)
    return dict(cfg=cfg, atoms=atoms, grid=grid, V=V, phantom=ph, X=X, traj=traj, b=b)


@functools.lru_cache(maxsize=2)
def mc_workload(seed=0, N=32, L=60, Ns=512, ncoils=4):
    """A cropped C1 acquired by ncoils coils (eq. (1)): b_c = the oracle's A (S_c X) + 40 dB noise;
    lamA = lambda_max of the multi-coil normal operator (oracle power iteration)."""
    cfg = mrfgen.get_config("C1", N=N, L=L, Ns=Ns)
    atoms, grid = mrfgen.make_dictionary(cfg)
    V, _ = mrfgen.subspace_basis(atoms, cfg["r"])
    ph = mrfgen.make_phantom(cfg, seed)
    X = mrfgen.truth_fingerprints(cfg, ph)
    traj = mrfgen.vds_spiral(N, L, Ns, cfg["n_interleaves"])
    S = mrfgen.coil_maps(N, ncoils, seed)
    b_clean = onufft.nufft_fwd_mc(X, traj, S)
    sig2 = mrfgen.noise_sigma(np.mean(np.abs(b_clean) ** 2), cfg["snr_db"])
    b = (b_clean + mrfgen.complex_noise(b_clean.shape, sig2, seed + 31)).astype(np.complex64)
    x0 = mrfgen.complex_noise((L, N, N), 1.0, seed + 37)
    lamA = onufft.operator_norm_mc(traj, N, S, x0, iters=20)
    return dict(cfg=cfg, atoms=atoms, grid=grid, V=V, phantom=ph, X=X, traj=traj, smaps=S, b=b, lamA=lamA)


@functools.lru_cache(maxsize=2)
def cart_workload(seed=0, N=64, L=100, n_spokes=4):
    """A cropped C1 under pseudo-radial Cartesian sampling (about 6% of k-space per frame at
    N = 64 with 4 spokes): b = the oracle's M F X + 40 dB noise on the sampled points (dense
    [L, N, N], zero elsewhere); lamA = 1 (F is unitary and M a projection)."""
    from oracle import cartesian as ocart
    cfg = mrfgen.get_config("C1", N=N, L=L)
    atoms, grid = mrfgen.make_dictionary(cfg)
    V, _ = mrfgen.subspace_basis(atoms, cfg["r"])
    ph = mrfgen.make_phantom(cfg, seed)
    X = mrfgen.truth_fingerprints(cfg, ph)
    mask = mrfgen.radial_cartesian_mask(N, L, n_spokes)
    b_clean = ocart.cart_fwd(X, mask)
    sig2 = mrfgen.noise_sigma(np.sum(np.abs(b_clean) ** 2) / mask.sum(), cfg["snr_db"])
    b = (b_clean + mask * mrfgen.complex_noise(b_clean.shape, sig2, seed + 41)).astype(np.complex64)
    return dict(cfg=cfg, atoms=atoms, grid=grid, V=V, phantom=ph, X=X, mask=mask, b=b, lamA=1.0)
