"""Pins of the oracle's Algorithm 1."""
import math

import numpy as np

import mrfgen
from oracle import match, metrics, nufft, recon


def _tiny_dict(rng, L, M=6):
    D = rng.standard_normal((M, L)) + 1j * rng.standard_normal((M, L))
    lut = np.stack([np.linspace(300, 2000, M), np.linspace(40, 200, M)], 1)
    return D, lut


def test_landweber_special_case_converges_to_lstsq():
    """lambda1 = lambda2 = 0 and V = I reduce the loop to Landweber iteration."""
    rng = np.random.default_rng(1)
    N, L, Ns = 4, 2, 48                              # overdetermined: unique LS solution
    traj = rng.uniform(-math.pi, math.pi, (L, Ns, 2))
    b = rng.standard_normal((L, Ns)) + 1j * rng.standard_normal((L, Ns))
    D, lut = _tiny_dict(rng, L)
    # dense operator of frame l, then the min-norm least-squares solution per frame
    x_ls = []
    lam = 0.0
    for l in range(L):
        A = np.stack([nufft.nufft_fwd(e.reshape(1, N, N), traj[l:l + 1])[0] for e in np.eye(N * N)], 1)
        lam = max(lam, np.linalg.eigvalsh(A.conj().T @ A).max())
        x_ls.append(np.linalg.lstsq(A, b[l], rcond=None)[0].reshape(N, N))
    x_ls = np.stack(x_ls)
    out = recon.recon(b, traj, D, lut, np.eye(L), N, 2, 1, 2, 4, lam1_0=0.0, lam2=0.0,
                      mu0=1.0 / lam, lamA=lam, n_max=1500)
    assert np.linalg.norm(out["X"] - x_ls) <= 1e-6 * np.linalg.norm(x_ls)
    c = np.array(out["stats"]["cost"])
    assert np.all(np.diff(c) <= 1e-12 * c[0])


def test_fully_sampled_cartesian_noise_free_recovers_grid_tissues():
    """A is (to the KB error) unitary: X^0 = X and the match returns the true atoms."""
    rng = np.random.default_rng(2)
    N, L = 8, 12
    D, lut = _tiny_dict(rng, L, M=5)
    lab = rng.integers(0, 5, (N, N))
    pd = rng.uniform(0.5, 2.0, (N, N))
    X = (D[lab] * pd[..., None]).transpose(2, 0, 1)
    k = np.arange(N) - N // 2
    ky, kx = np.meshgrid(k, k, indexing="ij")
    traj = np.repeat(np.stack([2 * math.pi * kx.ravel() / N, 2 * math.pi * ky.ravel() / N], -1)[None], L, 0)
    b = nufft.nufft_fwd(X, traj)
    _, _, vh = np.linalg.svd(D / np.linalg.norm(D, axis=1, keepdims=True), full_matrices=False)
    out = recon.recon(b, traj, D, lut, vh.conj().T, N, 4, 2, 3, 4, n_max=0)
    assert np.linalg.norm(out["X"] - X) <= 2e-4 * np.linalg.norm(X)
    np.testing.assert_array_equal(out["idx"].reshape(N, N), lab)
    np.testing.assert_allclose(out["maps"][2], pd, rtol=1e-3)


def test_c1_small_recon_improves_on_the_initial_match():
    """Directional check at C1's shapes on a cropped phantom (not a parity test)."""
    cfg = mrfgen.get_config("C1", N=32, L=60, Ns=512)
    atoms, grid = mrfgen.make_dictionary(cfg)
    V, _ = mrfgen.subspace_basis(atoms, cfg["r"])
    ph = mrfgen.make_phantom(cfg, 0)
    X = mrfgen.truth_fingerprints(cfg, ph)
    traj = mrfgen.vds_spiral(cfg["N"], cfg["L"], cfg["Ns"], 12)
    b = nufft.nufft_fwd(X, traj)
    b = b + mrfgen.complex_noise(b.shape, mrfgen.noise_sigma(np.mean(np.abs(b) ** 2), 40.0), 11)
    x0 = mrfgen.complex_noise((cfg["L"], cfg["N"], cfg["N"]), 1.0, 5)
    lamA = nufft.operator_norm(traj, cfg["N"], x0, iters=20)
    out = recon.recon(b, traj, atoms, grid["lut"], V, cfg["N"], 4, 2, 8, 8, n_max=6, lamA=lamA)
    init = match.match_subspace(nufft.nufft_adj(b, traj, cfg["N"]), atoms, grid["lut"], V)
    m = ph["mask"]
    e0 = metrics.nmse(ph["T1"], init[3][:, 0].reshape(32, 32), m)
    e1 = metrics.nmse(ph["T1"], out["maps"][0], m)
    assert e1 < e0
    assert metrics.snr_db(X, out["X"]) > metrics.snr_db(X, nufft.nufft_adj(b, traj, cfg["N"]))
