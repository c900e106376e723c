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


def _landweber_problem(seed=1, N=4, L=2, Ns=48):
    rng = np.random.default_rng(seed)
    traj = rng.uniform(-math.pi, math.pi, (L, Ns, 2))
    b = rng.standard_normal((L, Ns)) + 1j * rng.standard_normal((L, Ns))
    A = [np.stack([nufft.nufft_fwd(e.reshape(1, N, N), traj[l:l + 1])[0] for e in np.eye(N * N)], 1)
         for l in range(L)]
    lam = max(np.linalg.eigvalsh(a.conj().T @ a).max() for a in A)
    return rng, traj, b, A, lam


def test_stopping_rule_of_algorithm_1():
    """Algorithm 1 stops after the first iteration n with cost(n-1)/cost(n) - 1 < tol. With
    lambda1 = lambda2 = 0 and V = I the iterates are Landweber's, whose costs are computed here
    from the dense frame operators; tol is placed so that the printed ratio and the variant
    1 - cost(n)/cost(n-1) stop at different iterations, and the recon must follow the former."""
    rng, traj, b, A, lam = _landweber_problem()
    N, L = 4, 2
    mu = 1.0 / lam
    x = [a.conj().T @ b[l] for l, a in enumerate(A)]
    cost = []
    for n in range(60):
        r = [A[l] @ x[l] - b[l] for l in range(L)]
        cost.append(0.5 * sum(np.vdot(v, v).real for v in r))
        x = [x[l] - mu * (A[l].conj().T @ r[l]) for l in range(L)]
    cost = np.array(cost)
    ratio = cost[:-1] / cost[1:] - 1.0          # index n-1 holds the test after iteration n
    alt = 1.0 - cost[1:] / cost[:-1]
    assert np.all(np.diff(cost) < 0)
    # tol between the two forms at some iteration k, so they stop at different n
    tol = None
    for k in range(3, 40):
        t = 0.5 * (ratio[k] + alt[k])
        n_paper = 1 + int(np.argmax(ratio < t))
        n_alt = 1 + int(np.argmax(alt < t))
        if n_paper != n_alt and np.any(ratio < t):
            tol = t
            break
    assert tol is not None
    D, lut = _tiny_dict(rng, L)
    out = recon.recon(b, traj, D, lut, np.eye(L), N, 2, 1, 2, 4, lam1_0=0.0, lam2=0.0, mu0=mu, lamA=lam,
                      n_max=200, tol=tol)
    st = out["stats"]
    assert st["stop"] == "tolerance"
    assert st["iters"] == n_paper != n_alt
    np.testing.assert_allclose(st["cost"], cost[:n_paper + 1], rtol=1e-10)
    # without a tolerance all n_max iterations run
    out = recon.recon(b, traj, D, lut, np.eye(L), N, 2, 1, 2, 4, lam1_0=0.0, lam2=0.0, mu0=mu, lamA=lam,
                      n_max=n_paper + 3, tol=None)
    assert out["stats"]["iters"] == n_paper + 3 and out["stats"]["stop"] == "max_iter"


def _dense_SL(N, p, s, Lap):
    """The pixel operator S_L X = Q*(Q(X) L) of one frame as a dense N^2 x N^2 matrix."""
    from oracle import ops
    cols = [ops.laplacian_apply(e.reshape(1, N, N), Lap, p, s)[0].ravel() for e in np.eye(N * N)]
    return np.stack(cols, 1).real


def test_step_size_bounds_the_gradient_lipschitz_constant():
    """The step of reading Q9: mu = min(mu0, 1/(lamA + 2 c_max lambda1 max(L))) must not exceed
    1/lambda_max(A^H A + lambda1 S_L), the gradient's Lipschitz constant for eq. (15).
    (1) Random K-NN graphs with overlapping 4x4 patches and the dense NUFFT of a frame: the bound
        holds.
    (2) p = s (Q unitary) and one edge of weight w between two patches: lambda_max(S_L) = 2w =
        2 max(L) exactly, so with A^H A = eps I the bound is attained: mu lambda_max = 1.
    (3) 2x2 patches at stride 1 on a 3x3 image (coverage 4 at the centre), all four patches joined
        with weight w: a unit image at the centre has Rayleigh quotient sum_i L_ii = 12 w =
        c_max max(L), so the factor c_max is needed for the bound to hold."""
    from oracle import graph, patches
    # (1)
    rng = np.random.default_rng(3)
    N, p, s = 8, 4, 2
    traj = rng.uniform(-math.pi, math.pi, (1, 40, 2))
    A = np.stack([nufft.nufft_fwd(e.reshape(1, N, N), traj)[0] for e in np.eye(N * N)], 1)
    AhA = A.conj().T @ A
    lamA = np.linalg.eigvalsh(AhA).max()
    cmax = float(patches.coverage(N, p, s).max())
    assert cmax == 4.0
    for K in (1, 3, 8):
        maps = np.stack([rng.uniform(300, 2500, (N, N)), rng.uniform(40, 300, (N, N)), rng.uniform(0, 100, (N, N))])
        g = graph.knn_laplacian(maps, p, s, K)
        for lam1_0 in (0.01, 1.0, 100.0):
            lam1 = lam1_0 * g["lmax"]
            H = AhA + lam1 * _dense_SL(N, p, s, g["L"])
            mu = recon.step_size(10.0, lamA, lam1, g["lmax"], cmax)
            assert mu * np.linalg.eigvalsh(H).max() <= 1.0 + 1e-12
    # (2)
    w, eps = 0.7, 1e-3
    Lap = np.zeros((4, 4))
    Lap[0, 0] = Lap[1, 1] = w
    Lap[0, 1] = Lap[1, 0] = -w
    H = eps * np.eye(16) + 5.0 * _dense_SL(4, 2, 2, Lap)
    mu = recon.step_size(10.0, eps, 5.0, w, 1.0)
    assert abs(mu * np.linalg.eigvalsh(H).max() - 1.0) <= 1e-12
    # (3)
    assert patches.coverage(3, 2, 1).max() == 4.0
    Lap = w * (4.0 * np.eye(4) - np.ones((4, 4)))
    SL = _dense_SL(3, 2, 1, Lap)
    e = np.zeros(9)
    e[4] = 1.0
    assert abs(e @ SL @ e - 4 * 3 * w) <= 1e-12
    H = eps * np.eye(9) + 5.0 * SL
    mu = recon.step_size(10.0, eps, 5.0, 3 * w, 4.0)
    assert mu * np.linalg.eigvalsh(H).max() <= 1.0 + 1e-12


def test_multicoil_landweber_converges_to_the_stacked_lstsq():
    """Eq. (1) with coils and lambda1 = lambda2 = 0, V = I: the loop is Landweber iteration on the
    stacked system [A diag(S_1); ...; A diag(S_Nc)] x_l = [b_1l; ...; b_Nc,l], whose least-squares
    solution is formed here from the single-coil operator's columns and the maps by hand."""
    rng = np.random.default_rng(3)
    N, L, Ns, Nc = 4, 2, 9, 3                        # 27 rows per frame for 16 unknowns
    traj = rng.uniform(-math.pi, math.pi, (L, Ns, 2))
    S = rng.standard_normal((Nc, N, N)) + 1j * rng.standard_normal((Nc, N, N))
    b = rng.standard_normal((Nc, L, Ns)) + 1j * rng.standard_normal((Nc, L, Ns))
    D, lut = _tiny_dict(rng, L)
    x_ls, lam = [], 0.0
    for l in range(L):
        A = np.stack([nufft.nufft_fwd(e.reshape(1, N, N), traj[l:l + 1])[0] for e in np.eye(N * N)], 1)
        M = np.concatenate([A * S[c].ravel()[None, :] for c in range(Nc)])
        lam = max(lam, np.linalg.eigvalsh(M.conj().T @ M).max())
        x_ls.append(np.linalg.lstsq(M, b[:, l].ravel(), rcond=None)[0].reshape(N, N))
    x_ls = np.stack(x_ls)
    out = recon.recon(b, traj, D, lut, np.eye(L), N, 2, 1, 2, 4, lam1_0=0.0, lam2=0.0,
                      mu0=1.0 / lam, lamA=lam, n_max=3000, smaps=S)
    assert np.linalg.norm(out["X"] - x_ls) <= 1e-6 * np.linalg.norm(x_ls)
    c = np.array(out["stats"]["cost"])
    assert np.all(np.diff(c) <= 1e-12 * c[0])


def test_two_equal_coils_reduce_to_one():
    """S_1 = S_2 = 1/sqrt(2) with b_1 = b_2 = b/sqrt(2): the data term and its gradient are the
    single-coil ones, so the whole run (graph, costs, X) is the single-coil run."""
    cfg = mrfgen.get_config("C1", N=32, L=40, Ns=256)
    atoms, grid = mrfgen.make_dictionary(cfg)
    V, _ = mrfgen.subspace_basis(atoms, cfg["r"])
    X = mrfgen.truth_fingerprints(cfg, mrfgen.make_phantom(cfg, 0))
    traj = mrfgen.vds_spiral(cfg["N"], cfg["L"], cfg["Ns"], cfg["n_interleaves"])
    b = nufft.nufft_fwd(X, traj)
    b = b + 0.01 * np.abs(b).mean() * np.random.default_rng(4).standard_normal(b.shape)
    S = np.full((2, cfg["N"], cfg["N"]), 1 / math.sqrt(2))
    kw = dict(lam1_0=0.1, lam2=0.05, beta=0.2, mu0=0.5, n_max=2)
    one = recon.recon(b, traj, atoms, grid["lut"], V, cfg["N"], 4, 2, 6, 6, **kw)
    two = recon.recon(np.stack([b, b]) / math.sqrt(2), traj, atoms, grid["lut"], V, cfg["N"], 4, 2, 6, 6,
                      smaps=S, **kw)
    np.testing.assert_allclose(two["stats"]["cost"], one["stats"]["cost"], rtol=1e-10)
    assert np.linalg.norm(two["X"] - one["X"]) <= 1e-10 * np.linalg.norm(one["X"])
    assert np.array_equal(two["idx"], one["idx"])


def test_cartesian_fully_sampled_recon_is_the_truth():
    """Full Cartesian sampling (every mask entry 1): A = F is unitary, so X^0 = A^H b = X exactly
    and, with the manifold and LLR terms off and mu = 1, X^1 = X too; the match then returns the
    true atoms (truth built from grid atoms)."""
    rng = np.random.default_rng(5)
    N, L = 8, 12
    D = rng.standard_normal((5, L)) + 1j * rng.standard_normal((5, L))
    lut = np.stack([np.linspace(300, 2000, 5), np.linspace(40, 200, 5)], 1)
    k = rng.integers(0, 5, (N, N))
    X = np.moveaxis(D[k] * rng.uniform(0.5, 2.0, (N, N, 1)), -1, 0)
    mask = np.ones((L, N, N), np.uint8)
    from oracle import cartesian
    b = cartesian.cart_fwd(X, mask)
    u, s_, vh = np.linalg.svd(D, full_matrices=False)
    out = recon.recon(b, None, D, lut, vh.conj().T, N, 4, 2, 3, 4, lam1_0=0.0, lam2=0.0, mu0=1.0, lamA=1.0,
                      n_max=1, mask=mask)
    np.testing.assert_allclose(out["X"], X, rtol=0, atol=1e-10)
    assert np.array_equal(out["idx"].reshape(N, N), k)


def test_toeplitz_recon_follows_the_gridded_recon():
    """The Toeplitz normal operator gives the same iterates as A^H (A X - b) to the KB error, and
    the same costs: LLR-only (lambda1^0 = 0, so no graph decision enters the iterate), 4 iterations."""
    cfg = mrfgen.get_config("C1", N=32, L=40, Ns=256)
    atoms, grid = mrfgen.make_dictionary(cfg)
    V, _ = mrfgen.subspace_basis(atoms, cfg["r"])
    X = mrfgen.truth_fingerprints(cfg, mrfgen.make_phantom(cfg, 0))
    traj = mrfgen.vds_spiral(cfg["N"], cfg["L"], cfg["Ns"], cfg["n_interleaves"])
    b = nufft.nufft_fwd(X, traj)
    b = b + 0.01 * np.abs(b).mean() * np.random.default_rng(6).standard_normal(b.shape)
    kw = dict(lam1_0=0.0, lam2=0.05, beta=0.2, mu0=1.0, lamA=40.0, n_max=4)
    g = recon.recon(b, traj, atoms, grid["lut"], V, cfg["N"], 4, 2, 6, 6, **kw)
    t = recon.recon(b, traj, atoms, grid["lut"], V, cfg["N"], 4, 2, 6, 6, toeplitz=True, **kw)
    assert np.linalg.norm(t["X"] - g["X"]) <= 1e-4 * np.linalg.norm(g["X"])
    np.testing.assert_allclose(t["stats"]["cost"], g["stats"]["cost"], rtol=1e-4)
