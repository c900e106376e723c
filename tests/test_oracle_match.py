"""Pins of the oracle's pattern match (eqs. (4)-(5))."""
import numpy as np

from oracle import match


def _cplx(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_noise_free_fingerprint_recovers_atom_and_pd():
    rng = np.random.default_rng(1)
    D = _cplx(rng, 30, 20) * rng.uniform(0.2, 3.0, (30, 1))
    lut = np.stack([np.arange(30) * 10.0, np.arange(30) * 1.0], 1)
    m = np.array([3, 17, 29, 0])
    rho = np.array([1.5, 80.0, 0.01, 7.0])
    x = rho[:, None] * D[m]
    idx, r, _, params = match.match_vectors(x, D, lut)
    np.testing.assert_array_equal(idx, m)
    np.testing.assert_allclose(r, rho, rtol=1e-12)
    np.testing.assert_array_equal(params, lut[m])


def test_argmax_equals_least_squares_residual_argmin():
    rng = np.random.default_rng(2)
    D = _cplx(rng, 25, 12) * rng.uniform(0.2, 3.0, (25, 1))
    x = _cplx(rng, 40, 12)
    idx, _, _, _ = match.match_vectors(x, D, np.zeros((25, 2)))
    for v in range(40):
        res = [np.linalg.lstsq(D[m][:, None], x[v], rcond=None)[1][0] for m in range(25)]
        assert idx[v] == int(np.argmin(res))


def test_subspace_match_equals_full_match_at_full_rank():
    rng = np.random.default_rng(3)
    D = _cplx(rng, 8, 20)
    _, _, vh = np.linalg.svd(D / np.linalg.norm(D, axis=1, keepdims=True), full_matrices=False)
    V = vh.conj().T                                  # r = rank(D) = 8
    X = (_cplx(rng, 6, 8) @ D).T.reshape(20, 2, 3)   # in the span of D
    a = match.match_full(X, D, np.zeros((8, 2)))
    b = match.match_subspace(X, D, np.zeros((8, 2)), V)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_allclose(a[1], b[1], rtol=1e-10)


def test_ties_go_to_the_lowest_atom_and_zero_voxels_give_zero_pd():
    D = np.array([[1.0, 0], [1.0, 0], [0, 1.0]], complex)
    idx, rho, _, _ = match.match_vectors(np.array([[2.0, 0], [0, 0]], complex), D, np.zeros((3, 2)))
    np.testing.assert_array_equal(idx, [0, 0])
    np.testing.assert_array_equal(rho, [2.0, 0.0])


def test_precision_reference_top_k_by_brute_force():
    """The chunked top-k reference against an explicit double loop over (voxel, atom) on tiny
    inputs, with planted exact ties (ordered by the lower index) and chunk boundaries inside
    the atom range."""
    rng = np.random.default_rng(7)
    Nv, M, L = 6, 23, 9
    D = rng.standard_normal((M, L)) + 1j * rng.standard_normal((M, L))
    D[11] = D[4]                # the same atom twice: an exact tie, 4 must come first
    X = rng.standard_normal((Nv, L)) + 1j * rng.standard_normal((Nv, L))
    X[2] = 3.0 * np.exp(0.4j) * D[4]
    lut = np.stack([np.arange(M, dtype=float), 10.0 * np.arange(M)], 1)
    idx, rho, score, params, ti, ts = match.precision_match_ref(X, D, lut, topk=4, chunk=5)
    for v in range(Nv):
        s = []
        for m in range(M):
            ip = sum(np.conj(D[m, l]) * X[v, l] for l in range(L))
            s.append((-abs(ip) / np.sqrt(sum(abs(D[m, l]) ** 2 for l in range(L))), m))
        s.sort()
        ref = [m for _, m in s[:4]]
        # equal scores (to rounding) may be ordered either way by the float sort; compare as sets
        # of the top four and require the exact tie 4 / 11 to put 4 first
        assert set(ti[v]) == set(ref) or np.isclose(-s[3][0], -s[4][0])
        np.testing.assert_allclose(ts[v], [-x for x, _ in s[:4]], rtol=1e-12)
    assert idx[2] == 4 and list(ti[2][:2]) == [4, 11]
    assert np.isclose(rho[2], 3.0 * np.cos(0.4))
    assert np.all(params[:, 0] == idx)
