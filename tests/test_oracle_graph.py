"""Pins of the oracle's graph Laplacian (eqs. (7)-(11))."""
import numpy as np
import pytest
import scipy.spatial.distance

from oracle import graph, ops, patches


def test_three_node_example_eq11():
    """The symbolic three-node Laplacian of eq. (11), read from tests/golden, evaluated at
    arbitrary weights."""
    import os
    rows = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "eq11_three_node_laplacian.txt"))
    for w12, w13, w23 in ((0.3, 0.7, 0.11), (1.0, 0.0, 2.5)):
        W = np.array([[0, w12, w13], [w12, 0, w23], [w13, w23, 0]])
        expect = np.zeros((3, 3))
        for i, j, c12, c13, c23 in rows:
            expect[int(i), int(j)] = c12 * w12 + c13 * w13 + c23 * w23
        np.testing.assert_array_equal(graph.laplacian_from_weights(W), expect)


def _rand_maps(rng, N):
    return np.stack([rng.uniform(300, 2500, (N, N)), rng.uniform(40, 300, (N, N)), rng.uniform(0, 100, (N, N))])


@pytest.mark.parametrize("K", [1, 4, 8])
def test_laplacian_is_symmetric_psd_with_zero_row_sums(K):
    rng = np.random.default_rng(K)
    g = graph.knn_laplacian(_rand_maps(rng, 12), 4, 2, K)
    L = g["L"]
    assert np.allclose(L, L.T, atol=0, rtol=0)
    assert np.max(np.abs(L.sum(axis=1))) <= 1e-12
    assert np.linalg.eigvalsh(L).min() >= -1e-12
    assert g["lmax"] == np.max(np.diag(L))


def test_dense_graph_when_K_is_Np_minus_1():
    rng = np.random.default_rng(7)
    maps = _rand_maps(rng, 10)
    F = graph.patch_features(maps, 4, 2)
    Np = F.shape[0]
    sig2 = 0.37
    g = graph.knn_laplacian(maps, 4, 2, Np - 1, sigma2=sig2)
    W = np.exp(-scipy.spatial.distance.cdist(F, F, "sqeuclidean") / sig2)
    np.fill_diagonal(W, 0.0)
    np.testing.assert_allclose(g["L"], np.diag(W.sum(1)) - W, rtol=1e-12, atol=1e-14)


def test_features_are_patches_of_max_scaled_maps():
    rng = np.random.default_rng(8)
    maps = _rand_maps(rng, 8)
    F = graph.patch_features(maps, 4, 2)
    # patch 4 has origin (2, 2) on a 3x3 origin grid; channel 1 (T2) pixel (0, 1) of it
    assert F[4, 16 + 1] == maps[1, 2, 3] / maps[1].max()


def test_ties_go_to_the_lower_index():
    d2 = np.array([[0, 1, 1, 1], [1, 0, 2, 2], [1, 2, 0, 2], [1, 2, 2, 0]], float)
    nbr = graph.knn_lists(d2, 2)
    np.testing.assert_array_equal(nbr, [[1, 2], [0, 2], [0, 1], [0, 1]])


def test_median_rule_lower_median_of_positive_values():
    d2 = np.array([[0, 0.0, 4.0], [0.0, 0, 1.0], [4.0, 1.0, 0]])
    nbr = np.array([[1, 2], [0, 2], [1, 0]])
    # directed values: 0, 4, 0, 1, 1, 4 -> positive sorted 1, 1, 4, 4 -> lower median 1
    assert graph.median_rule(d2, nbr) == 1.0


def test_trace_form_equals_half_the_pairwise_form():
    """eq. (9) vs eq. (7): Tr(Q L Q^H) = (1/2) sum_{i,j} w_ij ||q_i - q_j||^2 for symmetric W."""
    rng = np.random.default_rng(9)
    N, p, s, L = 12, 4, 2, 3
    g = graph.knn_laplacian(_rand_maps(rng, N), p, s, 3)
    W = np.diag(np.diag(g["L"])) - g["L"]
    X = rng.standard_normal((L, N, N)) + 1j * rng.standard_normal((L, N, N))
    P = patches.Q(X, p, s)
    pair = 0.0
    for i in range(P.shape[0]):
        for j in range(P.shape[0]):
            pair += W[i, j] * np.sum(np.abs(P[i] - P[j]) ** 2)
    tr = np.vdot(X, ops.laplacian_apply(X, g["L"], p, s)).real
    assert abs(tr - 0.5 * pair) <= 1e-10 * abs(pair)


def test_one_sided_knn_edges_are_kept_with_their_weight():
    """Reading Q7: W = max(W, W^T). Four nodes with hand-chosen squared distances so that
    K-NN membership is one-sided: with K = 1, node 2's nearest is 0 and node 3's nearest is 1,
    but neither 0 nor 1 picks them back. Worked by hand (sigma^2 = 1): the symmetric weights
    are w01 = e^-1 (mutual), w02 = e^-2 (from 2 only), w13 = e^-4 (from 3 only); a mean
    (e^-2 / 2) or a min (0) would change L."""
    d2 = np.array([[0, 1, 2, 5],
                   [1, 0, 3, 4],
                   [2, 3, 0, 6],
                   [5, 4, 6, 0]], float)
    e1, e2, e4 = np.exp(-1.0), np.exp(-2.0), np.exp(-4.0)
    expect_L = np.array([[e1 + e2, -e1, -e2, 0.0],
                         [-e1, e1 + e4, 0.0, -e4],
                         [-e2, 0.0, e2, 0.0],
                         [0.0, -e4, 0.0, e4]])
    for sig2 in (1.0, 0.0):     # 0: median rule; the directed K-NN values 1, 1, 2, 4 give 1
        W, s2, nbr = graph.knn_weights(d2, 1, sig2)
        assert s2 == 1.0
        np.testing.assert_array_equal(nbr[:, 0], [1, 0, 0, 1])
        np.testing.assert_allclose(graph.laplacian_from_weights(W), expect_L, rtol=1e-15, atol=0)
    # K = 2: 0 and 1 pick {1, 2} and {0, 2}; 2 picks {0, 1}; 3 picks {1, 0}. Edges 3-0 and 3-1
    # come from node 3 alone and keep its weights e^-5 and e^-4.
    W, _, _ = graph.knn_weights(d2, 2, 1.0)
    expect_W = np.zeros((4, 4))
    for (i, j), d in {(0, 1): 1, (0, 2): 2, (1, 2): 3, (0, 3): 5, (1, 3): 4}.items():
        expect_W[i, j] = expect_W[j, i] = np.exp(-d)
    np.testing.assert_allclose(W, expect_W, rtol=1e-15, atol=0)
