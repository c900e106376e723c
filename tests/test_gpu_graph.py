"""GPU parity of the K-NN patch-graph Laplacian and the Laplacian apply against the oracle."""
import numpy as np
import pytest
import torch

from oracle import graph as ograph
from oracle import ops as oops
from tests.gpu_util import rel_l2, say, to_dev
from tests.workloads import c1_workload, random_maps

pytestmark = pytest.mark.gpu


def _dense(rowptr, col, val, n):
    L = np.zeros((n, n))
    for i in range(n):
        for e in range(rowptr[i], rowptr[i + 1]):
            L[i, col[e]] = val[e]
    return L


# FP32 squared distances of 3 p^2 features scaled to [0, 1]: rounding of the sum bounds the
# relative error by about 3 p^2 * 2^-24 (<= 1.2e-5 for p = 8), so neighbour choices may differ
# from the FP64 oracle only where the K-th and (K+1)-th distances are that close.
NEAR_TIE = 2e-5


def _kth(d2_row, i, K):
    srt = np.sort(np.delete(d2_row, i))
    return srt[K - 1], srt[K]


def _check_pattern(Lg, Lr, d2, K):
    diff = np.argwhere((np.abs(Lg) > 0) != (np.abs(Lr) > 0))
    for i, j in diff:
        ok = False
        for a, b in ((i, j), (j, i)):
            k1, k2 = _kth(d2[a], a, K)
            if abs(k2 - k1) <= NEAR_TIE * max(k1, 1e-30) and abs(d2[a, b] - k1) <= NEAR_TIE * max(k1, 1e-30):
                ok = True
        assert ok, f"entry ({i}, {j}) differs without a near-tie"
    return len(diff)


def _gpu_graph(maps, p, s, K, sigma2=0.0):
    from paper_2310_05647_amd import PatchGraph
    N = maps.shape[1]
    g = PatchGraph(N, p, s, max(K, 1), max_frames=64)
    g.build(to_dev(maps), K, sigma2)
    rp, col, val, inf = g.csr(torch.device("cuda:0"))
    return g, _dense(rp.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy(), inf["np"]), inf


@pytest.mark.parametrize("N,p,s,K", [(32, 4, 2, 8), (48, 8, 4, 16), (64, 4, 2, 1), (256, 8, 4, 16)])
def test_knn_laplacian_matches_oracle(N, p, s, K):
    say(f"graph parity N={N} p={p} s={s} K={K}")
    rng = np.random.default_rng(N + K)
    maps = random_maps(rng, N)
    _, Lg, inf = _gpu_graph(maps, p, s, K)
    ref = ograph.knn_laplacian(maps.astype(np.float64), p, s, K)
    assert abs(inf["sigma2"] - ref["sigma2"]) <= 1e-5 * ref["sigma2"]
    assert np.allclose(Lg, Lg.T, rtol=0, atol=0)
    assert np.max(np.abs(Lg.sum(1))) <= 1e-4 * np.max(np.abs(Lg))
    # the neighbour sets agree except at near-ties of the K-th distance (of row i or of row j,
    # since an edge enters row i also when i is among j's K nearest)
    Lr = ref["L"]
    n_flip = _check_pattern(Lg, Lr, ref["d2"], K)
    if n_flip:
        say(f"  {n_flip} entries differ at near-ties")
        same = (np.abs(Lg) > 0) == (np.abs(Lr) > 0)
        rows_ok = np.all(same, axis=1)
        np.testing.assert_allclose(Lg[rows_ok][:, rows_ok], Lr[rows_ok][:, rows_ok], rtol=2e-5,
                                   atol=2e-6 * np.abs(Lr).max())
        return
    np.testing.assert_allclose(Lg, Lr, rtol=2e-5, atol=2e-6 * np.abs(Lr).max())
    assert abs(inf["lmax"] - ref["lmax"]) <= 2e-5 * ref["lmax"]


def test_ties_in_piecewise_constant_maps_follow_the_lower_index_rule():
    rng = np.random.default_rng(5)
    maps = random_maps(rng, 32, zero_frac=0.5)
    maps[:, :16, :] = 0.0                     # a large all-zero region: many exact zero distances
    _, Lg, inf = _gpu_graph(maps, 4, 2, 8)
    ref = ograph.knn_laplacian(maps.astype(np.float64), 4, 2, 8)
    assert np.array_equal(np.abs(Lg) > 0, np.abs(ref["L"]) > 0)
    np.testing.assert_allclose(Lg, ref["L"], rtol=2e-5, atol=1e-6)


@pytest.mark.parametrize("N,p,s,K,L", [(32, 4, 2, 8, 5), (64, 8, 4, 16, 3), (64, 4, 2, 8, 40), (96, 8, 4, 16, 37)])
def test_laplacian_apply_and_quad_match_oracle(N, p, s, K, L):
    say(f"laplacian apply N={N} p={p} L={L}")
    rng = np.random.default_rng(N * L)
    maps = random_maps(rng, N)
    g, Lg, inf = _gpu_graph(maps, p, s, K)
    X = (rng.standard_normal((L, N, N)) + 1j * rng.standard_normal((L, N, N))).astype(np.complex64)
    Xd = to_dev(X)
    Y = g.apply(Xd).cpu().numpy()
    ref = oops.laplacian_apply(X, Lg, p, s)   # the operator of eq. (15) with the GPU's L
    e = rel_l2(Y, ref)
    q = float(g.quad(Xd).cpu().numpy()[0])
    qref = float(np.vdot(X.astype(np.complex128), ref).real)
    say(f"  apply rel-L2 {e:.2e}  quad rel {abs(q - qref) / abs(qref):.2e}")
    assert e <= 1e-5
    assert abs(q - qref) <= 1e-5 * abs(qref)
    # and the graph itself equals the oracle's (random maps: no ties)
    ref_g = ograph.knn_laplacian(maps.astype(np.float64), p, s, K)
    np.testing.assert_allclose(Lg, ref_g["L"], rtol=2e-5, atol=2e-6 * np.abs(Lg).max())


def test_graph_from_c1_phantom_maps():
    """Piecewise-constant maps: many distances tie in exact arithmetic and are broken by
    rounding, so the sets may differ at such ties; weights of the agreeing rows must match."""
    w = c1_workload()
    ph = w["phantom"]
    maps = np.stack([ph["T1"], ph["T2"], ph["PD"]]).astype(np.float32)
    _, Lg, inf = _gpu_graph(maps, 4, 2, 8)
    ref = ograph.knn_laplacian(maps.astype(np.float64), 4, 2, 8)
    n_flip = _check_pattern(Lg, ref["L"], ref["d2"], 8)
    say(f"  phantom graph: {n_flip} entries differ at exact-arithmetic ties")
    assert abs(inf["sigma2"] - ref["sigma2"]) <= 1e-5 * ref["sigma2"]


@pytest.mark.parametrize("N,zero_rows", [(64, 24), (64, 48), (128, 96)])
def test_quad_with_hub_rows_matches_oracle(N, zero_rows):
    """8 x 8 patches at stride 4 on maps with a large all-zero region: exact-zero distances make the
    lowest-index patches of the region everyone's nearest neighbours, so some rows hold far more
    than 2K entries (the trace kernel walks a row in windows of 64 entries), a trace tile holds
    more entries than its LDS keeps (the rest are read from global memory), and at N = 128 the
    hub's pairs span several tiles and leave the LDS windows (the out-of-window kernel).
    The trace against Re<X, Q*(Q(X) L)> formed by the oracle with the GPU's own L."""
    rng = np.random.default_rng(zero_rows)
    L = 9
    maps = random_maps(rng, N)
    maps[:, :zero_rows, :] = 0.0
    g, Lg, inf = _gpu_graph(maps, 8, 4, 16)
    n = Lg.shape[0]
    upper = max(int(np.count_nonzero(Lg[i, i + 1:])) for i in range(n))
    X = (rng.standard_normal((L, N, N)) + 1j * rng.standard_normal((L, N, N))).astype(np.complex64)
    q = float(g.quad(to_dev(X)).cpu().numpy()[0])
    qref = float(np.vdot(X.astype(np.complex128), oops.laplacian_apply(X, Lg, 8, 4)).real)
    say(f"  hub rows: longest upper row {upper}; quad rel {abs(q - qref) / abs(qref):.2e}")
    assert upper > 64
    assert abs(q - qref) <= 1e-5 * abs(qref)


def test_quad_on_smooth_256_maps_matches_oracle():
    """The graph of the 256 x 256 workload's maps (8 x 8 patches at stride 4, K = 16; mostly local
    edges, so most cell pairs meet inside the trace kernel's LDS window and the rest take the
    out-of-window kernel), 13 frames (a ragged last frame group): the trace against
    Re<X, Q*(Q(X) L)> formed by the oracle with the GPU's own L."""
    import os
    f = np.load(os.path.join(os.path.dirname(__file__), "golden", "c2_two_iterations.npz"))
    maps = f["maps"].astype(np.float32)
    g, Lg, inf = _gpu_graph(maps, 8, 4, 16)
    rng = np.random.default_rng(256)
    N, L = 256, 13
    X = (rng.standard_normal((L, N, N)) + 1j * rng.standard_normal((L, N, N))).astype(np.complex64)
    q = float(g.quad(to_dev(X)).cpu().numpy()[0])
    import scipy.sparse as sp
    qref = float(np.vdot(X.astype(np.complex128), oops.laplacian_apply(X, sp.csr_matrix(Lg), 8, 4)).real)
    say(f"  256 x 256 maps: quad rel {abs(q - qref) / abs(qref):.2e}")
    assert abs(q - qref) <= 1e-5 * abs(qref)
