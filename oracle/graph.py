"""Oracle: parameter-manifold patch graph and its Laplacian (Sec. III-A).

TEST INFRASTRUCTURE ONLY.

w_ij = exp(-||Q_{q_i}(M) - Q_{q_j}(M)||_F^2 / sigma^2)      (eq. (8))
L = D - W, D_ii = sum_j w_ij                                 (eq. (10); example eq. (11))
lambda1^n = lambda1^0 * max(L^n)                             (Algorithm 1, Sec. III-D)

Readings where the paper is silent:
  * features: the maps (T1, T2, PD) of the current estimate M, each channel divided by
    its maximum over the map (1 when that maximum is 0); the feature of patch i is its
    p x p x 3 block, flattened;
  * the graph is sparsified to the K nearest patches by squared distance (self
    excluded, ties broken towards the lower index j), then symmetrised with
    W = max(W, W^T); K = Np - 1 gives the dense graph of eq. (7);
  * sigma^2 = the lower median of the positive directed K-NN squared distances
    (1 when there are none), unless a positive sigma2 is given;
  * max(L) is the largest entry of L, i.e. the largest degree.
Pins: eq. (11) entry by entry, symmetry / zero row sums / PSD, the dense K = Np - 1
graph against scipy's cdist, and the pairwise-vs-trace identity of eqs. (7) and (9).
"""
import numpy as np

from .patches import patch_origins


def patch_features(maps, p, s):
    """maps [3, N, N] -> features [Np, 3 p^2] (channels scaled by their maxima)."""
    maps = np.asarray(maps, np.float64)
    C, N, _ = maps.shape
    scaled = np.empty_like(maps)
    for c in range(C):
        mx = maps[c].max()
        scaled[c] = maps[c] / (mx if mx > 0 else 1.0)
    org = patch_origins(N, p, s)
    F = np.empty((len(org), C * p * p))
    for i, (oy, ox) in enumerate(org):
        F[i] = scaled[:, oy:oy + p, ox:ox + p].ravel()
    return F


def pairwise_sqdist(F):
    """d2[i, j] = sum_f (F[i, f] - F[j, f])^2, written out as a sum of squared differences."""
    n = F.shape[0]
    d2 = np.empty((n, n))
    for i in range(n):
        diff = F - F[i][None, :]
        d2[i] = np.sum(diff * diff, axis=1)
    return d2


def knn_lists(d2, K):
    """[Np, K] neighbour indices: K smallest d2[i, j], j != i, ties -> lower j."""
    n = d2.shape[0]
    nbr = np.empty((n, K), np.int64)
    j = np.arange(n)
    for i in range(n):
        keep = j != i
        order = np.lexsort((j[keep], d2[i][keep]))      # by d2, then by j
        nbr[i] = j[keep][order[:K]]
    return nbr


def median_rule(d2, nbr):
    vals = np.sort(np.array([d2[i, j] for i in range(nbr.shape[0]) for j in nbr[i]]))
    vals = vals[vals > 0]
    if vals.size == 0:
        return 1.0
    return float(vals[(vals.size - 1) // 2])


def laplacian_from_weights(W):
    """L = D - W with D_ii = sum_j W_ij (eq. (10))."""
    W = np.asarray(W, np.float64)
    return np.diag(W.sum(axis=1)) - W


def knn_weights(d2, K, sigma2=0.0):
    """Symmetric K-NN weight matrix from squared distances d2 [Np, Np]: directed weights
    exp(-d2 / sigma^2) (eq. (8)) on each row's K nearest, then W = max(W, W^T).
    Returns (W, sigma2, nbr)."""
    d2 = np.asarray(d2, np.float64)
    n = d2.shape[0]
    K = min(int(K), n - 1)
    nbr = knn_lists(d2, K)
    sig2 = float(sigma2) if sigma2 and sigma2 > 0 else median_rule(d2, nbr)
    Wd = np.zeros((n, n))
    for i in range(n):
        for j in nbr[i]:
            Wd[i, j] = np.exp(-d2[i, j] / sig2)
    return np.maximum(Wd, Wd.T), sig2, nbr


def knn_laplacian(maps, p, s, K, sigma2=0.0):
    """Return dict(L dense [Np, Np], sigma2, lmax, nbr, d2)."""
    F = patch_features(maps, p, s)
    d2 = pairwise_sqdist(F)
    W, sig2, nbr = knn_weights(d2, K, sigma2)
    Lap = laplacian_from_weights(W)
    return dict(L=Lap, sigma2=sig2, lmax=float(Lap.max()), nbr=nbr, d2=d2)
