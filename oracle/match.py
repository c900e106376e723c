"""Oracle: dictionary pattern matching Phi_D (eqs. (4)-(5), Sec. II-B).

TEST INFRASTRUCTURE ONLY.

k = argmax_m |<d_m, x>| / ||d_m||,  eta = LUT[k],  rho = max(Re<d_k, x> / ||d_k||^2, 0)
with <d, x> = sum_l conj(d_l) x_l. Ties go to the lowest m.

Reading: eq. (5) prints ||d_k||_2^2 in the argmax denominator, which would rank atoms by
their least-squares amplitude rather than their similarity; the argmax here divides by
||d_k||_2 (the two coincide for unit-norm atoms, and the SVD-matching work the paper
cites matches unit-norm atoms). The rho formula is kept as printed.
Subspace form (the SVD compression the paper cites for matching): inner products are
taken between alpha = x V and the projected atoms d_m V (= <d_m, P_S x>); the norms
stay those of the full-length atoms.
Pins: exact recovery of rho d_m; equivalence of the argmax with the least-squares
residual argmin over complex rho; subspace = full match when r = rank(D).
"""
import numpy as np


def match_vectors(xv, atoms, lut, norms=None):
    """xv [Nv, Lf], atoms [M, Lf] -> (idx int64 [Nv], rho [Nv], score [Nv], params [Nv, P])."""
    xv = np.asarray(xv, np.complex128)
    D = np.asarray(atoms, np.complex128)
    if norms is None:
        norms = np.linalg.norm(D, axis=1)
    norms = np.asarray(norms, np.float64)
    ip = xv @ D.conj().T                             # [Nv, M] = <d_m, x_v>
    score = np.abs(ip) / norms[None, :]
    idx = np.argmax(score, axis=1)                   # first maximum = lowest m
    rows = np.arange(xv.shape[0])
    rho = np.maximum(ip[rows, idx].real / norms[idx] ** 2, 0.0)
    return idx, rho, score[rows, idx], np.asarray(lut, np.float64)[idx]


def match_full(X, atoms, lut):
    """Full-length match of X [L, N, N] (or [Nv, L] when 2-D)."""
    X = np.asarray(X)
    xv = X if X.ndim == 2 else X.reshape(X.shape[0], -1).T
    return match_vectors(xv, atoms, lut)


def match_subspace(X, atoms, lut, V):
    """Match in the span of V [L, r]: alpha = x V against d_m V, full-length norms."""
    X = np.asarray(X, np.complex128)
    V = np.asarray(V, np.complex128)
    xv = X if X.ndim == 2 else X.reshape(X.shape[0], -1).T
    D = np.asarray(atoms, np.complex128)
    norms = np.linalg.norm(D, axis=1)
    return match_vectors(xv @ V, D @ V, lut, norms)


def precision_match_ref(xv, atoms, lut, topk=4, chunk=4096):
    """Exhaustive FP64 full-length match of xv [Nv, L] against atoms [M, L] (the reference the
    low-precision forms are judged by), atoms taken in chunks of `chunk` so that the [Nv, M]
    score matrix is never held whole.

    Returns (idx, rho, score, params, top_idx [Nv, topk], top_score [Nv, topk]); the top-k
    list is ordered by score descending, equal scores by the lower atom index.
    """
    xv = np.asarray(xv, np.complex128)
    D = np.asarray(atoms, np.complex128)
    norms = np.linalg.norm(D, axis=1)
    Nv, M = xv.shape[0], D.shape[0]
    k = min(topk, M)
    best_s = np.full((Nv, k), -np.inf)
    best_i = np.full((Nv, k), -1, np.int64)
    best_ip = np.zeros((Nv, k), np.complex128)
    for m0 in range(0, M, chunk):
        m1 = min(M, m0 + chunk)
        ip = xv @ D[m0:m1].conj().T
        sc = np.abs(ip) / norms[None, m0:m1]
        s_all = np.concatenate([best_s, sc], axis=1)
        i_all = np.concatenate([best_i, np.broadcast_to(np.arange(m0, m1), sc.shape)], axis=1)
        p_all = np.concatenate([best_ip, ip], axis=1)
        # descending score, ties by ascending index: lexsort's last key is the primary one
        order = np.lexsort((i_all, -s_all), axis=1)[:, :k]
        best_s = np.take_along_axis(s_all, order, 1)
        best_i = np.take_along_axis(i_all, order, 1)
        best_ip = np.take_along_axis(p_all, order, 1)
    idx = best_i[:, 0]
    rho = np.maximum(best_ip[:, 0].real / norms[idx] ** 2, 0.0)
    return idx, rho, best_s[:, 0], np.asarray(lut, np.float64)[idx], best_i, best_s


def maps_from_match(idx, rho, lut, N):
    """[3, N, N] maps (T1, T2, PD) from a match result."""
    lut = np.asarray(lut, np.float64)
    return np.stack([lut[idx, 0].reshape(N, N), lut[idx, 1].reshape(N, N),
                     np.asarray(rho, np.float64).reshape(N, N)])
