"""Oracle: patch extraction Q_q, Casorati Q(X) and its adjoint Q* (Sec. III-A, III-B).

TEST INFRASTRUCTURE ONLY.

Readings where the paper is silent or garbled:
  * stride s = floor(p / 2) (the printed "s = p|2" is garbled; 11 -> 5 in Sec. III-D);
  * patch origins {0, s, 2s, ..., N - p} on each axis, with N - p appended when the
    last stride does not land on it (non-periodic boundary);
  * a patch Q_q(X) of X [L, N, N] is the p^2 x L Casorati matrix whose row r is the
    time course of pixel (oy + r // p, ox + r % p) (space x time);
  * patches are numbered in raster order of their origins (y outer, x inner).
Q* is the overlap-add of patches back to their positions; the coverage c = Q*Q(1).
Pins: the adjoint identity <Q X, P> = <X, Q* P> and the closed-form coverage.
"""
import numpy as np


def origins_1d(N, p, s):
    o = list(range(0, N - p + 1, s))
    if o[-1] != N - p:
        o.append(N - p)
    return np.array(o, np.int64)


def patch_origins(N, p, s):
    """[Np, 2] array of (oy, ox) in raster order."""
    o = origins_1d(N, p, s)
    return np.array([(oy, ox) for oy in o for ox in o], np.int64)


def Q(X, p, s):
    """X [L, N, N] -> patches [Np, p*p, L] (each a p^2 x L Casorati matrix)."""
    X = np.asarray(X)
    L, N, _ = X.shape
    org = patch_origins(N, p, s)
    out = np.empty((len(org), p * p, L), X.dtype)
    for i, (oy, ox) in enumerate(org):
        blk = X[:, oy:oy + p, ox:ox + p]                  # [L, p, p]
        out[i] = blk.reshape(L, p * p).T
    return out


def Qadj(P, N, p, s):
    """patches [Np, p*p, L] -> X [L, N, N] by overlap-add."""
    P = np.asarray(P)
    Np, pp, L = P.shape
    org = patch_origins(N, p, s)
    X = np.zeros((L, N, N), P.dtype)
    for i, (oy, ox) in enumerate(org):
        X[:, oy:oy + p, ox:ox + p] += P[i].T.reshape(L, p, p)
    return X


def coverage(N, p, s):
    """c(v) = number of patches that cover pixel v, [N, N]."""
    return Qadj(np.ones((len(patch_origins(N, p, s)), p * p, 1)), N, p, s)[0].real
