"""The orthonormal temporal basis of the projection P_S (eq. (17), Sec. III-B).

Algorithm 1 lists P_S among its predefined inputs, and the paper approximates the
basis d from the precomputed dictionary. This generator takes the top-r right
singular vectors of the unit-normalised dictionary, so that P_S(x) = x V V^H for a
row vector x in C^{1 x L}. Phase convention: the entry of largest magnitude in each
column of V is made real and positive.
"""
import numpy as np


def subspace_basis(atoms, r):
    """Return (V complex64 [L, r], singular values float64 of the unit-norm dictionary)."""
    D = np.asarray(atoms, np.complex128)
    D = D / np.linalg.norm(D, axis=1, keepdims=True)
    _, s, vh = np.linalg.svd(D, full_matrices=False)
    V = vh[:r].conj().T.copy()                      # [L, r]
    for k in range(r):
        i = int(np.argmax(np.abs(V[:, k])))
        V[:, k] *= np.conj(V[i, k]) / np.abs(V[i, k])
    return V.astype(np.complex64), s
