"""Oracle: evaluation metrics (Sec. IV-A). TEST INFRASTRUCTURE ONLY.

SNR  = -10 log10(||X - Xhat||_F^2 / ||X||_F^2)     eq. (24)
NMSE = ||mhat - m||^2 / ||m||^2                     eq. (25)
Reading: NMSE is taken over the ground-truth tissue mask when one is given.
"""
import numpy as np


def snr_db(X, Xhat):
    X = np.asarray(X, np.complex128); Xhat = np.asarray(Xhat, np.complex128)
    return float(-10.0 * np.log10(np.vdot(X - Xhat, X - Xhat).real / np.vdot(X, X).real))


def nmse(m, mhat, mask=None):
    m = np.asarray(m, np.float64); mhat = np.asarray(mhat, np.float64)
    if mask is not None:
        m, mhat = m[mask], mhat[mask]
    return float(np.sum((mhat - m) ** 2) / np.sum(m ** 2))
