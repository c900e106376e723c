"""Ground-truth fingerprints X_{i,j,:} = rho_{i,j} B(eta_{i,j}; theta) (eq. (2))."""
import numpy as np

from ._native import epg_fisp
from .sequence import fisp_sequence


def truth_fingerprints(cfg, phantom, L=None):
    """Return X complex64 [L, N, N] (frame-major) for the phantom's tissue voxels."""
    L = int(L or cfg["L"])
    fa, tr, te = fisp_sequence(L, cfg["fa_range"], cfg["fa_period"], cfg["tr_ms"], cfg["te_ms"])
    mask = phantom["mask"] & (phantom["PD"] > 0)
    N = mask.shape[0]
    t1 = phantom["T1"][mask]; t2 = phantom["T2"][mask]; pd = phantom["PD"][mask]
    # voxels that share (T1, T2) share a fingerprint: simulate each distinct pair once
    pairs, inv = np.unique(np.stack([t1, t2], 1), axis=0, return_inverse=True)
    sig = epg_fisp(pairs[:, 0], pairs[:, 1], fa, tr, te, cfg["epg_states"])
    X = np.zeros((L, N * N), np.complex64)
    idx = np.flatnonzero(mask.ravel())
    X[:, idx] = (sig[inv.ravel()] * pd[:, None].astype(np.float32)).T
    return X.reshape(L, N, N)
