"""Helpers shared by the GPU parity tests (host-side only)."""
import numpy as np
import torch


def dev():
    return torch.device("cuda:0")


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev())


def rel_l2(a, b):
    a = np.asarray(a, np.complex128); b = np.asarray(b, np.complex128)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def say(msg):
    print(msg, flush=True)


def nuc_fp32_gram(X, p, s):
    """Sum over the p x p patches (stride s) of sqrt(max(eig, 0)) of each patch Gram formed in FP32,
    as the GPU forms it: the nuclear norm with the FP32 Gram's floor on vanishing singular values."""
    L, N, _ = X.shape
    X32 = np.asarray(X).astype(np.complex64)
    out = 0.0
    for y0 in range(0, N - p + 1, s):
        for x0 in range(0, N - p + 1, s):
            Q = X32[:, y0:y0 + p, x0:x0 + p].reshape(L, -1).T
            out += np.sqrt(np.maximum(np.linalg.eigvalsh((Q @ Q.conj().T).astype(np.complex128)), 0.0)).sum()
    return out
