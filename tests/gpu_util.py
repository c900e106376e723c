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
