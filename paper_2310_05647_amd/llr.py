"""LLR proximal step binding: mrf_llr_prox."""
import ctypes

import torch

from ._lib import check, lib
from .util import need, ptr, stream_ptr, workspace


def llr_prox(X, p, s, tau, rank_cap, stream=None):
    """Returns (Q*(P') [L, n, n] complex64, nuclear norm (device float64 [1]))."""
    L, n, _ = X.shape
    need(X, torch.complex64, (L, n, n), "X")
    sz = ctypes.c_size_t()
    check(lib.mrf_llr_workspace_size(n, L, p, s, rank_cap, ctypes.byref(sz)), "mrf_llr_workspace_size")
    ws = workspace(sz.value, X.device)
    out = torch.empty_like(X)
    nuc = torch.empty(1, dtype=torch.float64, device=X.device)
    check(lib.mrf_llr_prox(ptr(X), ptr(out), n, L, p, s, float(tau), int(rank_cap), ptr(nuc), ptr(ws), ws.numel(),
                           stream_ptr(stream)), "mrf_llr_prox")
    return out, nuc
