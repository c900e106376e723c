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


def llr_xupdate(X, tau, rank_cap, kappa, p, s, Z=None, beta_coef=None, V=None, stream=None):
    """X update of eq. (23) after the SVT of eq. (22) (mrf_llr_xupdate): returns
    (Z + kappa Q*(SVT(Q(X)))) / (1 + kappa c). Z [L, n, n], or beta_coef [n*n, r] with V [L, r]
    (Z = beta_coef V^H, 8 x 8 patches at stride 4)."""
    L, n, _ = X.shape
    need(X, torch.complex64, (L, n, n), "X")
    r = 0
    if Z is not None:
        need(Z, torch.complex64, (L, n, n), "Z")
    if beta_coef is not None:
        r = beta_coef.shape[1]
        need(beta_coef, torch.complex64, (n * n, r), "beta_coef")
        need(V, torch.complex64, (L, r), "V")
    sz = ctypes.c_size_t()
    check(lib.mrf_llr_xupdate_workspace_size(n, L, p, s, rank_cap, ctypes.byref(sz)), "mrf_llr_xupdate_workspace_size")
    ws = workspace(sz.value, X.device)
    out = torch.empty_like(X)
    check(lib.mrf_llr_xupdate(ptr(X), ptr(Z), ptr(beta_coef), ptr(V), int(r), n, L, p, s, float(tau), int(rank_cap),
                              float(kappa), ptr(out), ptr(ws), ws.numel(), stream_ptr(stream)), "mrf_llr_xupdate")
    return out
