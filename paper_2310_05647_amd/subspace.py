"""Subspace projection and dictionary matching bindings."""
import ctypes

import torch

from ._lib import check, lib
from .util import need, ptr, stream_ptr, workspace


def subspace_coeffs(X, V, stream=None):
    """alpha [Nv, r] = X V for X [L, ...] (frame-major), V [L, r]."""
    L = X.shape[0]
    Nv = X[0].numel()
    r = V.shape[1]
    need(V, torch.complex64, (L, r), "V")
    sz = ctypes.c_size_t()
    check(lib.mrf_subspace_coeffs_workspace_size(L, Nv, r, ctypes.byref(sz)), "mrf_subspace_coeffs_workspace_size")
    ws = workspace(sz.value, X.device)
    out = torch.empty((Nv, r), dtype=torch.complex64, device=X.device)
    check(lib.mrf_subspace_coeffs(ptr(X), ptr(V), L, Nv, r, ptr(out), ptr(ws), ws.numel(), stream_ptr(stream)),
          "mrf_subspace_coeffs")
    return out


def subspace_coeffs_noalloc(X, V, out, stream=None):
    """out [Nv, r] = X V through mrf_subspace_coeffs_noalloc (no workspace; the library's static
    scratch array). The caller provides out."""
    L = X.shape[0]
    Nv = X[0].numel()
    r = V.shape[1]
    need(V, torch.complex64, (L, r), "V")
    need(out, torch.complex64, (Nv, r), "out")
    check(lib.mrf_subspace_coeffs_noalloc(ptr(X), ptr(V), L, Nv, r, ptr(out), stream_ptr(stream)),
          "mrf_subspace_coeffs_noalloc")
    return out


def subspace_project(U, V, stream=None):
    """P_S(U) = U V V^H for U [L, ...] frame-major."""
    L = U.shape[0]
    Nv = U[0].numel()
    r = V.shape[1]
    need(V, torch.complex64, (L, r), "V")
    sz = ctypes.c_size_t()
    check(lib.mrf_subspace_coeffs_workspace_size(L, Nv, r, ctypes.byref(sz)), "mrf_subspace_coeffs_workspace_size")
    ws = workspace(sz.value + Nv * r * 8, U.device)
    out = torch.empty_like(U)
    check(lib.mrf_subspace_project(ptr(U), ptr(V), L, Nv, r, ptr(out), ptr(ws), ws.numel(), stream_ptr(stream)),
          "mrf_subspace_project")
    return out


MATCH_MODES = {"fp32": 0, "bf16": 1, "fp8": 2, "bf16x3": 5}


def frames_to_voxels(X, stream=None):
    """[L, ...] complex64 image series (device) -> [Nv, L] voxel-major fingerprints."""
    L = X.shape[0]
    Nv = X.numel() // L
    need(X, torch.complex64, tuple(X.shape), "X")
    Y = torch.empty((Nv, L), dtype=torch.complex64, device=X.device)
    check(lib.mrf_frames_to_voxels(ptr(X), L, Nv, ptr(Y), stream_ptr(stream)), "mrf_frames_to_voxels")
    return Y


class Dictionary:
    """Device dictionary: atoms [M, L] complex64, lut [M, nparam] float32, optional basis V [L, r]."""

    def __init__(self, atoms, lut, V=None, stream=None):
        M, L = atoms.shape
        need(atoms, torch.complex64, (M, L), "atoms")
        need(lut, torch.float32, (M, lut.shape[1]), "lut")
        r = 0
        if V is not None:
            r = V.shape[1]
            need(V, torch.complex64, (L, r), "V")
        self.M, self.L, self.r, self.nparam = M, L, r, lut.shape[1]
        h = ctypes.c_void_p()
        check(lib.mrf_dict_create(ptr(atoms), ptr(lut), M, L, self.nparam, ptr(V), r, stream_ptr(stream),
                                  ctypes.byref(h)), "mrf_dict_create")
        self.handle = h

    def match_subspace(self, alpha, stream=None):
        """Returns (idx int32 [Nv], rho, score, params [Nv, nparam])."""
        Nv = alpha.shape[0]
        need(alpha, torch.complex64, (Nv, self.r), "alpha")
        dev = alpha.device
        idx = torch.empty(Nv, dtype=torch.int32, device=dev)
        rho = torch.empty(Nv, dtype=torch.float32, device=dev)
        score = torch.empty(Nv, dtype=torch.float32, device=dev)
        params = torch.empty((Nv, self.nparam), dtype=torch.float32, device=dev)
        check(lib.mrf_dict_match_subspace(self.handle, ptr(alpha), Nv, ptr(idx), ptr(rho), ptr(score), ptr(params),
                                          stream_ptr(stream)), "mrf_dict_match_subspace")
        return idx, rho, score, params

    def match(self, fp, mode="fp32", want_cand=False, depth=4, stream=None):
        """Full-length match of fp [Nv, L] complex64 (device). mode: "fp32", "bf16" or "fp8"
        (the `depth` best on MFMA in that precision, then an FP32 re-rank; mrf_dict_match_depth).
        Returns (idx, rho, score, params) and, with want_cand, the [Nv, depth] re-rank candidates."""
        Nv = fp.shape[0]
        need(fp, torch.complex64, (Nv, self.L), "fp")
        m = MATCH_MODES[mode]
        dev = fp.device
        sz = ctypes.c_size_t()
        check(lib.mrf_dict_match_workspace_size(self.handle, Nv, m, ctypes.byref(sz)), "mrf_dict_match_workspace_size")
        ws = torch.empty(max(1, sz.value), dtype=torch.uint8, device=dev)
        idx = torch.empty(Nv, dtype=torch.int32, device=dev)
        rho = torch.empty(Nv, dtype=torch.float32, device=dev)
        score = torch.empty(Nv, dtype=torch.float32, device=dev)
        params = torch.empty((Nv, self.nparam), dtype=torch.float32, device=dev)
        cand = torch.empty((Nv, depth), dtype=torch.int32, device=dev) if want_cand else None
        check(lib.mrf_dict_match_depth(self.handle, ptr(fp), Nv, m, int(depth), ptr(idx), ptr(rho), ptr(score),
                                       ptr(params), ptr(cand), ptr(ws), ws.numel(), stream_ptr(stream)),
              "mrf_dict_match_depth")
        out = (idx, rho, score, params)
        return out + (cand,) if want_cand else out

    def close(self):
        if getattr(self, "handle", None):
            lib.mrf_dict_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
