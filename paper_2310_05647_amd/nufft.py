"""NUFFT pair binding: mrf_nufft_plan_create / mrf_nufft_fwd / mrf_nufft_adj, and the multi-coil
operator F_u C of eq. (1) (mrf_nufft_fwd_mc / mrf_nufft_adj_mc / mrf_nufft_opnorm_mc)."""
import ctypes

import torch

from ._lib import NufftDesc, check, lib


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _need(t, dtype, shape, name):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous() and tuple(t.shape) == tuple(shape)):
        raise ValueError("%s must be a contiguous CUDA %s tensor of shape %s" % (name, dtype, tuple(shape)))


def autotune(n, traj, reps=3, stream=None):
    """Fastest strip width for this trajectory: returns (tile_cols, {tile_cols: mean pair ms})."""
    L, Ns, _ = traj.shape
    _need(traj, torch.float32, (L, Ns, 2), "traj")
    desc = NufftDesc(int(n), int(L), int(Ns), 6, 2, 0)
    best = ctypes.c_int()
    times = (ctypes.c_float * 3)()
    check(lib.mrf_nufft_autotune(ctypes.byref(desc), _ptr(traj), int(reps), ctypes.byref(best), times,
                                 _stream(stream)), "mrf_nufft_autotune")
    return best.value, {tx: t for tx, t in zip((8, 16, 32), times) if t >= 0}


class NufftPlan:
    """Plan of A / A^H for a fixed trajectory traj [L, Ns, 2] (float32, rad/pixel, device)."""

    def __init__(self, n, traj, tile_cols=0, stream=None):
        L, Ns, two = traj.shape
        _need(traj, torch.float32, (L, Ns, 2), "traj")
        self.n, self.L, self.Ns = int(n), int(L), int(Ns)
        desc = NufftDesc(self.n, self.L, self.Ns, 6, 2, int(tile_cols))
        h = ctypes.c_void_p()
        check(lib.mrf_nufft_plan_create(ctypes.byref(desc), _ptr(traj), _stream(stream), ctypes.byref(h)),
              "mrf_nufft_plan_create")
        self.handle = h
        sz = ctypes.c_size_t()
        check(lib.mrf_nufft_workspace_size(h, ctypes.byref(sz)), "mrf_nufft_workspace_size")
        self.ws = torch.empty(max(1, sz.value), dtype=torch.uint8, device=traj.device)

    def fwd(self, img, out=None, stream=None):
        _need(img, torch.complex64, (self.L, self.n, self.n), "img")
        if out is None:
            out = torch.empty((self.L, self.Ns), dtype=torch.complex64, device=img.device)
        _need(out, torch.complex64, (self.L, self.Ns), "ksp")
        check(lib.mrf_nufft_fwd(self.handle, _ptr(img), _ptr(out), _ptr(self.ws), self.ws.numel(), _stream(stream)),
              "mrf_nufft_fwd")
        return out

    def adj(self, ksp, out=None, stream=None):
        _need(ksp, torch.complex64, (self.L, self.Ns), "ksp")
        if out is None:
            out = torch.empty((self.L, self.n, self.n), dtype=torch.complex64, device=ksp.device)
        _need(out, torch.complex64, (self.L, self.n, self.n), "img")
        check(lib.mrf_nufft_adj(self.handle, _ptr(ksp), _ptr(out), _ptr(self.ws), self.ws.numel(), _stream(stream)),
              "mrf_nufft_adj")
        return out

    def opnorm(self, iters=30, seed=1, stream=None):
        """lambda_max(A^H A) by power iteration on the device."""
        lam = ctypes.c_double()
        check(lib.mrf_nufft_opnorm(self.handle, int(iters), int(seed), ctypes.byref(lam), _stream(stream)),
              "mrf_nufft_opnorm")
        return lam.value

    def _maps(self, smaps):
        if smaps.dim() != 3:
            raise ValueError("smaps must be [ncoils, n, n]")
        _need(smaps, torch.complex64, (smaps.shape[0], self.n, self.n), "smaps")
        return smaps.shape[0]

    def fwd_mc(self, smaps, img, out=None, stream=None):
        """ksp [ncoils, L, Ns]: every coil's samples of S_c img."""
        nc = self._maps(smaps)
        _need(img, torch.complex64, (self.L, self.n, self.n), "img")
        if out is None:
            out = torch.empty((nc, self.L, self.Ns), dtype=torch.complex64, device=img.device)
        _need(out, torch.complex64, (nc, self.L, self.Ns), "ksp")
        check(lib.mrf_nufft_fwd_mc(self.handle, _ptr(smaps), nc, _ptr(img), _ptr(out), _ptr(self.ws),
                                   self.ws.numel(), _stream(stream)), "mrf_nufft_fwd_mc")
        return out

    def adj_mc(self, smaps, ksp, out=None, stream=None):
        """img [L, n, n] = sum_c conj(S_c) A^H ksp_c."""
        nc = self._maps(smaps)
        _need(ksp, torch.complex64, (nc, self.L, self.Ns), "ksp")
        if out is None:
            out = torch.empty((self.L, self.n, self.n), dtype=torch.complex64, device=ksp.device)
        _need(out, torch.complex64, (self.L, self.n, self.n), "img")
        check(lib.mrf_nufft_adj_mc(self.handle, _ptr(smaps), nc, _ptr(ksp), _ptr(out), _ptr(self.ws),
                                   self.ws.numel(), _stream(stream)), "mrf_nufft_adj_mc")
        return out

    def opnorm_mc(self, smaps, iters=30, seed=1, stream=None):
        """lambda_max((F_u C)^H F_u C) by power iteration on the device."""
        nc = self._maps(smaps)
        lam = ctypes.c_double()
        check(lib.mrf_nufft_opnorm_mc(self.handle, _ptr(smaps), nc, int(iters), int(seed), ctypes.byref(lam),
                                      _stream(stream)), "mrf_nufft_opnorm_mc")
        return lam.value

    def close(self):
        if getattr(self, "handle", None):
            lib.mrf_nufft_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class CartPlan(NufftPlan):
    """Pseudo-radial Cartesian sampling (mrf_cart_plan_create): A_l X_l = M_l F X_l, F the unitary
    centred DFT. mask: uint8 [L, n, n] (device). k-space arrays are [L, n * n] (dense, zero where
    the mask is); every NufftPlan method applies."""

    def __init__(self, mask, stream=None):
        L, n, n2 = mask.shape
        if n != n2:
            raise ValueError("mask must be [L, n, n]")
        _need(mask, torch.uint8, (L, n, n), "mask")
        self.n, self.L, self.Ns = int(n), int(L), int(n) * int(n)
        h = ctypes.c_void_p()
        check(lib.mrf_cart_plan_create(self.n, self.L, _ptr(mask), _stream(stream), ctypes.byref(h)),
              "mrf_cart_plan_create")
        self.handle = h
        sz = ctypes.c_size_t()
        check(lib.mrf_nufft_workspace_size(h, ctypes.byref(sz)), "mrf_nufft_workspace_size")
        self.ws = torch.empty(max(1, sz.value), dtype=torch.uint8, device=mask.device)


class Toeplitz:
    """Toeplitz normal operator A^H A (mrf_toeplitz_create) for the trajectory traj [L, Ns, 2]
    (float32, device) of an n x n image series."""

    def __init__(self, n, traj, stream=None):
        L, Ns, _ = traj.shape
        _need(traj, torch.float32, (L, Ns, 2), "traj")
        self.n, self.L = int(n), int(L)
        desc = NufftDesc(self.n, self.L, int(Ns), 6, 2, 0)
        h = ctypes.c_void_p()
        check(lib.mrf_toeplitz_create(ctypes.byref(desc), _ptr(traj), _stream(stream), ctypes.byref(h)),
              "mrf_toeplitz_create")
        self.handle = h
        sz = ctypes.c_size_t()
        check(lib.mrf_toeplitz_workspace_size(h, ctypes.byref(sz)), "mrf_toeplitz_workspace_size")
        self.ws = torch.empty(max(1, sz.value), dtype=torch.uint8, device=traj.device)

    def normal(self, X, out=None, stream=None):
        """A^H A X for X [L, n, n] complex64."""
        _need(X, torch.complex64, (self.L, self.n, self.n), "X")
        if out is None:
            out = torch.empty_like(X)
        _need(out, torch.complex64, (self.L, self.n, self.n), "out")
        check(lib.mrf_toeplitz_normal(self.handle, _ptr(X), _ptr(out), _ptr(self.ws), self.ws.numel(),
                                      _stream(stream)), "mrf_toeplitz_normal")
        return out

    def close(self):
        if getattr(self, "handle", None):
            lib.mrf_toeplitz_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
