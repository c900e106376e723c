"""Patch graph binding: mrf_graph_create / mrf_knn_laplacian / mrf_laplacian_apply / _quad."""
import ctypes

import torch

from ._lib import check, lib
from .util import need, ptr, stream_ptr


class PatchGraph:
    """K-NN patch graph Laplacian on n x n maps with p x p patches at stride s."""

    def __init__(self, n, p, s, k_max, max_frames=1024):
        self.n, self.p, self.s = int(n), int(p), int(s)
        h = ctypes.c_void_p()
        check(lib.mrf_graph_create(self.n, self.p, self.s, int(k_max), int(max_frames), ctypes.byref(h)),
              "mrf_graph_create")
        self.handle = h

    def build(self, maps, K, sigma2=0.0, stream=None):
        need(maps, torch.float32, (3, self.n, self.n), "maps")
        check(lib.mrf_knn_laplacian(self.handle, ptr(maps), int(K), float(sigma2), stream_ptr(stream)),
              "mrf_knn_laplacian")

    def info(self, stream=None):
        np_, nnz = ctypes.c_int(), ctypes.c_int()
        rp, col, val = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        sig2, lmax = ctypes.c_double(), ctypes.c_double()
        check(lib.mrf_graph_info(self.handle, ctypes.byref(np_), ctypes.byref(nnz), ctypes.byref(rp),
                                 ctypes.byref(col), ctypes.byref(val), ctypes.byref(sig2), ctypes.byref(lmax),
                                 stream_ptr(stream)), "mrf_graph_info")
        return dict(np=np_.value, nnz=nnz.value, rowptr=rp.value, col=col.value, val=val.value,
                    sigma2=sig2.value, lmax=lmax.value)

    def csr(self, device):
        """Copies the CSR arrays into tensors (rowptr, col, val)."""
        inf = self.info()
        n, nnz = inf["np"], inf["nnz"]
        out = (torch.empty(n + 1, dtype=torch.int32, device=device), torch.empty(nnz, dtype=torch.int32, device=device),
               torch.empty(nnz, dtype=torch.float32, device=device))
        torch.cuda.synchronize()
        for t, src in zip(out, (inf["rowptr"], inf["col"], inf["val"])):
            if t.numel():
                check(_copy_d2d(t, src), "hipMemcpy")
        return out + (inf,)

    def apply(self, X, out=None, stream=None):
        L = X.shape[0]
        need(X, torch.complex64, (L, self.n, self.n), "X")
        if out is None:
            out = torch.empty_like(X)
        check(lib.mrf_laplacian_apply(self.handle, ptr(X), ptr(out), int(L), stream_ptr(stream)),
              "mrf_laplacian_apply")
        return out

    def quad(self, X, stream=None):
        L = X.shape[0]
        need(X, torch.complex64, (L, self.n, self.n), "X")
        out = torch.empty(1, dtype=torch.float64, device=X.device)
        check(lib.mrf_laplacian_quad(self.handle, ptr(X), int(L), ptr(out), stream_ptr(stream)),
              "mrf_laplacian_quad")
        return out

    def close(self):
        if getattr(self, "handle", None):
            lib.mrf_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_hip = None


def _copy_d2d(dst, src_ptr):
    """Device-to-device copy of dst.numel() elements from a raw device pointer (hipMemcpy)."""
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
    return _hip.hipMemcpy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src_ptr),
                          dst.numel() * dst.element_size(), 3)
