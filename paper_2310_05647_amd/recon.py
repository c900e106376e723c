"""Algorithm 1 binding: mrf_recon_create / set_coils / init / iterate / finish."""
import ctypes

import numpy as np
import torch

from ._lib import ReconParams, ReconStats, check, lib
from .util import need, ptr, stream_ptr


class Recon:
    """MS-LLR solver state for a NUFFT plan and a dictionary with a basis."""

    def __init__(self, plan, dictionary, p, s, K, rank_cap, lam1_0=0.1, lam2=0.1, beta=0.2, mu0=1.0, lamA=0.0,
                 sigma2=0.0, n_max=10, tol=-1.0, serial=0):
        """serial: bit 0 keeps the cost terms, bit 1 the rest of an iteration on the caller's stream
        (0: independent parts overlap on the recon's own streams; the results are the same)."""
        self.plan, self.dict = plan, dictionary
        self.params = ReconParams(int(p), int(s), int(K), int(rank_cap), float(lam1_0), float(lam2), float(beta),
                                  float(mu0), float(lamA), float(sigma2), int(n_max), float(tol), int(serial))
        h = ctypes.c_void_p()
        check(lib.mrf_recon_create(ctypes.byref(self.params), plan.handle, dictionary.handle, ctypes.byref(h)),
              "mrf_recon_create")
        self.handle = h
        self.n, self.L = plan.n, plan.L
        self.ncoils = 0

    def set_coils(self, smaps, stream=None):
        """Multi-coil data (eq. (1)): smaps [ncoils, n, n] complex64 (device; copied), or None for a
        single coil. b then is [ncoils, L, Ns] and lamA should come from plan.opnorm_mc(smaps)."""
        if smaps is None:
            check(lib.mrf_recon_set_coils(self.handle, None, 0, stream_ptr(stream)), "mrf_recon_set_coils")
            self.ncoils = 0
            return
        if smaps.dim() != 3:
            raise ValueError("smaps must be [ncoils, n, n]")
        need(smaps, torch.complex64, (smaps.shape[0], self.n, self.n), "smaps")
        check(lib.mrf_recon_set_coils(self.handle, ptr(smaps), smaps.shape[0], stream_ptr(stream)),
              "mrf_recon_set_coils")
        self.ncoils = smaps.shape[0]

    def set_toeplitz(self, toeplitz, stream=None):
        """Data-term gradient and value through a Toeplitz normal operator (built from this plan's
        trajectory), or None for the gridded pair; call before init."""
        self._toeplitz = toeplitz   # kept alive: the recon holds its handle by pointer
        check(lib.mrf_recon_set_toeplitz(self.handle, toeplitz.handle if toeplitz is not None else None,
                                         stream_ptr(stream)), "mrf_recon_set_toeplitz")

    def _b_shape(self):
        return ((self.ncoils,) if self.ncoils else ()) + (self.L, self.plan.Ns)

    def init(self, b, X0=None, stream=None):
        need(b, torch.complex64, self._b_shape(), "b")
        self._b = b
        check(lib.mrf_recon_init(self.handle, ptr(b), ptr(X0), stream_ptr(stream)), "mrf_recon_init")

    def iterate(self, n, stream=None):
        stopped = ctypes.c_int()
        check(lib.mrf_recon_iterate(self.handle, int(n), ctypes.byref(stopped), stream_ptr(stream)),
              "mrf_recon_iterate")
        return bool(stopped.value)

    def inject_graph(self, k, L, sigma2, lmax):
        """Graph number k of the run is taken as given (mrf_recon_inject_graph): L is the dense
        Laplacian [Np, Np] (numpy, or a sparse matrix with .toarray()); its CSR keeps the non-zeros
        and the diagonal, as float32."""
        L = np.asarray(L.toarray() if hasattr(L, "toarray") else L)
        nz = (L != 0) | np.eye(L.shape[0], dtype=bool)
        rows, cols = np.nonzero(nz)                      # row-major: rows ascending, columns ascending
        rowptr = np.zeros(L.shape[0] + 1, np.int32)
        np.cumsum(np.bincount(rows, minlength=L.shape[0]), out=rowptr[1:])
        col = np.ascontiguousarray(cols, np.int32)
        val = np.ascontiguousarray(L[rows, cols], np.float32)
        ip = ctypes.POINTER(ctypes.c_int)
        check(lib.mrf_recon_inject_graph(self.handle, int(k), int(col.size), rowptr.ctypes.data_as(ip),
                                         col.ctypes.data_as(ip), val.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                         float(sigma2), float(lmax)), "mrf_recon_inject_graph")

    MATCH_MODES = {"subspace": 4, "fp32": 0, "bf16": 1, "fp8": 2, "learned": 3, "bf16x3": 5}

    def set_final_match(self, mode="subspace", mlp=None, theta=0.0):
        """The final match of the run (mrf_recon_set_final_match): "subspace" (default), "fp32",
        "bf16", "fp8" (full-length) or "learned" (with mlp and the gate threshold theta)."""
        check(lib.mrf_recon_set_final_match(self.handle, self.MATCH_MODES[mode], mlp.handle if mlp is not None else None,
                                            float(theta)), "mrf_recon_set_final_match")

    def checkpoint(self, stream=None):
        """The run's state between iterations (mrf_recon_checkpoint_save) as a host uint8 tensor."""
        n = ctypes.c_size_t()
        check(lib.mrf_recon_checkpoint_bytes(self.handle, ctypes.byref(n)), "mrf_recon_checkpoint_bytes")
        buf = torch.empty(n.value, dtype=torch.uint8)
        check(lib.mrf_recon_checkpoint_save(self.handle, ctypes.c_void_p(buf.data_ptr()), n.value, stream_ptr(stream)),
              "mrf_recon_checkpoint_save")
        return buf

    def restore(self, b, buf, stream=None):
        """Continues a run from checkpoint(); b are the run's measurements."""
        need(b, torch.complex64, self._b_shape(), "b")
        self._b = b
        check(lib.mrf_recon_checkpoint_load(self.handle, ptr(b), ctypes.c_void_p(buf.data_ptr()), buf.numel(),
                                            stream_ptr(stream)), "mrf_recon_checkpoint_load")

    def set_serial(self, serial):
        """Schedule mask for later iterations (see the constructor's serial)."""
        check(lib.mrf_recon_set_serial(self.handle, int(serial)), "mrf_recon_set_serial")

    def finish(self, stream=None):
        dev = self._b.device
        n, L = self.n, self.L
        X = torch.empty((L, n, n), dtype=torch.complex64, device=dev)
        maps = torch.empty((3, n, n), dtype=torch.float32, device=dev)
        idx = torch.empty(n * n, dtype=torch.int32, device=dev)
        rho = torch.empty(n * n, dtype=torch.float32, device=dev)
        check(lib.mrf_recon_finish(self.handle, ptr(X), ptr(maps), ptr(idx), ptr(rho), stream_ptr(stream)),
              "mrf_recon_finish")
        return dict(X=X, maps=maps, idx=idx, rho=rho)

    def stats(self):
        st = ReconStats()
        check(lib.mrf_recon_get_stats(self.handle, ctypes.byref(st)), "mrf_recon_get_stats")
        k = st.iters + 1
        g = st.n_graph
        return dict(iters=st.iters, stop=st.stop_reason, cost=list(st.cost[:k]), data=list(st.data[:k]),
                    tr=list(st.tr[:k]), nuc=list(st.nuc[:k]), mu=list(st.mu[:g]), lam1=list(st.lam1[:g]),
                    sigma2=list(st.sigma2[:g]), lmax=list(st.lmax[:g]), iter_ms=list(st.iter_ms[:k]))

    def run(self, b, X0=None, stream=None):
        self.init(b, X0, stream)
        self.iterate(self.params.n_max, stream)
        out = self.finish(stream)
        out["stats"] = self.stats()
        return out

    def close(self):
        if getattr(self, "handle", None):
            lib.mrf_recon_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def recon_batched(recons, streams, n):
    """Advances several initialised Recon objects by up to n iterations each, every slice's work on
    its own torch stream (mrf_recon_batched). Returns the number of slices still running."""
    if len(recons) != len(streams) or not recons:
        raise ValueError("need one stream per slice")
    hs = (ctypes.c_void_p * len(recons))(*[r.handle.value for r in recons])
    ss = (ctypes.c_void_p * len(streams))(*[s.cuda_stream for s in streams])
    active = ctypes.c_int()
    check(lib.mrf_recon_batched(len(recons), hs, ss, int(n), ctypes.byref(active)), "mrf_recon_batched")
    return active.value
