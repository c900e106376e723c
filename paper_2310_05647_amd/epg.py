"""FISP signal model by EPG on the device (mrf_epg_fisp) and off-grid parameter draws
(mrf_epg_random_params): dictionaries and training signals made on the GPU."""
import ctypes

import torch

from ._lib import check, lib
from .util import need, ptr, stream_ptr


def epg_fisp(t1, t2, fa_deg, tr_ms, te_ms, b1=None, n_states=24, out=None, stream=None):
    """Signals complex64 [M, L] (PD = 1) for float32 device tensors t1, t2 (and b1) [M] in ms and the
    train fa_deg, tr_ms [L]."""
    M, L = t1.numel(), fa_deg.numel()
    for t, name in ((t1, "t1"), (t2, "t2")):
        need(t, torch.float32, (M,), name)
    if b1 is not None:
        need(b1, torch.float32, (M,), "b1")
    need(fa_deg, torch.float32, (L,), "fa_deg")
    need(tr_ms, torch.float32, (L,), "tr_ms")
    if out is None:
        out = torch.empty((M, L), dtype=torch.complex64, device=t1.device)
    need(out, torch.complex64, (M, L), "out")
    check(lib.mrf_epg_fisp(M, L, int(n_states), ptr(t1), ptr(t2), ptr(b1), ptr(fa_deg), ptr(tr_ms), float(te_ms),
                           ptr(out), stream_ptr(stream)), "mrf_epg_fisp")
    return out


def random_params(n, seed, t1_range, t2_range, b1_range=(1.0, 1.0), device="cuda", stream=None):
    """float32 [n, 3] (T1, T2, B1): T1, T2 log-uniform with T2 <= T1, B1 uniform (Philox on the device)."""
    params = torch.empty((n, 3), dtype=torch.float32, device=device)
    check(lib.mrf_epg_random_params(int(n), ctypes.c_uint64(int(seed)), float(t1_range[0]), float(t1_range[1]),
                                    float(t2_range[0]), float(t2_range[1]), float(b1_range[0]), float(b1_range[1]),
                                    ptr(params), stream_ptr(stream)), "mrf_epg_random_params")
    return params


def params_columns(params, stream=None):
    """[3, n] float32 (T1 row, T2 row, B1 row) from params [n, 3]."""
    n = params.shape[0]
    need(params, torch.float32, (n, 3), "params")
    cols = torch.empty((3, n), dtype=torch.float32, device=params.device)
    check(lib.mrf_epg_params_to_columns(n, ptr(params), ptr(cols), stream_ptr(stream)), "mrf_epg_params_to_columns")
    return cols
