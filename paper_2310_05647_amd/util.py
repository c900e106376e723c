"""Marshalling helpers shared by the binding modules."""
import ctypes

import torch


def stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def need(t, dtype, shape, name):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous() and tuple(t.shape) == tuple(shape)):
        raise ValueError("%s must be a contiguous CUDA %s tensor of shape %s (got %s %s %s)"
                         % (name, dtype, tuple(shape), t.dtype, tuple(t.shape), t.device))


def workspace(nbytes, device):
    return torch.empty(max(1, int(nbytes)), dtype=torch.uint8, device=device)


_hip = None


def _hiplib():
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
    return _hip


def copy_from_ptr(dst, src_ptr):
    """dst (device tensor) <- dst.numel() elements at a raw device pointer (hipMemcpy, device to device)."""
    return _hiplib().hipMemcpy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src_ptr),
                               dst.numel() * dst.element_size(), 3)


def copy_to_ptr(dst_ptr, src):
    """src.numel() elements of a device tensor -> a raw device pointer (hipMemcpy, device to device)."""
    return _hiplib().hipMemcpy(ctypes.c_void_p(dst_ptr), ctypes.c_void_p(src.data_ptr()),
                               src.numel() * src.element_size(), 3)
