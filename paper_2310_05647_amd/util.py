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
