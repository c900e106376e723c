"""Loads libmrf.so and declares the C-ABI signatures of include/mrf.h."""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libmrf.so")

if not os.path.exists(library_path):
    raise ImportError(
        "libmrf.so is not built (%s). Build it with `python paper_2310_05647_amd/build.py` "
        "or __graft_entry__.build(); there is no fallback implementation." % library_path)

lib = ctypes.CDLL(library_path)

c_int, c_float, c_size_t, c_void_p = ctypes.c_int, ctypes.c_float, ctypes.c_size_t, ctypes.c_void_p
c_char_p = ctypes.c_char_p
P = ctypes.POINTER


class NufftDesc(ctypes.Structure):
    _fields_ = [("n", c_int), ("nframes", c_int), ("nsamp", c_int), ("kb_width", c_int),
                ("oversamp", c_int), ("tile_cols", c_int)]


def _decl(name, args, res=c_int):
    f = getattr(lib, name)
    f.argtypes = args
    f.restype = res
    return f


_decl("mrf_status_string", [c_int], c_char_p)
_decl("mrf_last_error", [], c_char_p)
_decl("mrf_version", [], c_int)
_decl("mrf_timing_enable", [c_int])
_decl("mrf_timing_report", [c_char_p, c_size_t])
_decl("mrf_nufft_plan_create", [P(NufftDesc), c_void_p, c_void_p, P(c_void_p)])
_decl("mrf_nufft_plan_destroy", [c_void_p])
_decl("mrf_nufft_workspace_size", [c_void_p, P(c_size_t)])
_decl("mrf_nufft_fwd", [c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p])
_decl("mrf_nufft_adj", [c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p])


class MrfError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = "%s failed: %s (%s)" % (where, lib.mrf_status_string(status).decode(),
                                       lib.mrf_last_error().decode())
        super().__init__(msg)


def check(status, where):
    if status != 0:
        raise MrfError(status, where)


def timing_enable(on=True):
    check(lib.mrf_timing_enable(1 if on else 0), "mrf_timing_enable")


def timing_report():
    """Synchronises recorded launch events; returns {kernel: (launches, total_ms, min_ms, max_ms)}."""
    buf = ctypes.create_string_buffer(1 << 16)
    check(lib.mrf_timing_report(buf, len(buf)), "mrf_timing_report")
    out = {}
    for line in buf.value.decode().splitlines():
        name, n, tot, mn, mx = line.split()
        out[name] = (int(n), float(tot), float(mn), float(mx))
    return out
