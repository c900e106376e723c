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


class ReconParams(ctypes.Structure):
    _fields_ = [("p", c_int), ("s", c_int), ("K", c_int), ("rank_cap", c_int), ("lam1_0", c_float),
                ("lam2", c_float), ("beta", c_float), ("mu0", c_float), ("lamA", ctypes.c_double),
                ("sigma2", c_float), ("n_max", c_int), ("tol", ctypes.c_double), ("serial", c_int)]


class MlpTrainCfg(ctypes.Structure):
    _fields_ = [("batch", c_int), ("steps", c_int), ("first_step", c_int), ("total_steps", c_int), ("lr", c_float),
                ("beta1", c_float), ("beta2", c_float), ("eps", c_float), ("cosine", c_int), ("snr_lo", c_float),
                ("snr_hi", c_float), ("seed", ctypes.c_uint64), ("bf16", c_int)]


MAX_ITERS = 512
_D = ctypes.c_double * (MAX_ITERS + 1)


class ReconStats(ctypes.Structure):
    _fields_ = [("iters", c_int), ("stop_reason", c_int), ("n_graph", c_int), ("cost", _D), ("data", _D),
                ("tr", _D), ("nuc", _D), ("mu", _D), ("lam1", _D), ("sigma2", _D), ("lmax", _D),
                ("iter_ms", _D)]


def _decl(name, args, res=c_int):
    f = getattr(lib, name)
    f.argtypes = args
    f.restype = res
    return f


_decl("mrf_status_string", [c_int], c_char_p)
_decl("mrf_last_error", [], c_char_p)
_decl("mrf_version", [], c_int)
_decl("mrf_build_info", [], c_char_p)
_decl("mrf_timing_enable", [c_int])
_decl("mrf_timing_report", [c_char_p, c_size_t])
_decl("mrf_nufft_plan_create", [P(NufftDesc), c_void_p, c_void_p, P(c_void_p)])
_decl("mrf_nufft_plan_destroy", [c_void_p])
_decl("mrf_nufft_workspace_size", [c_void_p, P(c_size_t)])
_decl("mrf_nufft_fwd", [c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p])
_decl("mrf_nufft_adj", [c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p])
_decl("mrf_nufft_opnorm", [c_void_p, c_int, ctypes.c_uint, P(ctypes.c_double), c_void_p])
_decl("mrf_cart_plan_create", [c_int, c_int, c_void_p, c_void_p, P(c_void_p)])
_decl("mrf_epg_fisp", [c_int, c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_float, c_void_p,
                       c_void_p])
_decl("mrf_epg_random_params", [c_int, ctypes.c_uint64, c_float, c_float, c_float, c_float, c_float, c_float,
                                c_void_p, c_void_p])
_decl("mrf_epg_params_to_columns", [c_int, c_void_p, c_void_p, c_void_p])
_decl("mrf_toeplitz_create", [P(NufftDesc), c_void_p, c_void_p, P(c_void_p)])
_decl("mrf_toeplitz_destroy", [c_void_p])
_decl("mrf_toeplitz_workspace_size", [c_void_p, P(c_size_t)])
_decl("mrf_toeplitz_normal", [c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p])
_decl("mrf_nufft_fwd_mc", [c_void_p, c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p])
_decl("mrf_nufft_adj_mc", [c_void_p, c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p])
_decl("mrf_nufft_opnorm_mc", [c_void_p, c_void_p, c_int, c_int, ctypes.c_uint, P(ctypes.c_double), c_void_p])
_decl("mrf_nufft_autotune", [P(NufftDesc), c_void_p, c_int, P(c_int), P(c_float), c_void_p])
_decl("mrf_graph_create", [c_int, c_int, c_int, c_int, c_int, P(c_void_p)])
_decl("mrf_graph_destroy", [c_void_p])
_decl("mrf_knn_laplacian", [c_void_p, c_void_p, c_int, c_float, c_void_p])
_decl("mrf_graph_info", [c_void_p, P(c_int), P(c_int), P(c_void_p), P(c_void_p), P(c_void_p),
                         P(ctypes.c_double), P(ctypes.c_double), c_void_p])
_decl("mrf_laplacian_apply", [c_void_p, c_void_p, c_void_p, c_int, c_void_p])
_decl("mrf_laplacian_quad", [c_void_p, c_void_p, c_int, c_void_p, c_void_p])
_decl("mrf_llr_workspace_size", [c_int, c_int, c_int, c_int, c_int, P(c_size_t)])
_decl("mrf_llr_prox", [c_void_p, c_void_p, c_int, c_int, c_int, c_int, c_float, c_int, c_void_p, c_void_p,
                       c_size_t, c_void_p])
_decl("mrf_llr_xupdate_workspace_size", [c_int, c_int, c_int, c_int, c_int, P(c_size_t)])
_decl("mrf_llr_xupdate", [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_int, c_int, c_float, c_int,
                          ctypes.c_double, c_void_p, c_void_p, c_size_t, c_void_p])
_decl("mrf_subspace_coeffs_workspace_size", [c_int, c_int, c_int, P(c_size_t)])
_decl("mrf_subspace_coeffs", [c_void_p, c_void_p, c_int, c_int, c_int, c_void_p, c_void_p, c_size_t, c_void_p])
_decl("mrf_subspace_coeffs_noalloc", [c_void_p, c_void_p, c_int, c_int, c_int, c_void_p, c_void_p])
_decl("mrf_subspace_project", [c_void_p, c_void_p, c_int, c_int, c_int, c_void_p, c_void_p, c_size_t, c_void_p])
_decl("mrf_dict_create", [c_void_p, c_void_p, c_int, c_int, c_int, c_void_p, c_int, c_void_p, P(c_void_p)])
_decl("mrf_dict_destroy", [c_void_p])
_decl("mrf_dict_match_subspace", [c_void_p, c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p])
_decl("mrf_dict_match_workspace_size", [c_void_p, c_int, c_int, P(c_size_t)])
_decl("mrf_dict_match", [c_void_p, c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                         c_size_t, c_void_p])
_decl("mrf_dict_match_depth", [c_void_p, c_void_p, c_int, c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p,
                               c_void_p, c_void_p, c_size_t, c_void_p])
_decl("mrf_frames_to_voxels", [c_void_p, c_int, c_int, c_void_p, c_void_p])
_u64 = ctypes.c_uint64
_decl("mrf_mlp_create", [c_int, c_int, c_int, c_int, _u64, c_void_p, P(c_void_p)])
_decl("mrf_mlp_destroy", [c_void_p])
_decl("mrf_mlp_param_count", [c_void_p, P(c_size_t)])
_decl("mrf_mlp_params", [c_void_p, P(c_void_p), P(c_void_p)])
_decl("mrf_mlp_reset_optimizer", [c_void_p, c_void_p])
_decl("mrf_mlp_set_grid", [c_void_p, c_int, ctypes.c_double, ctypes.c_double, c_int, ctypes.c_double, ctypes.c_double,
                           c_void_p, c_void_p])
_decl("mrf_mlp_target_stats", [c_void_p, c_void_p, c_void_p, c_void_p])
_decl("mrf_mlp_train_workspace_size", [c_void_p, c_int, P(c_size_t)])
_decl("mrf_mlp_state_bytes", [c_void_p, P(c_size_t)])
_decl("mrf_mlp_save", [c_void_p, c_void_p, c_size_t, c_void_p])
_decl("mrf_mlp_load", [c_void_p, c_void_p, c_size_t, c_void_p])
_decl("mrf_mlp_synth", [c_void_p, c_void_p, _u64, c_int, c_int, c_float, c_float, c_void_p, c_void_p, c_void_p, c_void_p])
_decl("mrf_mlp_forward", [c_void_p, c_void_p, c_int, c_int, c_void_p, c_void_p, c_size_t, c_void_p])
_decl("mrf_mlp_grads", [c_void_p, c_void_p, c_void_p, c_int, c_int, c_void_p, c_void_p, c_size_t, c_void_p])
_decl("mrf_mlp_adam_step", [c_void_p, c_float, c_float, c_float, c_float, c_void_p])
_decl("mrf_mlp_train", [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p])
_decl("mrf_mlp_match_workspace_size", [c_void_p, c_int, P(c_size_t)])
_decl("mrf_mlp_match", [c_void_p, c_void_p, c_void_p, c_int, c_int, c_float, c_void_p, c_void_p, c_void_p, c_void_p,
                        c_void_p, P(c_int), c_void_p, c_size_t, c_void_p])
_decl("mrf_recon_create", [P(ReconParams), c_void_p, c_void_p, P(c_void_p)])
_decl("mrf_recon_destroy", [c_void_p])
_decl("mrf_recon_batched", [c_int, c_void_p, c_void_p, c_int, P(c_int)])
_decl("mrf_recon_init", [c_void_p, c_void_p, c_void_p, c_void_p])
_decl("mrf_recon_set_coils", [c_void_p, c_void_p, c_int, c_void_p])
_decl("mrf_recon_set_toeplitz", [c_void_p, c_void_p, c_void_p])
_decl("mrf_recon_iterate", [c_void_p, c_int, P(c_int), c_void_p])
_decl("mrf_recon_set_serial", [c_void_p, c_int])
_decl("mrf_recon_finish", [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p])
_decl("mrf_recon_get_stats", [c_void_p, P(ReconStats)])
_decl("mrf_recon_set_final_match", [c_void_p, c_int, c_void_p, c_float])
_decl("mrf_recon_checkpoint_bytes", [c_void_p, P(c_size_t)])
_decl("mrf_recon_checkpoint_save", [c_void_p, c_void_p, c_size_t, c_void_p])
_decl("mrf_recon_checkpoint_load", [c_void_p, c_void_p, c_void_p, c_size_t, c_void_p])
_decl("mrf_recon_inject_graph", [c_void_p, c_int, c_int, P(c_int), P(c_int), P(c_float), ctypes.c_double,
                                 ctypes.c_double])
_decl("mrf_recon", [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, P(ReconStats), c_void_p])


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


def build_info():
    """{'sources-sha256': ..., 'built': ..., 'arch': ...} of the loaded library (mrf_build_info)."""
    return dict(kv.split("=", 1) for kv in lib.mrf_build_info().decode().split())


def built_from_current_sources():
    """True when the loaded library's source hash equals the hash of the sources in this tree."""
    from . import build
    return build_info().get("sources-sha256") == build.source_sha()
