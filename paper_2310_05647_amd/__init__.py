"""Python binding of libmrf, the MI355X hot path of the MS-LLR MRF reconstruction.

Argument marshalling only: every step runs in the HIP kernels of libmrf.so. Tensors are
torch device tensors (PyTorch provides device memory and the stream); their data pointers
and the current HIP stream are handed to the C-ABI calls of include/mrf.h. Importing this
package fails loudly when libmrf.so has not been built.
"""
from ._lib import (MrfError, build_info, built_from_current_sources, check, lib, library_path,  # noqa: F401
                   timing_enable, timing_report)
from .nufft import CartPlan, NufftPlan, Toeplitz, autotune  # noqa: F401
from .epg import epg_fisp, params_columns, random_params  # noqa: F401
from .graph import PatchGraph  # noqa: F401
from .llr import llr_prox, llr_xupdate  # noqa: F401
from .subspace import (Dictionary, frames_to_voxels, subspace_coeffs, subspace_coeffs_noalloc,  # noqa: F401
                       subspace_project)
from .recon import Recon, recon_batched  # noqa: F401
from .mlp import MLP  # noqa: F401
