"""Seeded synthetic inputs for the MS-LLR MRF reconstruction (arXiv 2310.05647).

This package is shared by the CPU oracle's tests and by the GPU library's tests and
benchmark. It draws random numbers and simulates the inputs the method takes
(sequence, dictionary + look-up table, projection basis, phantom maps, ground-truth
fingerprints, trajectories and Cartesian masks, coil sensitivities, measurement noise). It contains none of the
reconstruction's own arithmetic: no NUFFT, no patch operator, no graph, no
thresholding and no matching.
"""
from .configs import CONFIGS, get_config
from .sequence import fisp_sequence
from .dictionary import make_dictionary, param_grid
from .subspace import subspace_basis
from .phantom import make_phantom
from .fingerprints import truth_fingerprints
from .traj import radial_cartesian_mask, vds_spiral
from .noise import complex_noise, noise_sigma
from .coils import coil_maps

__all__ = [
    "CONFIGS", "get_config", "fisp_sequence", "make_dictionary", "param_grid",
    "subspace_basis", "make_phantom", "truth_fingerprints", "vds_spiral", "radial_cartesian_mask",
    "complex_noise", "noise_sigma", "coil_maps",
]
