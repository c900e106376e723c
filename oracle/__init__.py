"""CPU oracle for the MS-LLR reconstruction (arXiv 2310.05647). TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct FP64 / complex128 NumPy implementation of every step
of the GPU hot path. It exists to check the GPU library. Only the tests, the smoke
check and the benchmark's CPU-baseline leg may import it; the GPU library never calls
it, and it imports nothing from the GPU library. Library primitives (numpy.fft,
numpy.linalg) serve as single steps; nothing is blocked, fused or reordered.

Modules and the passages they follow:
  nufft    A = F_u (single coil) and its adjoint, eq. (1); KB gridding, NUDFT
  patches  patch extractor Q_q, Casorati Q(X), adjoint Q*, eqs. (7), (9), (13)
  graph    patch weights and graph Laplacian, eqs. (8), (10), (11)
  ops      Laplacian apply (eq. (15)), projection P_S (eq. (17)), SVT (eq. (22)),
           X update (eq. (23)), cost (Algorithm 1)
  match    pattern matching Phi_D, eqs. (4)-(5)
  recon    Algorithm 1
  mlp      the learned matcher (20-256-256-256-2 MLP), forward / backward / Adam
  metrics  SNR eq. (24), NMSE eq. (25)

Functions without an independent pin say "parity unpinned" in their docstring.
"""
from . import nufft, patches, graph, ops, match, recon, mlp, metrics  # noqa: F401
