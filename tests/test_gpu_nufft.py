"""GPU parity of the NUFFT pair (mrf_nufft_fwd / mrf_nufft_adj) against the FP64 oracle.

Bar: rel-L2 <= 1e-5 per the FP32-operator tolerance; both sides use the same gridding
(KB width 6 on the 2x grid), so the difference measures FP32 rounding only.
"""
import math

import numpy as np
import pytest
import torch

import mrfgen
from oracle import nufft as onufft
from tests.gpu_util import rel_l2, say, to_dev

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _rand(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)


def _edge_traj(rng, L, Ns):
    t = rng.uniform(-math.pi, math.pi, (L, Ns, 2)).astype(np.float32)
    # special positions: the -pi edge, just below +pi, the origin, exact grid points
    t[:, 0] = [-math.pi, -math.pi]
    t[:, 1] = [np.nextafter(np.float32(math.pi), 0), 0.0]
    t[:, 2] = [0.0, 0.0]
    t[:, 3] = [2 * math.pi * 3 / 32, -2 * math.pi * 5 / 32]
    return t


@pytest.mark.parametrize("N,L,Ns,tx", [(16, 3, 37, 0), (32, 4, 200, 8), (32, 2, 1, 16), (64, 3, 333, 32),
                                       (128, 2, 700, 0), (192, 2, 500, 0), (192, 3, 301, 16), (256, 2, 257, 0),
                                       (320, 2, 600, 0), (512, 1, 300, 0)])
def test_random_trajectory_parity(N, L, Ns, tx):
    from paper_2310_05647_amd import NufftPlan
    say(f"nufft parity N={N} L={L} Ns={Ns} tile_cols={tx}")
    rng = np.random.default_rng(N + Ns)
    traj = _edge_traj(rng, L, Ns) if Ns >= 4 else rng.uniform(-3, 3, (L, Ns, 2)).astype(np.float32)
    X = _rand(rng, L, N, N)
    y = _rand(rng, L, Ns)
    plan = NufftPlan(N, to_dev(traj), tile_cols=tx)
    b = plan.fwd(to_dev(X)).cpu().numpy()
    a = plan.adj(to_dev(y)).cpu().numpy()
    eb = rel_l2(b, onufft.nufft_fwd(X, traj))
    ea = rel_l2(a, onufft.nufft_adj(y, traj, N))
    say(f"  fwd rel-L2 {eb:.2e}  adj rel-L2 {ea:.2e}")
    assert eb <= TOL and ea <= TOL


def test_c1_spiral_parity_all_frames():
    from paper_2310_05647_amd import NufftPlan
    cfg = mrfgen.get_config("C1")
    say("nufft parity C1 (64x64, L=100, Ns=1024)")
    traj = mrfgen.vds_spiral(cfg["N"], cfg["L"], cfg["Ns"], cfg["n_interleaves"])
    ph = mrfgen.make_phantom(cfg, 1)
    X = mrfgen.truth_fingerprints(cfg, ph)
    rng = np.random.default_rng(0)
    y = _rand(rng, cfg["L"], cfg["Ns"])
    plan = NufftPlan(cfg["N"], to_dev(traj))
    b = plan.fwd(to_dev(X)).cpu().numpy()
    a = plan.adj(to_dev(y)).cpu().numpy()
    eb, ea = rel_l2(b, onufft.nufft_fwd(X, traj)), rel_l2(a, onufft.nufft_adj(y, traj, cfg["N"]))
    say(f"  fwd {eb:.2e} adj {ea:.2e}")
    assert eb <= TOL and ea <= TOL


def test_c2_full_size_sampled_frames_and_adjoint_identity():
    from paper_2310_05647_amd import NufftPlan
    cfg = mrfgen.get_config("C2")
    N, L, Ns = cfg["N"], cfg["L"], cfg["Ns"]
    say("nufft parity C2 full size (256x256, L=1000, Ns=2048), sampled frames")
    traj = mrfgen.vds_spiral(N, L, Ns, cfg["n_interleaves"])
    rng = np.random.default_rng(2)
    X = _rand(rng, L, N, N)
    y = _rand(rng, L, Ns)
    plan = NufftPlan(N, to_dev(traj))
    Xd, yd = to_dev(X), to_dev(y)
    b = plan.fwd(Xd)
    a = plan.adj(yd)
    torch.cuda.synchronize()
    frames = [0, 1, 517, L - 1]
    bh, ah = b.cpu().numpy(), a.cpu().numpy()
    for f in frames:
        eb = rel_l2(bh[f], onufft.nufft_fwd(X[f:f + 1], traj[f:f + 1])[0])
        ea = rel_l2(ah[f], onufft.nufft_adj(y[f:f + 1], traj[f:f + 1], N)[0])
        say(f"  frame {f}: fwd {eb:.2e} adj {ea:.2e}")
        assert eb <= TOL and ea <= TOL
    lhs = np.vdot(bh.astype(np.complex128), y.astype(np.complex128))
    rhs = np.vdot(X.astype(np.complex128), ah.astype(np.complex128))
    say(f"  adjoint identity rel diff {abs(lhs - rhs) / abs(lhs):.2e}")
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


def test_adjoint_is_deterministic():
    from paper_2310_05647_amd import NufftPlan
    cfg = mrfgen.get_config("C1")
    traj = mrfgen.vds_spiral(cfg["N"], cfg["L"], cfg["Ns"], cfg["n_interleaves"])
    y = to_dev(_rand(np.random.default_rng(3), cfg["L"], cfg["Ns"]))
    plan = NufftPlan(cfg["N"], to_dev(traj))
    a1 = plan.adj(y).clone()
    a2 = plan.adj(y)
    assert torch.equal(a1, a2)
