"""Pseudo-radial Cartesian sampling on the GPU (mrf_cart_plan_create: A_l = M_l F, F the unitary
centred DFT) against the FP64 oracle (oracle.cartesian), and Algorithm 1 on it.

  * the pair: rel-L2 <= 1e-5 (the FP32-operator bar) for every supported size class, exact zeros
    off the mask, the adjoint identity, and the multi-coil pair;
  * Algorithm 1 on the oracle's graphs: X, costs and step sizes within the non-Cartesian recon's
    bars;
  * the LLR-only ablation (lambda1^0 = 0): the manifold term is off, so no graph enters the
    iterate and the two runs follow each other freely; X and the data term within 1e-5 after 10
    iterations, the nuclear-norm term within the floor of its FP32 patch Gram.
"""
import numpy as np
import pytest
import torch

import mrfgen
from oracle import cartesian as ocart
from oracle import recon as orecon
from tests.gpu_util import nuc_fp32_gram, rel_l2, say, to_dev
from tests.workloads import cart_workload

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _rand(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)


@pytest.mark.parametrize("N,L,spokes", [(32, 3, 3), (64, 2, 5), (192, 2, 9), (256, 2, 13), (320, 1, 16),
                                        (512, 1, 25)])
def test_cartesian_pair_parity(N, L, spokes):
    from paper_2310_05647_amd import CartPlan
    say(f"cartesian pair N={N} L={L} spokes={spokes}")
    rng = np.random.default_rng(N)
    mask = mrfgen.radial_cartesian_mask(N, L, spokes)
    X, Y = _rand(rng, L, N, N), _rand(rng, L, N, N)
    plan = CartPlan(to_dev(mask))
    b = plan.fwd(to_dev(X)).cpu().numpy().reshape(L, N, N)
    a = plan.adj(to_dev(Y.reshape(L, N * N))).cpu().numpy()
    rb, ra = ocart.cart_fwd(X, mask), ocart.cart_adj(Y, mask)
    eb, ea = rel_l2(b, rb), rel_l2(a, ra)
    say(f"  fwd rel-L2 {eb:.2e}  adj rel-L2 {ea:.2e}  sampled {mask.mean():.3f}")
    assert eb <= TOL and ea <= TOL
    assert np.all(b[mask == 0] == 0)
    lhs = np.vdot(b.astype(np.complex128), Y.astype(np.complex128))
    rhs = np.vdot(X.astype(np.complex128), a.astype(np.complex128))
    assert abs(lhs - rhs) <= 1e-5 * np.linalg.norm(b) * np.linalg.norm(Y)


def test_cartesian_multicoil_pair_parity():
    from paper_2310_05647_amd import CartPlan
    rng = np.random.default_rng(9)
    N, L, Nc = 128, 3, 4
    mask = mrfgen.radial_cartesian_mask(N, L, 7)
    S = mrfgen.coil_maps(N, Nc, seed=3)
    X, Y = _rand(rng, L, N, N), _rand(rng, Nc, L, N, N)
    plan = CartPlan(to_dev(mask))
    b = plan.fwd_mc(to_dev(S), to_dev(X)).cpu().numpy().reshape(Nc, L, N, N)
    a = plan.adj_mc(to_dev(S), to_dev(Y.reshape(Nc, L, N * N))).cpu().numpy()
    eb = rel_l2(b, ocart.cart_fwd_mc(X, mask, S))
    ea = rel_l2(a, ocart.cart_adj_mc(Y, mask, S))
    say(f"  multi-coil cartesian fwd {eb:.2e} adj {ea:.2e}")
    assert eb <= TOL and ea <= TOL
    lam = plan.opnorm_mc(to_dev(S), iters=30)
    assert lam <= 1.0 + 1e-4          # sum_c |S_c|^2 = 1, F unitary, M a projection


def _gpu_recon(w, n_max, lam1_0=None, graphs=None):
    from paper_2310_05647_amd import CartPlan, Dictionary, Recon
    cfg = w["cfg"]
    plan = CartPlan(to_dev(w["mask"]))
    d = Dictionary(to_dev(w["atoms"]), to_dev(w["grid"]["lut"]), to_dev(w["V"]))
    rc = Recon(plan, d, cfg["p"], cfg["s"], cfg["K"], cfg["r_llr"],
               lam1_0=cfg["lam1_0"] if lam1_0 is None else lam1_0, lam2=cfg["lam2"], beta=cfg["beta"],
               mu0=cfg["mu0"], lamA=w["lamA"], n_max=n_max, tol=-1.0)
    if graphs is not None:
        st = graphs["stats"]
        for k, Lap in enumerate(st["graphs"]):
            rc.inject_graph(k, Lap, st["sigma2"][k], st["lmax"][k])
    N, L = cfg["N"], cfg["L"]
    out = rc.run(to_dev(w["b"].reshape(L, N * N)))
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if torch.is_tensor(v) else v) for k, v in out.items()}


def _oracle(w, n_max, lam1_0=None):
    cfg = w["cfg"]
    return orecon.recon(w["b"], None, w["atoms"], w["grid"]["lut"], w["V"], cfg["N"], cfg["p"], cfg["s"], cfg["K"],
                        cfg["r_llr"], lam1_0=cfg["lam1_0"] if lam1_0 is None else lam1_0, lam2=cfg["lam2"],
                        beta=cfg["beta"], mu0=cfg["mu0"], lamA=w["lamA"], n_max=n_max, keep_graphs=True,
                        mask=w["mask"])


def test_cartesian_recon_follows_the_oracle_with_its_graphs():
    w = cart_workload()
    o = _oracle(w, 8)
    say("cartesian recon: 8 iterations on the oracle's graphs")
    g = _gpu_recon(w, 8, graphs=o)
    cg, co = np.array(g["stats"]["cost"]), np.array(o["stats"]["cost"])
    ec = np.abs(cg - co) / co
    emu = np.max(np.abs(np.array(g["stats"]["mu"]) - np.array(o["stats"]["mu"])) / np.array(o["stats"]["mu"]))
    ex = rel_l2(g["X"], o["X"])
    agree = float(np.mean(g["idx"] == o["idx"]))
    say(f"  X rel-L2 {ex:.2e}; cost rel {ec.max():.2e}; mu rel {emu:.2e}; index agreement {agree:.4f}")
    # the cost of Algorithm 1 changes with every rebuilt graph (lambda1 and L), so it need not fall
    # monotonically here (the oracle's does not either); the GPU follows it value by value
    assert g["stats"]["iters"] == 8
    assert ex <= 1e-5 and ec.max() <= 1e-5 and emu <= 1e-6
    assert agree >= 0.995


def test_llr_only_ablation_runs_freely_with_the_oracle():
    """lambda1^0 = 0: no graph enters the iterate (the step size is min(mu0, 1/lamA)), so both runs
    take their own graphs and still agree: X and the data term within 1e-5, no manifold term.

    The nuclear-norm term of the cost is the one reported value that does not reach 1e-5 here: the
    GPU takes the singular values as square roots of the eigenvalues of a patch Gram formed in FP32,
    whose rounding (about L u |Q|_F^2) turns each vanishing singular value into up to
    sqrt(L u) sigma_1. The SVT, which zeroes those values, and X are unaffected; the cost's nuclear
    norm reads high by that floor. Its bar is three times the floor of an FP32 Gram of the oracle's
    own X (the difference has the size that mechanism produces, and no more)."""
    w = cart_workload()
    cfg = w["cfg"]
    o = _oracle(w, 10, lam1_0=0.0)
    g = _gpu_recon(w, 10, lam1_0=0.0)
    st = g["stats"]
    data_o = np.array([t[0] for t in o["stats"]["terms"]])
    nuc_o = np.array([t[2] for t in o["stats"]["terms"]])
    ex = rel_l2(g["X"], o["X"])
    # relative to the cost: at n = 0 the data term vanishes (X^0 = F^H M b and b is zero off the mask)
    ed = np.max(np.abs(np.array(st["data"]) - data_o) / np.array(o["stats"]["cost"]))
    en = abs(st["nuc"][-1] - nuc_o[-1]) / nuc_o[-1]
    floor = abs(nuc_fp32_gram(o["X"], cfg["p"], cfg["s"]) - nuc_o[-1]) / nuc_o[-1]
    say(f"LLR-only (lambda1^0 = 0), 10 iterations: X rel-L2 {ex:.2e}, data term rel {ed:.2e}, "
        f"nuclear norm rel {en:.2e} (FP32-Gram floor on the oracle's X {floor:.2e})")
    assert ex <= 1e-5 and ed <= 1e-5
    assert en <= 3 * floor + 1e-5
