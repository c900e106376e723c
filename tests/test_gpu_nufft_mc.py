"""Multi-coil acquisition on the GPU (eq. (1): A = F_u C) against the FP64 oracle.

  * the pair mrf_nufft_fwd_mc / mrf_nufft_adj_mc: rel-L2 <= 1e-5 overall and per coil (the
    single-coil operator's FP32 bar; the map multiply adds one rounding per pixel);
  * a unit map on one coil gives the single-coil transforms bit for bit;
  * the adjoint identity <A x, y> = <x, A^H y> on the GPU's own outputs;
  * lambda_max of the multi-coil normal operator against the oracle's power iteration, and not
    above the single-coil one when sum_c |S_c|^2 = 1 (then (F_u C)^H F_u C <= lambda_max(A^H A));
  * Algorithm 1 with coils (mrf_recon_set_coils) on the oracle's graphs: X, costs and step sizes
    within the single-coil recon's bars; checkpoint/resume with coils bit for bit.
"""
import numpy as np
import pytest
import torch

import mrfgen
from oracle import nufft as onufft
from oracle import recon as orecon
from tests.gpu_util import rel_l2, say, to_dev
from tests.workloads import mc_workload

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _rand(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)


@pytest.mark.parametrize("N,L,Ns,Nc", [(32, 3, 200, 4), (64, 2, 333, 8), (32, 1, 1, 2), (128, 2, 517, 3)])
def test_multicoil_pair_parity(N, L, Ns, Nc):
    from paper_2310_05647_amd import NufftPlan
    say(f"multi-coil nufft parity N={N} L={L} Ns={Ns} coils={Nc}")
    rng = np.random.default_rng(N * 10 + Nc)
    traj = rng.uniform(-np.pi, np.pi, (L, Ns, 2)).astype(np.float32)
    S = mrfgen.coil_maps(N, Nc, seed=Nc)
    X = _rand(rng, L, N, N)
    y = _rand(rng, Nc, L, Ns)
    plan = NufftPlan(N, to_dev(traj))
    b = plan.fwd_mc(to_dev(S), to_dev(X)).cpu().numpy()
    a = plan.adj_mc(to_dev(S), to_dev(y)).cpu().numpy()
    rb = onufft.nufft_fwd_mc(X, traj, S)
    ra = onufft.nufft_adj_mc(y, traj, N, S)
    eb, ea = rel_l2(b, rb), rel_l2(a, ra)
    ec = max(rel_l2(b[c], rb[c]) for c in range(Nc))
    say(f"  fwd rel-L2 {eb:.2e} (worst coil {ec:.2e})  adj rel-L2 {ea:.2e}")
    assert eb <= TOL and ec <= TOL and ea <= TOL


def test_unit_map_is_the_single_coil_operator():
    from paper_2310_05647_amd import NufftPlan
    rng = np.random.default_rng(5)
    N, L, Ns = 64, 3, 400
    traj = rng.uniform(-np.pi, np.pi, (L, Ns, 2)).astype(np.float32)
    plan = NufftPlan(N, to_dev(traj))
    one = torch.ones((1, N, N), dtype=torch.complex64, device="cuda")
    X, y = to_dev(_rand(rng, L, N, N)), to_dev(_rand(rng, L, Ns))
    assert torch.equal(plan.fwd_mc(one, X)[0], plan.fwd(X))
    assert torch.equal(plan.adj_mc(one, y[None].contiguous()), plan.adj(y))


def test_multicoil_adjoint_identity():
    from paper_2310_05647_amd import NufftPlan
    rng = np.random.default_rng(6)
    N, L, Ns, Nc = 64, 4, 700, 6
    traj = rng.uniform(-np.pi, np.pi, (L, Ns, 2)).astype(np.float32)
    S = to_dev(mrfgen.coil_maps(N, Nc, seed=2))
    plan = NufftPlan(N, to_dev(traj))
    X, y = to_dev(_rand(rng, L, N, N)), to_dev(_rand(rng, Nc, L, Ns))
    Ax = plan.fwd_mc(S, X).cpu().numpy().astype(np.complex128)
    Ahy = plan.adj_mc(S, y).cpu().numpy().astype(np.complex128)
    lhs = np.vdot(Ax, y.cpu().numpy().astype(np.complex128))
    rhs = np.vdot(X.cpu().numpy().astype(np.complex128), Ahy)
    say(f"  <A x, y> {lhs:.6e}  <x, A^H y> {rhs:.6e}")
    assert abs(lhs - rhs) <= 1e-5 * np.linalg.norm(Ax) * np.linalg.norm(y.cpu().numpy())


def test_multicoil_operator_norm():
    from paper_2310_05647_amd import NufftPlan
    w = mc_workload()
    N = w["cfg"]["N"]
    plan = NufftPlan(N, to_dev(w["traj"]))
    S = to_dev(w["smaps"])
    lam_mc = plan.opnorm_mc(S, iters=40)
    lam_1 = plan.opnorm(iters=40)
    say(f"  lambda_max multi-coil {lam_mc:.5f} (oracle {w['lamA']:.5f}), single coil {lam_1:.5f}")
    assert abs(lam_mc - w["lamA"]) <= 1e-2 * w["lamA"]
    assert lam_mc <= lam_1 * (1 + 1e-4)


def _gpu_recon(w, n_max, graphs=None, smaps=True):
    from paper_2310_05647_amd import Dictionary, NufftPlan, Recon
    cfg = w["cfg"]
    plan = NufftPlan(cfg["N"], to_dev(w["traj"]))
    d = Dictionary(to_dev(w["atoms"]), to_dev(w["grid"]["lut"]), to_dev(w["V"]))
    rc = Recon(plan, d, cfg["p"], cfg["s"], cfg["K"], cfg["r_llr"], lam1_0=cfg["lam1_0"], lam2=cfg["lam2"],
               beta=cfg["beta"], mu0=cfg["mu0"], lamA=w["lamA"], n_max=n_max, tol=-1.0)
    if smaps:
        rc.set_coils(to_dev(w["smaps"]))
    if graphs is not None:
        st = graphs["stats"]
        for k, Lap in enumerate(st["graphs"]):
            rc.inject_graph(k, Lap, st["sigma2"][k], st["lmax"][k])
    return rc


_ORACLE = {}


def _oracle(n_max):
    if n_max not in _ORACLE:
        w = mc_workload()
        cfg = w["cfg"]
        say(f"oracle: {n_max} multi-coil iterations")
        _ORACLE[n_max] = orecon.recon(w["b"], w["traj"], w["atoms"], w["grid"]["lut"], w["V"], cfg["N"], cfg["p"],
                                      cfg["s"], cfg["K"], cfg["r_llr"], lam1_0=cfg["lam1_0"], lam2=cfg["lam2"],
                                      beta=cfg["beta"], mu0=cfg["mu0"], lamA=w["lamA"], n_max=n_max,
                                      keep_graphs=True, smaps=w["smaps"])
    return _ORACLE[n_max]


def test_multicoil_recon_follows_the_oracle_with_its_graphs():
    w = mc_workload()
    o = _oracle(6)
    say("multi-coil recon: 6 iterations on the oracle's graphs")
    rc = _gpu_recon(w, 6, graphs=o)
    out = rc.run(to_dev(w["b"]))
    torch.cuda.synchronize()
    st = out["stats"]
    cg, co = np.array(st["cost"]), np.array(o["stats"]["cost"])
    ec = np.abs(cg - co) / co
    emu = np.max(np.abs(np.array(st["mu"]) - np.array(o["stats"]["mu"])) / np.array(o["stats"]["mu"]))
    ex = rel_l2(out["X"].cpu().numpy(), o["X"])
    agree = float(np.mean(out["idx"].cpu().numpy() == o["idx"]))
    say(f"  X rel-L2 {ex:.2e}; cost rel {ec.max():.2e}; mu rel {emu:.2e}; index agreement {agree:.4f}")
    assert st["iters"] == 6 and np.all(np.diff(cg) < 0)
    assert ex <= 1e-5 and ec.max() <= 1e-5 and emu <= 1e-6
    assert agree >= 0.995


def test_multicoil_checkpoint_resume_is_bit_identical():
    from paper_2310_05647_amd._lib import MrfError
    w = mc_workload()
    b = to_dev(w["b"])
    ref = _gpu_recon(w, 6).run(b)
    a = _gpu_recon(w, 6)
    a.init(b)
    a.iterate(3)
    ck = a.checkpoint()
    c = _gpu_recon(w, 6)
    c.restore(b, ck)
    c.iterate(3)
    out = c.finish()
    assert torch.equal(out["X"], ref["X"]) and c.stats()["cost"] == ref["stats"]["cost"]
    single = _gpu_recon(w, 6, smaps=False)
    with pytest.raises(MrfError) as ei:
        single.restore(b[0].contiguous(), ck)
    assert ei.value.status == 2
