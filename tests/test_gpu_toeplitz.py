"""The Toeplitz normal operator on the GPU (mrf_toeplitz_normal) against the oracle's
(oracle.toeplitz, the same gridded kernel, FP64), and Algorithm 1 run through it.

  * A^H A X: rel-L2 <= 1e-5 against the oracle's circulant form (the FP32-operator bar) at
    several sizes, and within the KB error (1e-4) of the GPU's own gridded pair adj(fwd(X));
    Hermitian: <Z, T X> = <T Z, X>;
  * Algorithm 1 in the Toeplitz mode on the oracle's graphs against the oracle's Toeplitz run: X
    within 1e-5; each data term within 1e-5 of <X, A^H A X> (it is a difference of three terms,
    0.5 <X, A^H A X> - Re <X, A^H b> + 0.5 ||b||^2, summed in FP64 from FP32 operands, so the
    FP32 error of A^H A X enters at the scale of the largest); the trace within 1e-5; the nuclear
    norm within three times its FP32-Gram floor on the oracle's X (patches the SVT has made
    rank-deficient read their vanishing singular values as sqrt(L u) sigma_1, as in the gridded
    mode);
  * checkpoint/resume in the Toeplitz mode bit for bit.
"""
import numpy as np
import pytest
import torch

import mrfgen
from oracle import recon as orecon
from oracle import toeplitz as otoep
from tests.gpu_util import nuc_fp32_gram, rel_l2, say, to_dev
from tests.workloads import c1_workload

pytestmark = pytest.mark.gpu


def _rand(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)


@pytest.mark.parametrize("N,L,Ns", [(16, 3, 97), (32, 4, 300), (64, 2, 1024), (128, 2, 517), (256, 1, 2048)])
def test_toeplitz_normal_parity(N, L, Ns):
    from paper_2310_05647_amd import NufftPlan, Toeplitz
    say(f"toeplitz N={N} L={L} Ns={Ns}")
    rng = np.random.default_rng(N + L)
    traj = rng.uniform(-np.pi, np.pi, (L, Ns, 2)).astype(np.float32)
    X, Z = _rand(rng, L, N, N), _rand(rng, L, N, N)
    T = Toeplitz(N, to_dev(traj))
    TX = T.normal(to_dev(X)).cpu().numpy()
    TZ = T.normal(to_dev(Z)).cpu().numpy()
    ref = otoep.toeplitz_normal(X, otoep.kernel_spectrum(otoep.psf_circulant(traj, N)))
    e = rel_l2(TX, ref)
    plan = NufftPlan(N, to_dev(traj))
    pair = plan.adj(plan.fwd(to_dev(X))).cpu().numpy()
    ep = rel_l2(TX, pair)
    h = abs(np.vdot(Z.astype(np.complex128), TX) - np.vdot(TZ.astype(np.complex128), X))
    say(f"  rel-L2 vs oracle {e:.2e}; vs gridded pair {ep:.2e}; Hermitian defect {h / abs(np.vdot(Z, TX)):.1e}")
    assert e <= 1e-5
    assert ep <= 1e-4
    assert h <= 1e-5 * np.linalg.norm(Z) * np.linalg.norm(TX)


def _gpu(w, n_max, graphs=None, toeplitz=True):
    from paper_2310_05647_amd import Dictionary, NufftPlan, Recon, Toeplitz
    cfg = w["cfg"]
    plan = NufftPlan(cfg["N"], to_dev(w["traj"]))
    d = Dictionary(to_dev(w["atoms"]), to_dev(w["grid"]["lut"]), to_dev(w["V"]))
    rc = Recon(plan, d, cfg["p"], cfg["s"], cfg["K"], cfg["r_llr"], lam1_0=cfg["lam1_0"], lam2=cfg["lam2"],
               beta=cfg["beta"], mu0=cfg["mu0"], lamA=w["lamA"], n_max=n_max, tol=-1.0)
    if toeplitz:
        rc.set_toeplitz(Toeplitz(cfg["N"], to_dev(w["traj"])))
    if graphs is not None:
        st = graphs["stats"]
        for k, Lap in enumerate(st["graphs"]):
            rc.inject_graph(k, Lap, st["sigma2"][k], st["lmax"][k])
    return rc


def test_toeplitz_recon_follows_the_oracle_with_its_graphs():
    w = c1_workload()
    cfg = w["cfg"]
    o = orecon.recon(w["b"], w["traj"], w["atoms"], w["grid"]["lut"], w["V"], cfg["N"], cfg["p"], cfg["s"], cfg["K"],
                     cfg["r_llr"], lam1_0=cfg["lam1_0"], lam2=cfg["lam2"], beta=cfg["beta"], mu0=cfg["mu0"],
                     lamA=w["lamA"], n_max=6, keep_graphs=True, toeplitz=True)
    say("toeplitz recon: 6 iterations on the oracle's graphs")
    rc = _gpu(w, 6, graphs=o)
    out = rc.run(to_dev(w["b"]))
    torch.cuda.synchronize()
    st = out["stats"]
    bn2 = float(np.vdot(w["b"].astype(np.complex128), w["b"].astype(np.complex128)).real)
    d_o = np.array([t[0] for t in o["stats"]["terms"]])
    tr_o = np.array([t[1] for t in o["stats"]["terms"]])
    nuc_o = np.array([t[2] for t in o["stats"]["terms"]])
    # the size of the three parts: 0.5 <X, A^H A X> ~ data + Re <X, A^H b>, bounded by 2 data + ||b||^2
    scale = 2 * d_o + bn2
    ex = rel_l2(out["X"].cpu().numpy(), o["X"])
    ed = np.max(np.abs(np.array(st["data"]) - d_o) / scale)
    etr = np.max(np.abs(np.array(st["tr"]) - tr_o) / np.abs(tr_o))
    en = abs(st["nuc"][-1] - nuc_o[-1]) / nuc_o[-1]
    floor = abs(nuc_fp32_gram(o["X"], cfg["p"], cfg["s"]) - nuc_o[-1]) / nuc_o[-1]
    say(f"  X rel-L2 {ex:.2e}; data term rel (to its parts) {ed:.2e}; trace rel {etr:.2e}; "
        f"nuclear rel {en:.2e} (FP32-Gram floor {floor:.2e})")
    assert st["iters"] == 6
    assert ex <= 1e-5
    assert ed <= 1e-5 and etr <= 1e-5
    assert en <= 3 * floor + 1e-5


def test_toeplitz_iterates_follow_the_gridded_pair():
    """The same run with the gridded pair: X within the KB error over 4 iterations."""
    w = c1_workload()
    cfg = w["cfg"]
    o = orecon.recon(w["b"], w["traj"], w["atoms"], w["grid"]["lut"], w["V"], cfg["N"], cfg["p"], cfg["s"], cfg["K"],
                     cfg["r_llr"], lam1_0=cfg["lam1_0"], lam2=cfg["lam2"], beta=cfg["beta"], mu0=cfg["mu0"],
                     lamA=w["lamA"], n_max=4, keep_graphs=True)
    a = _gpu(w, 4, graphs=o, toeplitz=True).run(to_dev(w["b"]))
    g = _gpu(w, 4, graphs=o, toeplitz=False).run(to_dev(w["b"]))
    torch.cuda.synchronize()
    e = rel_l2(a["X"].cpu().numpy(), g["X"].cpu().numpy())
    ec = np.max(np.abs(np.array(a["stats"]["cost"]) - np.array(g["stats"]["cost"])) / np.array(g["stats"]["cost"]))
    say(f"toeplitz vs gridded pair, 4 iterations: X rel-L2 {e:.2e}, cost rel {ec:.2e}")
    assert e <= 1e-4 and ec <= 1e-3


def test_toeplitz_checkpoint_resume_is_bit_identical():
    w = c1_workload()
    b = to_dev(w["b"])
    ref = _gpu(w, 6).run(b)
    a = _gpu(w, 6)
    a.init(b)
    a.iterate(3)
    ck = a.checkpoint()
    c = _gpu(w, 6)
    c.restore(b, ck)
    c.iterate(3)
    out = c.finish()
    assert torch.equal(out["X"], ref["X"]) and c.stats()["cost"] == ref["stats"]["cost"]
