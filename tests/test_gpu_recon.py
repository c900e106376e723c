"""Algorithm 1 (mrf_recon) run freely, each side building its own graphs, against the oracle at C1.

Here each run builds its graphs from its own match, so arg-max near-ties (FP32 here, FP64 in the
oracle; most in background voxels with PD = 0, where every atom fits the aliasing equally badly)
change the graph, hence sigma^2, max(L), lambda1 and mu. That this, and not drift, is what
separates the runs is measured in test_gpu_recon_parity.py: with the oracle's graphs injected,
10 iterations agree to 6e-7 in X and 2e-7 in the costs. Free-running bars (iteration count fixed,
tolerance disabled): for up to two iterations the T1 and T2 maps within 0.5% rel-L2 and index
agreement >= 0.995; X within 1e-3; the costs within 1e-3 up to iteration 1 and 2e-3 at iteration
2, whose graph was built from the iteration-1 match (two rounds of flips moved it by 1.5e-3).
After 10 iterations both runs must have monotone costs and tissue T1/T2 errors against the
ground truth of comparable size.
"""
import numpy as np
import pytest
import torch

from oracle import recon as orecon
from tests.gpu_util import rel_l2, say, to_dev
from tests.workloads import c1_workload

pytestmark = pytest.mark.gpu


def _gpu_recon(w, n_max, **kw):
    from paper_2310_05647_amd import Dictionary, NufftPlan, Recon
    cfg = w["cfg"]
    plan = NufftPlan(cfg["N"], to_dev(w["traj"]))
    d = Dictionary(to_dev(w["atoms"]), to_dev(w["grid"]["lut"]), to_dev(w["V"]))
    rc = Recon(plan, d, cfg["p"], cfg["s"], cfg["K"], cfg["r_llr"], lam1_0=cfg["lam1_0"], lam2=cfg["lam2"],
               beta=cfg["beta"], mu0=cfg["mu0"], lamA=w["lamA"], n_max=n_max, tol=-1.0, **kw)
    out = rc.run(to_dev(w["b"]))
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if torch.is_tensor(v) else v) for k, v in out.items()}


def _oracle_recon(w, n_max):
    cfg = w["cfg"]
    return orecon.recon(w["b"], w["traj"], w["atoms"], w["grid"]["lut"], w["V"], cfg["N"], cfg["p"], cfg["s"],
                        cfg["K"], cfg["r_llr"], lam1_0=cfg["lam1_0"], lam2=cfg["lam2"], beta=cfg["beta"],
                        mu0=cfg["mu0"], lamA=w["lamA"], n_max=n_max)


@pytest.mark.parametrize("n_max", [0, 1, 2])
def test_c1_recon_matches_oracle(n_max):
    w = c1_workload()
    say(f"recon C1 n_max={n_max}")
    g = _gpu_recon(w, n_max)
    o = _oracle_recon(w, n_max)
    ex = rel_l2(g["X"], o["X"])
    e1 = rel_l2(g["maps"][0], o["maps"][0])
    e2 = rel_l2(g["maps"][1], o["maps"][1])
    agree = float(np.mean(g["idx"] == o["idx"]))
    say(f"  X rel-L2 {ex:.2e}  T1 {e1:.2e}  T2 {e2:.2e}  index agreement {agree:.4f}")
    say(f"  cost gpu {np.round(g['stats']['cost'], 3)}")
    say(f"  cost ora {np.round(o['stats']['cost'], 3)}")
    say(f"  lmax gpu {np.round(g['stats']['lmax'], 4)}  ora {np.round(o['stats']['lmax'], 4)}")
    say(f"  sig2 gpu {np.round(g['stats']['sigma2'], 6)}  ora {np.round(o['stats']['sigma2'], 6)}")
    say(f"  mu   gpu {np.round(g['stats']['mu'], 7)}  ora {np.round(o['stats']['mu'], 7)}")
    assert e1 <= 5e-3 and e2 <= 5e-3
    assert g["stats"]["iters"] == n_max
    assert agree >= 0.995
    # Costs up to iteration 1 within 1e-3. The iteration-2 cost comes from the graph built on the
    # iteration-1 match, and that arg-max (over the dictionary, decided in FP32 here and FP64 in the
    # oracle) flips at near-ties in background voxels; each flip moves sigma^2, max(L), lambda1 and
    # mu. Two rounds of such flips (index agreement >= 0.995) have moved it by up to 1.5e-3 while
    # A and A^H agree with the oracle to 1e-7, hence 2e-3 there; on the oracle's graphs the same
    # costs agree to 2e-7 (test_gpu_recon_parity.py).
    cg, co = np.array(g["stats"]["cost"]), np.array(o["stats"]["cost"])
    np.testing.assert_allclose(cg[:2], co[:2], rtol=1e-3)
    np.testing.assert_allclose(cg[2:], co[2:], rtol=2e-3)
    assert ex <= 1e-3


def test_c1_recon_ten_iterations_quality():
    from oracle import metrics
    w = c1_workload()
    say("recon C1 n_max=10: flip-robust comparison")
    g = _gpu_recon(w, 10)
    o = _oracle_recon(w, 10)
    ph = w["phantom"]
    m = ph["mask"]
    cg, co = np.array(g["stats"]["cost"]), np.array(o["stats"]["cost"])
    assert g["stats"]["iters"] == 10 and np.all(np.diff(cg) < 0) and np.all(np.diff(co) < 0)
    np.testing.assert_allclose(cg[:2], co[:2], rtol=1e-3)
    for c, name in ((0, "T1"), (1, "T2")):
        eg = metrics.nmse(ph[name], g["maps"][c], m)
        eo = metrics.nmse(ph[name], o["maps"][c], m)
        say(f"  {name} NMSE (tissue) gpu {eg:.4f} oracle {eo:.4f}")
        assert eg <= 1.5 * eo + 0.02
    say(f"  index agreement {np.mean(g['idx'] == o['idx']):.4f}")


def test_overlapped_schedule_equals_serial():
    """The two-stream schedule runs the same kernels on the same inputs as the serialised one:
    X, the match and every cost agree bit for bit (a race between the overlapped parts would not)."""
    w = c1_workload()
    say("recon C1 n_max=3: overlapped vs serialised schedule")
    a = _gpu_recon(w, 3, serial=3)
    b = _gpu_recon(w, 3, serial=0)
    assert np.array_equal(a["X"], b["X"])
    assert np.array_equal(a["idx"], b["idx"])
    assert a["stats"]["cost"] == b["stats"]["cost"]
