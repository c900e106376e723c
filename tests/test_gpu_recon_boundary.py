"""The recon's boundary beyond Algorithm 1's loop: checkpoint/resume, the final match modes and the
per-iteration wall times; the MLP's save/load.

  * checkpoint: 10 iterations in one run equal, bit for bit (X, match, every cost), 5 iterations,
    a checkpoint through host memory, a new recon restored from it and 5 more; likewise a
    checkpoint taken right after the initialisation;
  * final match: for each mode the recon's idx and maps equal what the standalone calls give on
    the same X^ (mrf_dict_match on its voxel time courses, mrf_mlp_match on X^ V);
  * MLP state: a restored network has the saved parameters, gives the same learned match, and one
    more training step from either gives the same parameters.
"""
import numpy as np
import pytest
import torch

from tests.gpu_util import say, to_dev
from tests.workloads import c1_workload

pytestmark = pytest.mark.gpu


def _objects(w):
    from paper_2310_05647_amd import Dictionary, NufftPlan
    return NufftPlan(w["cfg"]["N"], to_dev(w["traj"])), Dictionary(to_dev(w["atoms"]), to_dev(w["grid"]["lut"]),
                                                                  to_dev(w["V"]))


def _recon(w, plan, d, n_max):
    from paper_2310_05647_amd import Recon
    cfg = w["cfg"]
    return Recon(plan, d, cfg["p"], cfg["s"], cfg["K"], cfg["r_llr"], lam1_0=cfg["lam1_0"], lam2=cfg["lam2"],
                 beta=cfg["beta"], mu0=cfg["mu0"], lamA=w["lamA"], n_max=n_max, tol=-1.0)


@pytest.mark.parametrize("split", [5, 0])
def test_checkpoint_resume_is_bit_identical(split):
    w = c1_workload()
    plan, d = _objects(w)
    b = to_dev(w["b"])
    full = _recon(w, plan, d, 10)
    ref = full.run(b)
    a = _recon(w, plan, d, 10)
    a.init(b)
    a.iterate(split)
    ck = a.checkpoint()
    a.close()
    c = _recon(w, plan, d, 10)
    c.restore(b, ck)
    c.iterate(10 - split)
    out = c.finish()
    out["stats"] = c.stats()
    torch.cuda.synchronize()
    say(f"checkpoint after {split}: {ck.numel() / 1e6:.1f} MB; X equal {torch.equal(out['X'], ref['X'])}")
    assert torch.equal(out["X"], ref["X"]) and torch.equal(out["idx"], ref["idx"])
    assert out["stats"]["iters"] == 10
    assert out["stats"]["cost"] == ref["stats"]["cost"]
    assert out["stats"]["mu"] == ref["stats"]["mu"] and out["stats"]["sigma2"] == ref["stats"]["sigma2"]
    assert all(t > 0 for t in ref["stats"]["iter_ms"])


def test_checkpoint_refuses_a_recon_of_other_sizes():
    from paper_2310_05647_amd._lib import MrfError
    w = c1_workload()
    plan, d = _objects(w)
    b = to_dev(w["b"])
    a = _recon(w, plan, d, 2)
    a.init(b)
    ck = a.checkpoint()
    w2 = c1_workload(N=32, L=100)
    plan2, d2 = _objects(w2)
    c = _recon(w2, plan2, d2, 2)
    with pytest.raises(MrfError) as ei:
        c.restore(to_dev(w2["b"]), ck)
    assert ei.value.status == 2


def test_final_match_modes_equal_the_standalone_calls():
    from paper_2310_05647_amd import MLP, frames_to_voxels, subspace_coeffs
    w = c1_workload()
    plan, d = _objects(w)
    b = to_dev(w["b"])
    rc = _recon(w, plan, d, 2)
    base = rc.run(b)
    X = base["X"]
    fp = frames_to_voxels(X)
    N = w["cfg"]["N"]
    for mode in ("fp32", "bf16", "fp8"):
        rc.set_final_match(mode)
        out = rc.finish()
        idx, rho, _, prm = d.match(fp, mode=mode)[:4]
        torch.cuda.synchronize()
        say(f"final match {mode}: idx equal {torch.equal(out['idx'], idx)}; "
            f"agreement with the subspace match {float((out['idx'] == base['idx']).float().mean()):.4f}")
        assert torch.equal(out["X"], X)
        assert torch.equal(out["idx"], idx) and torch.equal(out["rho"], rho)
        assert torch.equal(out["maps"][0].reshape(-1), prm[:, 0]) and torch.equal(out["maps"][1].reshape(-1), prm[:, 1])
        assert torch.equal(out["maps"][2].reshape(-1), rho)
    net = MLP(n_in=2 * w["V"].shape[1], hidden=64, layers=2, seed=4)
    net.set_grid(w["grid"])
    net.train(d, steps=50, batch=512, lr=1e-3, total_steps=50, bf16=False)
    rc.set_final_match("learned", net, theta=0.05)
    out = rc.finish()
    ref = net.match(d, subspace_coeffs(X, to_dev(w["V"])), theta=0.05, bf16=False)
    torch.cuda.synchronize()
    say(f"final match learned: fallback {ref['n_fallback']} of {N * N}")
    assert torch.equal(out["idx"], ref["idx"]) and torch.equal(out["rho"], ref["rho"])
    assert torch.equal(out["maps"][0].reshape(-1), ref["t12"][:, 0])
    assert torch.equal(out["maps"][1].reshape(-1), ref["t12"][:, 1])
    rc.set_final_match("subspace")
    again = rc.finish()
    assert torch.equal(again["idx"], base["idx"]) and torch.equal(again["maps"], base["maps"])


def test_mlp_save_load_round_trip():
    from paper_2310_05647_amd import MLP, subspace_coeffs
    w = c1_workload()
    _, d = _objects(w)
    net = MLP(n_in=2 * w["V"].shape[1], hidden=64, layers=2, seed=7)
    net.set_grid(w["grid"])
    net.train(d, steps=30, batch=256, lr=1e-3, total_steps=60, bf16=True)
    state = net.save()
    other = MLP(n_in=2 * w["V"].shape[1], hidden=64, layers=2, seed=99)
    other.load(state)
    assert torch.equal(other.get_params(), net.get_params())
    alpha = subspace_coeffs(to_dev(w["X"].astype(np.complex64)), to_dev(w["V"]))
    m1 = net.match(d, alpha, theta=0.02)
    m2 = other.match(d, alpha, theta=0.02)
    assert torch.equal(m1["idx"], m2["idx"]) and torch.equal(m1["t12"], m2["t12"])
    # training continues identically (Adam moments and step count restored)
    net.train(d, steps=5, batch=256, lr=1e-3, total_steps=60, first_step=30, bf16=True)
    other.train(d, steps=5, batch=256, lr=1e-3, total_steps=60, first_step=30, bf16=True)
    torch.cuda.synchronize()
    say(f"mlp state {state.numel() / 1e3:.0f} kB; parameters equal after 5 more steps "
        f"{torch.equal(net.get_params(), other.get_params())}")
    assert torch.equal(net.get_params(), other.get_params())
