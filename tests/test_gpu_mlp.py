"""GPU learned match (MLP training and inference kernels) against the oracle's FP64 MLP.

Batch synthesis: atom indices identical (the same Philox counters), features and targets to
FP32 rounding. Gradients: FP32 mode to rel-L2 1e-5 per tensor; BF16 mode (operands of every
product rounded to BF16) within 3e-2 of the oracle run with BF16-rounded activations. One Adam
step to 1e-6. Inference + gate: the grid atom, residual and fallback decision agree with the
oracle except at decision boundaries within rounding. A short training run shows the gain over
the plain match on off-grid fingerprints.
"""
import numpy as np
import pytest
import torch

import mrfgen
from mrfgen._native import epg_fisp
from oracle import match as omatch
from oracle import mlp as omlp
from tests.gpu_util import rel_l2, say, to_dev
from tests.workloads import c1_workload

pytestmark = pytest.mark.gpu

SIZES = [20, 256, 256, 256, 2]


def _flat(params):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params]).astype(np.float32)


def _unflat(flat, sizes=SIZES):
    out, o = [], 0
    for i, j in zip(sizes[:-1], sizes[1:]):
        W = flat[o:o + i * j].reshape(j, i); o += i * j
        b = flat[o:o + j]; o += j
        out.append((W.astype(np.float64), b.astype(np.float64)))
    return out


@pytest.fixture(scope="module")
def setup():
    from paper_2310_05647_amd import MLP, Dictionary
    w = c1_workload()
    atoms, lut, V, grid = w["atoms"], w["grid"]["lut"], w["V"], w["grid"]
    d = Dictionary(to_dev(atoms), to_dev(lut), to_dev(V))
    net = MLP(n_in=2 * V.shape[1], hidden=256, layers=3, seed=5)
    net.set_grid(grid)
    D = atoms.astype(np.complex128)
    norms = np.linalg.norm(D, axis=1)
    Dr_unit = (D @ V.astype(np.complex128)) / norms[:, None]
    return dict(atoms=atoms, lut=lut, V=V, grid=grid, d=d, net=net, Dr_unit=Dr_unit, norms=norms)


def test_synth_batch_matches_oracle(setup):
    s = setup
    L = s["atoms"].shape[1]
    for step in (0, 3):
        z, t, m = [x.cpu().numpy() for x in s["net"].synth(s["d"], seed=0x1234ABCD9876, step=step, batch=777)]
        alpha, mref = omlp.synth_batch(s["Dr_unit"], 0x1234ABCD9876, step, 777, 20.0, 60.0, L)
        np.testing.assert_array_equal(m, mref)
        zref = omlp.features(alpha)
        mean, std = omlp.target_stats(s["lut"])
        tref = (np.log(np.asarray(s["lut"], np.float64)[mref, :2]) - mean) / std
        ez, et = np.abs(z - zref).max(), np.abs(t - tref).max()
        say(f"synth step {step}: max |dz| {ez:.2e}, max |dt| {et:.2e}")
        assert ez <= 1e-5 and et <= 1e-5
    st = s["net"].target_stats(s["d"])
    np.testing.assert_allclose(st, np.concatenate(omlp.target_stats(s["lut"])), rtol=1e-10)


def _batch(s, B, step):
    L = s["atoms"].shape[1]
    alpha, m = omlp.synth_batch(s["Dr_unit"], 77, step, B, 20.0, 60.0, L)
    z = omlp.features(alpha).astype(np.float32)
    mean, std = omlp.target_stats(s["lut"])
    t = ((np.log(np.asarray(s["lut"], np.float64)[m, :2]) - mean) / std).astype(np.float32)
    return z, t


@pytest.mark.parametrize("bf16,B", [(False, 300), (False, 4096), (True, 1024)])
def test_gradients_match_oracle(setup, bf16, B):
    s = setup
    params = omlp.init_params(SIZES, 3)
    flat = _flat(params)
    s["net"].set_params(to_dev(flat))
    z, t = _batch(s, B, 1)
    loss, g = s["net"].grads(to_dev(z), to_dev(t), bf16=bf16)
    p64 = _unflat(flat)
    rnd = omlp.bf16_round if bf16 else None
    lref, gref = omlp.loss_and_grads(p64, z.astype(np.float64), t.astype(np.float64), act_round=rnd)
    gg = _unflat(g.cpu().numpy())
    tol = 3e-2 if bf16 else 1e-5
    worst = 0.0
    for (dW, db), (rW, rb) in zip(gg, gref):
        worst = max(worst, rel_l2(dW, rW), rel_l2(db, rb))
    say(f"grads bf16={bf16} B={B}: loss {loss:.6f} vs {lref:.6f}, worst rel-L2 {worst:.2e}")
    assert abs(loss - lref) <= (1e-2 if bf16 else 1e-6) * lref
    assert worst <= tol


def test_bf16_gradients_with_unaligned_widths_match_oracle(setup):
    """Hidden width 30 (not a multiple of 4) and a ragged batch: the backward and weight-gradient
    products of a layer then run as two launches instead of one (their operands do not allow
    16-byte loads), and the split-K slices of every layer are still summed by the one finishing
    launch. BF16 gradients against the oracle with BF16-rounded activations, as above."""
    from paper_2310_05647_amd import MLP
    s = setup
    sizes = [20, 30, 30, 2]
    net = MLP(n_in=sizes[0], hidden=sizes[1], layers=len(sizes) - 2, seed=2)
    params = omlp.init_params(sizes, 7)
    flat = _flat(params)
    net.set_params(to_dev(flat))
    z, t = _batch(s, 1000, 2)
    loss, g = net.grads(to_dev(z), to_dev(t), bf16=True)
    lref, gref = omlp.loss_and_grads(_unflat(flat, sizes), z.astype(np.float64), t.astype(np.float64),
                                     act_round=omlp.bf16_round)
    gg = _unflat(g.cpu().numpy(), sizes)
    worst = max(max(rel_l2(dW, rW), rel_l2(db, rb)) for (dW, db), (rW, rb) in zip(gg, gref))
    say(f"grads bf16, widths {sizes}: loss {loss:.6f} vs {lref:.6f}, worst rel-L2 {worst:.2e}")
    assert abs(loss - lref) <= 1e-2 * lref
    assert worst <= 3e-2


def test_forward_and_adam_step_match_oracle(setup):
    s = setup
    params = omlp.init_params(SIZES, 4)
    flat = _flat(params)
    net = s["net"]
    net.set_params(to_dev(flat))
    net.reset_optimizer()
    z, t = _batch(s, 512, 2)
    y = net.forward(to_dev(z)).cpu().numpy()
    yref, _ = omlp.forward(_unflat(flat), z.astype(np.float64))
    assert rel_l2(y, yref) <= 1e-5
    _, g = net.grads(to_dev(z), to_dev(t))
    net.adam_step(1e-3)
    new = _unflat(net.get_params().cpu().numpy())
    ref = omlp.adam_step(_unflat(flat), _unflat(g.cpu().numpy()), {}, 1e-3)
    worst = max(max(np.abs(a - b).max() for a, b in zip(nw, rf)) for nw, rf in zip(new, ref))
    say(f"adam step: max |dp| {worst:.2e}")
    assert worst <= 1e-6


@pytest.mark.parametrize("bf16,hidden", [(True, 256), (False, 256), (True, 30)])
def test_training_run_equals_its_steps_taken_one_by_one(setup, bf16, hidden):
    """The training entry point groups its launches (the BF16 step sums the weight gradients of all
    layers, takes the Adam step and draws the next batch in one launch); its parameters and losses
    equal those of the same steps taken through the separate calls: batch synthesis, gradients,
    Adam step with the cosine rate. A ragged batch (1000) leaves partial tiles everywhere."""
    from paper_2310_05647_amd import MLP
    s = setup
    seed, first, steps, total, lr, B = 0x5EED, 5, 4, 20, 2e-3, 1000
    lr32 = float(np.float32(lr))                 # the rate as the library holds it
    a = MLP(n_in=2 * s["V"].shape[1], hidden=hidden, layers=3, seed=11)
    b = MLP(n_in=2 * s["V"].shape[1], hidden=hidden, layers=3, seed=11)
    losses = a.train(s["d"], steps, batch=B, lr=lr, first_step=first, total_steps=total, seed=seed,
                     bf16=bf16).cpu().numpy()
    ref = []
    for step in range(first, first + steps):
        z, t, _ = b.synth(s["d"], seed=seed, step=step, batch=B)
        loss, _ = b.grads(z, t, bf16=bf16)
        ref.append(loss)
        b.adam_step(float(np.float32(lr32 * 0.5 * (1.0 + np.cos(np.pi * step / total)))))
    pa, pb = a.get_params().cpu().numpy(), b.get_params().cpu().numpy()
    worst = float(np.abs(pa - pb).max())
    say(f"train vs steps ({'bf16' if bf16 else 'fp32'}, hidden {hidden}): max |dp| {worst:.2e}, "
        f"losses {losses} vs {np.array(ref)}")
    assert worst <= 1e-7 * max(1.0, float(np.abs(pb).max()))
    np.testing.assert_allclose(losses, np.array(ref, dtype=np.float32), rtol=1e-6)


def test_learned_match_and_gate_match_oracle(setup):
    s = setup
    params = omlp.init_params(SIZES, 6)
    flat = _flat(params)
    s["net"].set_params(to_dev(flat))
    rng = np.random.default_rng(2)
    m = rng.integers(0, s["atoms"].shape[0], 3000)
    x = s["atoms"][m] * np.exp(1j * rng.uniform(0, 6.28, (3000, 1))) * rng.uniform(1, 50, (3000, 1))
    x = x + 0.05 * (rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape))
    alpha = (x @ s["V"]).astype(np.complex64)
    out = s["net"].match(s["d"], to_dev(alpha), theta=0.02, bf16=False)
    g = s["grid"]
    ref = omlp.learned_match(alpha.astype(np.complex128), _unflat(flat), omlp.target_stats(s["lut"]), s["Dr_unit"],
                             s["norms"], g["t1_axis"], g["t2_axis"], g["grid_index"], 0.02)
    fb = out["fallback"].cpu().numpy().astype(bool)
    resid = out["resid"].cpu().numpy()
    idx = out["idx"].cpu().numpy()
    gated = ~fb & ~ref["fallback"]
    same_k = idx[gated] == ref["k"][gated]
    say(f"learned match: fallback {fb.sum()} (oracle {ref['fallback'].sum()}), grid atom agreement {same_k.mean():.4f}")
    assert same_k.mean() >= 0.999
    np.testing.assert_allclose(resid[gated][same_k], ref["residual"][gated][same_k], atol=2e-5)
    assert np.all((fb == ref["fallback"]) | (np.abs(ref["residual"] - 0.02) <= 2e-5))
    t12 = out["t12"].cpu().numpy()
    np.testing.assert_allclose(t12[gated, 0], ref["T1"][gated], rtol=1e-4)
    # gated-out voxels carry the exhaustive subspace match
    ridx, _, _, _ = omatch.match_subspace(x[fb], s["atoms"], s["lut"], s["V"])
    assert np.mean(idx[fb] == ridx) >= 0.999
    assert out["n_fallback"] == int(fb.sum())


def test_training_gains_over_plain_match_on_off_grid_fingerprints(setup):
    """Off-grid truth: the plain match can only return grid values; the trained network
    interpolates. The gated learned match (theta chosen here) must reach a lower T1 and T2
    NMSE than the plain exhaustive subspace match on the same noisy fingerprints."""
    s = setup
    net = s["net"]
    net.set_params(to_dev(_flat(omlp.init_params(SIZES, 9))))
    net.reset_optimizer()
    steps = 3000
    losses = net.train(s["d"], steps=steps, batch=1024, lr=1e-3, total_steps=steps, snr_lo=20.0, snr_hi=60.0,
                       seed=11, bf16=True).cpu().numpy()
    say(f"training: loss {losses[:10].mean():.4f} -> {losses[-50:].mean():.5f}")
    assert losses[-50:].mean() < 0.05 * losses[:10].mean()
    cfg = mrfgen.get_config("C1")
    rng = np.random.default_rng(21)
    n = 4096
    t1 = np.exp(rng.uniform(np.log(300.0), np.log(2500.0), n))
    t2 = np.minimum(np.exp(rng.uniform(np.log(40.0), np.log(300.0), n)), t1)
    fa, tr, te = mrfgen.fisp_sequence(cfg["L"], cfg["fa_range"], cfg["fa_period"], cfg["tr_ms"], cfg["te_ms"])
    x = epg_fisp(t1, t2, fa, tr, te, cfg["epg_states"]) * 80.0 * np.exp(1j * rng.uniform(0, 6.28, (n, 1)))
    x = x + mrfgen.complex_noise(x.shape, mrfgen.noise_sigma(np.mean(np.abs(x) ** 2), 40.0), 22)
    alpha = (x @ s["V"]).astype(np.complex64)
    idx, _, _, params = [a.cpu().numpy() for a in s["d"].match_subspace(to_dev(alpha))]

    def nmse(est, tru):
        return float(np.sum((est - tru) ** 2) / np.sum(tru ** 2))

    plain = (nmse(params[:, 0], t1), nmse(params[:, 1], t2))
    best = None
    for theta in (0.002, 0.005, 0.01, 0.02, 1.0):
        out = net.match(s["d"], to_dev(alpha), theta=theta, bf16=True)
        t12 = out["t12"].cpu().numpy()
        lm = (nmse(t12[:, 0], t1), nmse(t12[:, 1], t2))
        say(f"theta {theta}: learned NMSE T1 {lm[0]:.2e} T2 {lm[1]:.2e} (fallback {out['n_fallback']}); "
            f"plain T1 {plain[0]:.2e} T2 {plain[1]:.2e}")
        if lm[0] <= plain[0] and lm[1] <= plain[1] and best is None:
            best = theta
    assert best is not None
