"""Pins of the oracle's learned matcher: Philox, gradients, Adam, features, bf16 rounding."""
import numpy as np
import pytest
import torch

from oracle import mlp


@pytest.mark.parametrize("ctr,key,expect", [
    ((0, 0, 0, 0), (0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff,) * 4, (0xffffffff, 0xffffffff), (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
])
def test_philox_known_answers(ctr, key, expect):
    """Known-answer vectors published with the Random123 Philox4x32-10 generator."""
    out = mlp.philox4x32_10(np.array(ctr, np.uint64)[None], np.array(key, np.uint64)[None])[0]
    assert tuple(int(v) for v in out) == expect


def test_backward_matches_central_differences():
    rng = np.random.default_rng(1)
    params = mlp.init_params([20, 16, 16, 16, 2], seed=3)
    params = [(W, rng.standard_normal(b.shape) * 0.1) for W, b in params]
    z = rng.standard_normal((7, 20))
    t = rng.standard_normal((7, 2))
    _, grads = mlp.loss_and_grads(params, z, t)
    h = 1e-6
    for li in range(4):
        for j in range(2):
            arr = params[li][j]
            for _ in range(6):
                idx = tuple(rng.integers(0, n) for n in arr.shape)
                old = arr[idx]
                arr[idx] = old + h
                lp, _ = mlp.loss_and_grads(params, z, t)
                arr[idx] = old - h
                lm, _ = mlp.loss_and_grads(params, z, t)
                arr[idx] = old
                fd = (lp - lm) / (2 * h)
                an = grads[li][j][idx]
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)) + 1e-9


def test_first_adam_step_closed_form():
    rng = np.random.default_rng(2)
    params = [(rng.standard_normal((3, 4)), rng.standard_normal(3))]
    grads = [(rng.standard_normal((3, 4)), rng.standard_normal(3))]
    state = {}
    new = mlp.adam_step(params, grads, state, lr=1e-2)
    for (W, b), (gW, gb), (nW, nb) in zip(params, grads, new):
        np.testing.assert_allclose(nW, W - 1e-2 * gW / (np.abs(gW) + 1e-8), rtol=1e-12)
        np.testing.assert_allclose(nb, b - 1e-2 * gb / (np.abs(gb) + 1e-8), rtol=1e-12)


def test_features_are_phase_and_scale_invariant():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((5, 10)) + 1j * rng.standard_normal((5, 10))
    z = mlp.features(a)
    z2 = mlp.features(a * 3.7 * np.exp(1j * 0.9))
    np.testing.assert_allclose(z, z2, atol=1e-12)
    np.testing.assert_allclose(np.sum(z * z, axis=1), 1.0, rtol=1e-12)
    assert np.all(z[:, 0] >= 0) and np.all(np.abs(z[:, 10]) < 1e-12)


def test_bf16_rounding_matches_torch():
    x = np.random.default_rng(4).standard_normal(10000).astype(np.float32) * 100
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16_round(x), ref)


def test_synth_batch_statistics():
    rng = np.random.default_rng(5)
    M, r, L = 50, 10, 1000
    Dr = rng.standard_normal((M, r)) + 1j * rng.standard_normal((M, r))
    Dr /= np.linalg.norm(Dr, axis=1, keepdims=True)
    alpha, m = mlp.synth_batch(Dr, seed=123, step=0, batch=20000, snr_lo=30.0, snr_hi=30.0, L=L)
    assert m.min() >= 0 and m.max() < M and len(np.unique(m)) == M
    # phase-aligned residual is the noise: E|n|^2 = r sigma^2 with sigma^2 = 10^-3 / L
    proj = np.sum(Dr[m].conj() * alpha, axis=1)
    noise = alpha - (proj / np.abs(proj))[:, None] * Dr[m]
    var = np.mean(np.sum(np.abs(noise) ** 2, axis=1))
    expect = (r - 1) * 1e-3 / L + 0.0    # one of r noise dims is absorbed by the phase fit (approx.)
    assert abs(var - expect) < 0.1 * expect
    a2, m2 = mlp.synth_batch(Dr, seed=123, step=0, batch=20000, snr_lo=30.0, snr_hi=30.0, L=L)
    np.testing.assert_array_equal(alpha, a2)
