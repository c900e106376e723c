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


def test_gate_grid_atom_hand_worked_cases():
    """Gate atom = the kept grid atom nearest in (log T1, log T2). A 3 x 3 grid with T1 axis
    100, 300, 900 ms (log step ln 3 = 1.0986) and T2 axis 50, 100, 200 ms (log step ln 2 = 0.6931);
    T2 <= T1 keeps (0,0) (0,1) | (1,0) (1,1) (1,2) | (2,0) (2,1) (2,2), atoms 0..7 in that order.
    Worked by hand, distances in log units:
      (110, 200): (0,2) is not kept; (0,1) at sqrt(ln(1.1)^2 + ln(2)^2) = 0.700 beats
                  (1,2) at ln(300/110) = 1.003                                       -> atom 1
      (164, 200): 0.45 of a T1 step above row 0: (1,2) at ln(300/164) = 0.604 beats (0,1) at
                  sqrt(ln(1.64)^2 + ln(2)^2) = 0.852 (rounding each axis and clamping T2 into
                  row 0 would give atom 1)                                           -> atom 4
      (300, 110): (1,1) at ln(1.1) = 0.095                                           -> atom 3
      (300, 30):  below the T2 axis: (1,0) at ln(50/30) = 0.511                      -> atom 2
      (100, 50), (900, 200): grid points                                             -> atoms 0, 7"""
    t1 = np.array([100.0, 300.0, 900.0])
    t2 = np.array([50.0, 100.0, 200.0])
    gi = -np.ones((3, 3, 1), np.int32)
    m = 0
    for a in range(3):
        for b in range(3):
            if t2[b] <= t1[a]:
                gi[a, b, 0] = m
                m += 1
    assert m == 8
    pts = np.log(np.array([[110, 200], [164, 200], [300, 110], [300, 30], [100, 50], [900, 200]], float))
    np.testing.assert_array_equal(mlp.nearest_grid_atom(pts, t1, t2, gi), [1, 4, 3, 2, 0, 7])


def test_gate_grid_atom_is_per_axis_rounding_inside_the_kept_region():
    """On a rectangular log grid the nearest point is the per-axis rounding; where that point is
    kept it is also the nearest kept atom (C1's 60 x 40 grid, random predictions)."""
    import mrfgen
    grid = mrfgen.param_grid(mrfgen.get_config("C1"))
    l1, l2 = np.log(grid["t1_axis"]), np.log(grid["t2_axis"])
    rng = np.random.default_rng(6)
    p = np.stack([rng.uniform(l1[0] - 0.1, l1[-1] + 0.1, 4000), rng.uniform(l2[0] - 0.1, l2[-1] + 0.1, 4000)], 1)
    i1 = np.clip(np.rint((p[:, 0] - l1[0]) / (l1[1] - l1[0])), 0, len(l1) - 1).astype(int)
    i2 = np.clip(np.rint((p[:, 1] - l2[0]) / (l2[1] - l2[0])), 0, len(l2) - 1).astype(int)
    kept = grid["grid_index"][i1, i2, 0]
    inside = kept >= 0
    assert inside.sum() > 1000 and (~inside).sum() > 100
    k = mlp.nearest_grid_atom(p, grid["t1_axis"], grid["t2_axis"], grid["grid_index"])
    np.testing.assert_array_equal(k[inside], kept[inside])
    # outside the kept region the chosen atom is kept and no kept atom is nearer
    assert np.all(k >= 0)
    T1, T2 = np.log(grid["lut"][:, 0].astype(np.float64)), np.log(grid["lut"][:, 1].astype(np.float64))
    out = np.flatnonzero(~inside)[:50]
    for v in out:
        d2 = (p[v, 0] - T1) ** 2 + (p[v, 1] - T2) ** 2
        assert d2[k[v]] <= d2.min() + 1e-9
