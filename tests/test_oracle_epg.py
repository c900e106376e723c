"""Pins of the oracle's EPG FISP model (the dictionary step, eqs. (2)-(3))."""
import numpy as np

import mrfgen
from oracle import epg


def _train(L, seed=0):
    rng = np.random.default_rng(seed)
    return rng.uniform(5, 70, L), rng.uniform(10, 15, L), 2.0


def test_epg_equals_an_isochromat_ensemble():
    """Without truncation (K >= L + 1) the configuration states are the Fourier coefficients of a
    spin ensemble dephased by the gradient; with more spins than twice the highest order the
    ensemble mean is F+_0 exactly."""
    fa, tr, te = _train(12)
    for t1, t2, b1 in ((800.0, 60.0, 1.0), (1500.0, 300.0, 0.85), (300.0, 250.0, 1.15)):
        ref = epg.isochromat_fisp(t1, t2, fa, tr, te, n_iso=64, b1=b1)
        got = epg.epg_fisp([t1], [t2], fa, tr, te, n_states=13, b1=[b1])[0]
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)


def test_first_frame_closed_form():
    """Frame 0: Z_0 = 1 - 2 exp(-TR/T1) after the inversion, then F+_0 = -i sin(a) Z_0."""
    fa, tr, te = _train(3, 1)
    t1, t2 = np.array([400.0, 1200.0]), np.array([50.0, 100.0])
    s = epg.epg_fisp(t1, t2, fa, tr, te)[:, 0]
    z0 = 1 - 2 * np.exp(-tr[0] / t1)
    np.testing.assert_allclose(s, -1j * np.sin(np.deg2rad(fa[0])) * z0 * np.exp(-te / t2), rtol=1e-14)


def test_b1_scales_the_flip_angles():
    fa, tr, te = _train(40, 2)
    a = epg.epg_fisp([900.0], [80.0], fa, tr, te, b1=[1.1])
    b = epg.epg_fisp([900.0], [80.0], 1.1 * fa, tr, te)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-14)


def test_no_relaxation_keeps_the_magnetisation_bounded():
    """T1, T2 -> infinity: rotations and shifts only; the signal never exceeds 1."""
    fa, tr, te = _train(200, 3)
    s = epg.epg_fisp([1e12], [1e12], fa, tr, te, n_states=201)
    assert np.abs(s).max() <= 1 + 1e-12


def test_matches_the_input_generator():
    """The C simulator that builds the dictionaries (float32 output) is the same model."""
    cfg = mrfgen.get_config("C1")
    fa, tr, te = mrfgen.fisp_sequence(cfg["L"], cfg["fa_range"], cfg["fa_period"], cfg["tr_ms"], cfg["te_ms"])
    rng = np.random.default_rng(4)
    t1 = rng.uniform(300, 3000, 20)
    t2 = rng.uniform(20, 300, 20)
    b1 = rng.uniform(0.8, 1.2, 20)
    from mrfgen._native import epg_fisp as c_epg
    ref = c_epg(t1, t2, fa, tr, te, 24, b1=b1)
    got = epg.epg_fisp(t1, t2, fa, tr, te, 24, b1=b1)
    assert np.abs(got - ref).max() <= 2e-7 * np.abs(ref).max()


def test_random_params_ranges_and_rule():
    p = epg.random_params(20000, 7, (100.0, 4000.0), (20.0, 2000.0), (0.8, 1.2))
    T1, T2, B1 = p.T
    assert np.all((T1 >= 100) & (T1 <= 4000)) and np.all((T2 >= 20) & (T2 <= T1 * (1 + 1e-12)))
    assert np.all((B1 >= 0.8) & (B1 <= 1.2))
    # log T1 is uniform: its mean is the midpoint of the log range (to sampling error)
    assert abs(np.log(T1).mean() - 0.5 * (np.log(100) + np.log(4000))) < 0.03
    # a different seed gives different draws, the same seed the same
    assert not np.allclose(p, epg.random_params(20000, 8, (100.0, 4000.0), (20.0, 2000.0), (0.8, 1.2)))
    np.testing.assert_array_equal(p, epg.random_params(20000, 7, (100.0, 4000.0), (20.0, 2000.0), (0.8, 1.2)))
