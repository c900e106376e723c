"""The EPG FISP model on the GPU (mrf_epg_fisp, mrf_epg_random_params) against the FP64 oracle.

  * signals: rel-L2 <= 1e-5 per parameter set (FP32 over up to 1000 frames) for K = 8, 16, 24
    and 32 states, with B1, on ragged counts (not a multiple of the 256-set block) and trains of
    1, 37 and 1000 frames;
  * off-grid parameters: the same Philox draws as the oracle (T1, T2, B1 within 1e-5 relative,
    FP32 exp/log against FP64), T2 <= T1 for every set;
  * the C1 dictionary made on the GPU equals the input generator's (mrfgen, FP64 C simulator,
    float32 output) to 3e-5 per atom: on this smooth, constant-TR train the 100-step recurrence
    has a larger FP32 floor — the oracle's recurrence evaluated in float32 (numpy, on the CPU)
    is off by up to 2.1e-5 for the atoms at T1 = 1667 ms — and the GPU measures 9.6e-6.
"""
import numpy as np
import pytest
import torch

import mrfgen
from oracle import epg as oepg
from tests.gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


def _train(L, seed=0):
    rng = np.random.default_rng(seed)
    return rng.uniform(5, 70, L).astype(np.float32), rng.uniform(10, 15, L).astype(np.float32), 2.0


@pytest.mark.parametrize("K,L,M", [(8, 37, 300), (16, 1, 17), (24, 1000, 513), (32, 200, 260)])
def test_epg_signals_parity(K, L, M):
    from paper_2310_05647_amd import epg_fisp
    say(f"epg K={K} L={L} M={M}")
    fa, tr, te = _train(L, K)
    p = oepg.random_params(M, 11 + K, (100.0, 4000.0), (20.0, 2000.0), (0.8, 1.2)).astype(np.float32)
    got = epg_fisp(to_dev(p[:, 0].copy()), to_dev(p[:, 1].copy()), to_dev(fa), to_dev(tr), te,
                   b1=to_dev(p[:, 2].copy()), n_states=K).cpu().numpy()
    ref = oepg.epg_fisp(p[:, 0], p[:, 1], fa, tr, te, n_states=K, b1=p[:, 2])
    err = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
    say(f"  worst per-atom rel-L2 {err.max():.2e}, median {np.median(err):.2e}")
    assert err.max() <= 1e-5


def test_random_params_match_the_oracle():
    from paper_2310_05647_amd import params_columns, random_params
    n = 5000
    p = random_params(n, 123, (100.0, 4000.0), (20.0, 2000.0), (0.8, 1.2)).cpu().numpy()
    ref = oepg.random_params(n, 123, (100.0, 4000.0), (20.0, 2000.0), (0.8, 1.2))
    e = np.abs(p - ref) / np.abs(ref)
    say(f"random params: max rel diff {e.max():.2e}")
    assert e.max() <= 1e-5
    assert np.all(p[:, 1] <= p[:, 0])
    cols = params_columns(torch.from_numpy(p).cuda()).cpu().numpy()
    np.testing.assert_array_equal(cols, p.T)


def test_gpu_dictionary_equals_the_input_generator():
    from paper_2310_05647_amd import epg_fisp
    cfg = mrfgen.get_config("C1")
    atoms, grid = mrfgen.make_dictionary(cfg)
    fa, tr, te = mrfgen.fisp_sequence(cfg["L"], cfg["fa_range"], cfg["fa_period"], cfg["tr_ms"], cfg["te_ms"])
    got = epg_fisp(to_dev(grid["T1"].astype(np.float32)), to_dev(grid["T2"].astype(np.float32)),
                   to_dev(fa.astype(np.float32)), to_dev(tr.astype(np.float32)), te,
                   n_states=cfg["epg_states"]).cpu().numpy()
    err = np.linalg.norm(got - atoms, axis=1) / np.linalg.norm(atoms, axis=1)
    say(f"C1 dictionary ({atoms.shape[0]} atoms) on the GPU: worst per-atom rel-L2 {err.max():.2e}")
    assert err.max() <= 3e-5
