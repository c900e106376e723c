"""Workload configurations C1..C5.

Sizes follow the five benchmark configurations of this project (plain small, plain
paper-like scale, precision match, learned match, batched slices). Hyper-parameter
defaults follow the paper's implementation details (Sec. III-D): lambda1^0 = 0.1,
lambda2 = 0.1, beta = 1/5, mu = 1, patch stride = floor(p/2).
"""
import copy

_COMMON = dict(
    W=6,                 # Kaiser-Bessel width (grid cells)
    osf=2,               # grid oversampling: G = 2N
    fa_range=(5.0, 60.0),
    fa_period=250,       # frames per sinusoidal flip-angle lobe
    tr_ms=12.0,
    te_ms=2.0,
    epg_states=24,
    vds_alpha=1.5,
    snr_db=40.0,
    pd_scale=100.0,
    lam1_0=0.1,
    lam2=0.1,
    beta=0.2,
    mu0=1.0,
    tol=1e-5,
)

CONFIGS = {
    "C1": dict(_COMMON, name="C1", N=64, L=100, Ns=1024, n_interleaves=24,
               t1_grid=(100.0, 4000.0, 60), t2_grid=(20.0, 600.0, 40), r=10,
               p=4, s=2, K=8, r_llr=8, iters=10, phantom="regions", n_regions=6),
    "C2": dict(_COMMON, name="C2", N=256, L=1000, Ns=2048, n_interleaves=48,
               t1_grid=(100.0, 4000.0, 140), t2_grid=(20.0, 600.0, 100), r=10,
               p=8, s=4, K=16, r_llr=10, iters=30, phantom="smooth", n_blobs=24),
    "C3": dict(_COMMON, name="C3", N=256, L=1000, Ns=2048, n_interleaves=48,
               t1_grid=(100.0, 4000.0, 115), t2_grid=(20.0, 600.0, 100),
               b1_values=(0.8, 0.9, 1.0, 1.1, 1.2), r=10, phantom="smooth", n_blobs=24,
               n_fingerprints=65536),
    "C4": dict(_COMMON, name="C4", N=256, L=1000, Ns=2048, n_interleaves=48,
               t1_grid=(100.0, 4000.0, 140), t2_grid=(20.0, 600.0, 100), r=10,
               phantom="smooth", n_blobs=24, mlp_hidden=(256, 256, 256),
               train_samples=2_000_000, epochs=20, batch=4096, snr_train_db=(20.0, 60.0)),
    "C5": dict(_COMMON, name="C5",
               slices=[dict(N=128, L=500, interleaves_per_frame=2),
                       dict(N=128, L=1000, interleaves_per_frame=1),
                       dict(N=192, L=500, interleaves_per_frame=2),
                       dict(N=192, L=1000, interleaves_per_frame=1),
                       dict(N=256, L=500, interleaves_per_frame=2),
                       dict(N=256, L=1000, interleaves_per_frame=1),
                       dict(N=320, L=500, interleaves_per_frame=2),
                       dict(N=320, L=1000, interleaves_per_frame=1)],
               Ns=2048, n_interleaves=48,
               t1_grid=(100.0, 4000.0, 140), t2_grid=(20.0, 600.0, 100), r=10,
               p=8, s=4, K=16, r_llr=10, iters=30, phantom="smooth", n_blobs=24),
}


def get_config(name, **overrides):
    """Return a deep copy of configuration `name` with `overrides` applied."""
    cfg = copy.deepcopy(CONFIGS[name])
    cfg.update(overrides)
    return cfg
