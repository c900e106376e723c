"""Benchmark of the MS-LLR hot path on one MI355X.

A step is one iteration of Algorithm 1 on the paper-scale workload (256 x 256 phantom, L = 1000
FISP frames, 1 of 48 variable-density spiral interleaves per frame with 2048 samples, 12 179-atom
dictionary compressed to a rank-10 subspace, 8 x 8 patches at stride 4, K = 16, rank cap 10):
gradient step with one NUFFT pair, subspace projection, patch-graph Laplacian, per-patch SVT,
X update, cost (NUFFT residual, FP64 patch eigen-analysis, Laplacian trace), per-iteration
dictionary match and graph rebuild. Every iteration applies exactly one A and one A^H over all
L frames, so iterations/s is the NUFFT pairs/s of the solve. Inputs are synthetic and resident
in HBM before timing starts.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_MFMA_TFLOPS = 157.3
FP64_VECTOR_TFLOPS = 78.6
METRIC = "NUFFT pairs/s, fingerprints matched/s; learned vs plain at fixed T1/T2 error"


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def build_workload(seed=0):
    import mrfgen
    cfg = mrfgen.get_config("C2")
    t = time.time()
    atoms, grid = mrfgen.make_dictionary(cfg)
    V, _ = mrfgen.subspace_basis(atoms, cfg["r"])
    ph = mrfgen.make_phantom(cfg, seed)
    X = mrfgen.truth_fingerprints(cfg, ph)
    traj = mrfgen.vds_spiral(cfg["N"], cfg["L"], cfg["Ns"], cfg["n_interleaves"])
    log("workload generated in %.1f s (%d atoms)" % (time.time() - t, atoms.shape[0]))
    return cfg, atoms, grid, V, ph, X, traj


def algorithmic_work(name, cfg, E, Np):
    """(bound, amount, unit) of one launch of `name` at this workload; amounts in bytes or flops."""
    N, L, Ns = cfg["N"], cfg["L"], cfg["Ns"]
    G = 2 * N
    pp = cfg["p"] ** 2
    M, r = 12179, cfg["r"]
    img = L * N * N * 8          # one complex64 image series
    T = L * N * G * 8            # row-pass intermediate (N rows of the 2N grid per frame)
    table = {
        "nufft_row_fwd": ("hbm", img + T),
        "nufft_row_adj": ("hbm", T + img),
        "nufft_col_fwd": ("hbm", T + E * 64 + E * 8),
        "nufft_col_adj": ("hbm", E * 64 + E * 8 + T),
        # 8 x 8 patches at stride 4: the five distinct 16 x 16 cell-pair blocks of each 4 x 4 cell
        # (8 flops per complex MAC), of which every patch Gram is assembled; otherwise the Hermitian
        # half of each patch Gram
        "llr_gram": ("mfma", 8.0 * 256 * 5 * (N // 4) ** 2 * L if (cfg["p"], cfg["s"]) == (8, 4)
                     else 4.0 * pp * (pp + 1) * L * Np),
        "llr_tridiag": ("fp64", 16.0 / 3.0 * pp ** 3 * Np),          # complex Hermitian tridiagonalisation
        "match_subspace": ("mfma", 8.0 * N * N * M * r),
        "subspace_reduce": ("hbm", img),                            # one series per call (X V, then (A^H r) V)
        "subspace_expand": ("hbm", img),
        "llr_coef": ("hbm", img + Np * cfg["r_llr"] * L * 8),
        # with 8 x 8 patches at stride 4 the update forms Z = beta V^H in its tiles: it reads C
        # (and beta, V: a few MB) and writes X
        "llr_xupdate": ("hbm", img + Np * cfg["r_llr"] * L * 8 + N * N * r * 8 + L * r * 8),
        "lap_quad": ("hbm", img),
    }
    if name not in table:
        return None
    bound, amount = table[name]
    return bound, amount


def _nmse(est, tru, mask):
    e, t = est[mask], tru[mask]
    return float(np.sum((e - t) ** 2) / np.sum(t ** 2))


def _time(torch, fn, reps):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def bench_precision_match(torch, mrf, dev, fp, truth, mask, oracle_sample=256, depths=(4, 8, 16, 32)):
    """Full-length match of the 65 536 fingerprints (the reconstructed 256 x 256 series) against
    the 50 000-atom T1 x T2 x B1 dictionary in FP32, and in BF16 and FP8 with an FP32 re-rank of
    the best `depth` candidates for each depth: fingerprints/s, T1/T2 NMSE against the truth over
    the tissue, and index agreement with the oracle's FP64 exhaustive match on a sample of tissue
    voxels. For each low precision, the smallest depth whose NMSEs are within 1% of FP32's and
    whose agreement is >= 0.99 ("equal error"), and its speed against FP32's."""
    import mrfgen
    from oracle import match as omatch
    cfg3 = mrfgen.get_config("C3")
    t0 = time.perf_counter()
    atoms, grid = mrfgen.make_dictionary(cfg3)
    cpu_dict_s = time.perf_counter() - t0
    lut = grid["lut"]
    # the same 50 000-atom T1 x T2 x B1 dictionary made on the device (EPG, FP32)
    fa, tr, te = mrfgen.fisp_sequence(cfg3["L"], cfg3["fa_range"], cfg3["fa_period"], cfg3["tr_ms"], cfg3["te_ms"])
    cols = [torch.from_numpy(grid[k].astype(np.float32)).to(dev) for k in ("T1", "T2", "B1")]
    fa_d, tr_d = torch.from_numpy(fa.astype(np.float32)).to(dev), torch.from_numpy(tr.astype(np.float32)).to(dev)
    gen = lambda: mrf.epg_fisp(cols[0], cols[1], fa_d, tr_d, te, b1=cols[2], n_states=cfg3["epg_states"])
    gpu_atoms = gen()
    gpu_dict_ms = _time(torch, gen, 3)
    ga = gpu_atoms.cpu().numpy()
    dict_err = float(np.max(np.linalg.norm(ga - atoms, axis=1) / np.linalg.norm(atoms, axis=1)))
    del gpu_atoms, ga
    log("C3 dictionary (%d atoms x %d frames): CPU generator %.2f s, GPU EPG %.2f ms, worst per-atom rel diff %.1e"
        % (atoms.shape[0], atoms.shape[1], cpu_dict_s, gpu_dict_ms, dict_err))
    d = mrf.Dictionary(torch.from_numpy(atoms).to(dev), torch.from_numpy(lut).to(dev))
    Nv = fp.shape[0]
    rng = np.random.default_rng(0)
    sample = rng.choice(np.flatnonzero(mask.ravel()), oracle_sample, replace=False)
    t0 = time.time()
    ref_idx = omatch.precision_match_ref(fp[sample].cpu().numpy(), atoms, lut)[0]
    log("C3 oracle sample (%d voxels) %.1f s" % (oracle_sample, time.time() - t0))
    out = {"atoms": int(atoms.shape[0]), "fingerprints": int(Nv), "L": int(atoms.shape[1]),
           "epg_dictionary": dict(gpu_ms=round(gpu_dict_ms, 3), cpu_generator_s=round(cpu_dict_s, 3),
                                  atoms_per_s_gpu=round(atoms.shape[0] / gpu_dict_ms * 1e3, 1),
                                  worst_rel_diff_vs_cpu=dict_err),
           "fingerprints_from": "the GPU reconstruction of the 256 x 256 series after its 30 iterations"}

    def run(mode, depth):
        ms = _time(torch, lambda: d.match(fp, mode=mode, depth=depth), 1 if mode == "fp32" else 3)
        idx, rho, score, params = [t.cpu().numpy() for t in d.match(fp, mode=mode, depth=depth)]
        r = dict(depth=depth, ms=round(ms, 3), fingerprints_per_s=round(Nv / ms * 1e3, 1),
                 tflops=round(8.0 * Nv * atoms.shape[0] * atoms.shape[1] / ms / 1e9, 1),
                 nmse_t1=_nmse(params[:, 0], truth[0].ravel(), mask.ravel()),
                 nmse_t2=_nmse(params[:, 1], truth[1].ravel(), mask.ravel()),
                 agree_fp64_sample=float(np.mean(idx[sample] == ref_idx)))
        log("C3 %s depth %d: %.2f ms, %.3g fp/s, NMSE T1 %.2e T2 %.2e, agreement %.3f" % (
            mode, depth, ms, r["fingerprints_per_s"], r["nmse_t1"], r["nmse_t2"], r["agree_fp64_sample"]))
        return r

    out["fp32"] = run("fp32", 4)
    f32 = out["fp32"]
    for mode in ("bf16", "bf16x3", "fp8"):
        out[mode] = {"depth_%d" % k: run(mode, k) for k in (depths if mode != "bf16x3" else depths[:2])}
        eq = None
        for k in (depths if mode != "bf16x3" else depths[:2]):
            r = out[mode]["depth_%d" % k]
            if (r["nmse_t1"] <= 1.01 * f32["nmse_t1"] and r["nmse_t2"] <= 1.01 * f32["nmse_t2"]
                    and r["agree_fp64_sample"] >= 0.99):
                eq = dict(depth=k, ms=r["ms"], speedup_vs_fp32=round(f32["ms"] / r["ms"], 2))
                break
        out[mode]["equal_error"] = eq
        log("C3 %s equal-error point: %s" % (mode, eq))
    d.close()
    return out


def offgrid_pool(torch, mrf, dev, cfg, V, n=200_000, seed=5):
    """A training dictionary of n off-grid atoms made on the device: (T1, T2) drawn log-uniformly
    over the C2 grid's ranges with T2 <= T1 (Philox), signals by the EPG kernel on the C2 train."""
    import mrfgen
    fa, tr, te = mrfgen.fisp_sequence(cfg["L"], cfg["fa_range"], cfg["fa_period"], cfg["tr_ms"], cfg["te_ms"])
    torch.cuda.synchronize()
    t = time.perf_counter()
    params = mrf.random_params(n, seed, cfg["t1_grid"][:2], cfg["t2_grid"][:2])
    cols = mrf.params_columns(params)
    atoms = mrf.epg_fisp(cols[0].contiguous(), cols[1].contiguous(), torch.from_numpy(fa.astype(np.float32)).to(dev),
                         torch.from_numpy(tr.astype(np.float32)).to(dev), te, n_states=cfg["epg_states"])
    pool = mrf.Dictionary(atoms, params[:, :2].contiguous(), torch.from_numpy(V).to(dev))
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t
    del atoms
    log("off-grid training pool: %d EPG atoms made on the device in %.3f s" % (n, gen_s))
    return pool, gen_s


def bench_learned_match(torch, mrf, dev, d, V, Xn, truth, mask, grid, epochs=20, batch=4096, samples=2_000_000,
                        max_steps=None, train_d=None):
    """MLP trained on the device (2 M noisy atoms per epoch, SNR 20-60 dB, BF16 GEMMs), then the
    gated learned match on the 65 536 reconstructed fingerprints against the plain FP32 exhaustive
    subspace match: for a sweep of gate thresholds the T1/T2 NMSE over the tissue and how many
    voxels (and tissue voxels) fall back; the largest threshold at which both learned NMSEs are
    <= the plain ones, and fingerprints/s of both there (each includes the projection
    alpha = x V)."""
    net = mrf.MLP(n_in=2 * V.shape[1], hidden=256, layers=3, seed=1)
    net.set_grid(grid)
    steps_per_epoch = (samples + batch - 1) // batch
    steps = epochs * steps_per_epoch if max_steps is None else max_steps
    torch.cuda.synchronize()
    t0 = time.time()
    losses = net.train(train_d if train_d is not None else d, steps=steps, batch=batch, lr=1e-3, total_steps=steps,
                       seed=2, bf16=True)
    torch.cuda.synchronize()
    train_s = time.time() - t0
    lo = losses.cpu().numpy()
    log("MLP training: %d steps in %.2f s, loss %.4f -> %.6f" % (steps, train_s, lo[:20].mean(), lo[-100:].mean()))
    Vd = torch.from_numpy(V).to(dev)
    Nv = Xn[0].numel()
    alpha = mrf.subspace_coeffs(Xn, Vd)
    plain = d.match_subspace(alpha)
    pp = plain[3].cpu().numpy()
    m = mask.ravel()
    t1, t2 = truth[0].ravel(), truth[1].ravel()
    plain_err = (_nmse(pp[:, 0], t1, m), _nmse(pp[:, 1], t2, m))
    choice = None
    sweep = {}
    for theta in (1.0, 0.01, 1e-3, 3e-4, 1e-4, 5e-5, 2e-5, 1e-5, 0.0):
        r = net.match(d, alpha, theta=theta, bf16=True)
        t12 = r["t12"].cpu().numpy()
        fb = r["fallback"].cpu().numpy().astype(bool)
        err = (_nmse(t12[:, 0], t1, m), _nmse(t12[:, 1], t2, m))
        sweep[str(theta)] = dict(nmse_t1=err[0], nmse_t2=err[1], fallback=int(r["n_fallback"]),
                                 tissue_fallback=int(np.sum(fb & m)))
        if choice is None and err[0] <= plain_err[0] and err[1] <= plain_err[1]:
            choice = theta
    theta = choice if choice is not None else 0.0
    ms_plain = _time(torch, lambda: d.match_subspace(mrf.subspace_coeffs(Xn, Vd)), 5)
    ms_proj = _time(torch, lambda: mrf.subspace_coeffs(Xn, Vd), 5)
    ms_learn = _time(torch, lambda: net.match(d, mrf.subspace_coeffs(Xn, Vd), theta=theta, bf16=True), 5)
    out = dict(train_steps=steps, train_s=round(train_s, 3),
               train_ms_per_epoch=round(1e3 * train_s * steps_per_epoch / steps, 2),
               final_loss=float(lo[-100:].mean()), plain_nmse_t1=plain_err[0], plain_nmse_t2=plain_err[1],
               theta=theta, sweep=sweep, projection_ms=round(ms_proj, 4),
               plain_ms=round(ms_plain, 4), learned_ms=round(ms_learn, 4),
               plain_fingerprints_per_s=round(Nv / ms_plain * 1e3, 1),
               learned_fingerprints_per_s=round(Nv / ms_learn * 1e3, 1))
    log("learned at theta %s: %.3f ms vs plain %.3f ms; NMSE sweep %s" % (theta, ms_learn, ms_plain, sweep))
    net.close()
    return out


def bench_multicoil(torch, mrf, dev, plan, d, cfg, Xtrue, ncoils=8, iters=3):
    """Multi-coil acquisition (eq. (1), A = F_u C) on the 256 x 256, L = 1000 series with ncoils
    smooth synthetic sensitivities: the F_u C / (F_u C)^H pair, and Algorithm 1's iteration with
    the residual over every coil (iters iterations after one warm-up)."""
    import mrfgen
    S = torch.from_numpy(mrfgen.coil_maps(cfg["N"], ncoils, seed=0)).to(dev)
    X = torch.from_numpy(Xtrue).to(dev)
    kb = plan.fwd_mc(S, X)
    img = torch.empty_like(X)
    pair_ms = _time(torch, lambda: (plan.fwd_mc(S, X, kb), plan.adj_mc(S, kb, img)), 5)
    bh = kb.cpu().numpy()
    b = torch.from_numpy(bh + mrfgen.complex_noise(bh.shape, mrfgen.noise_sigma(np.mean(np.abs(bh) ** 2),
                                                                                   cfg["snr_db"]), 23)).to(dev)
    del kb, img, X
    lam = plan.opnorm_mc(S, 20)
    rc = mrf.Recon(plan, d, cfg["p"], cfg["s"], cfg["K"], cfg["r_llr"], lam1_0=cfg["lam1_0"], lam2=cfg["lam2"],
                   beta=cfg["beta"], mu0=cfg["mu0"], lamA=lam, n_max=100000, tol=-1.0)
    rc.set_coils(S)
    rc.init(b)
    rc.iterate(1)
    it_ms = _time(torch, lambda: rc.iterate(1), iters)
    st = rc.stats()
    rc.close()
    log("multi-coil (%d coils): pair %.3f ms, iteration %.3f ms" % (ncoils, pair_ms, it_ms))
    return dict(coils=ncoils, pair_ms=round(pair_ms, 4), pair_ms_per_coil=round(pair_ms / ncoils, 4),
                coil_frame_pairs_per_s=round(1e3 * ncoils * cfg["L"] / pair_ms, 1), lamA=round(lam, 4),
                iteration_ms=round(it_ms, 4), iterations_per_s=round(1e3 / it_ms, 3),
                cost_decreasing=bool(np.all(np.diff(st["cost"]) < 0)))


def bench_toeplitz(torch, mrf, dev, plan, d, cfg, traj_dev, b, lamA, iters=5):
    """Toeplitz normal operator (NEXT-2) at 256 x 256, L = 1000: set-up time, one A^H A against the
    gridded pair A^H A, Algorithm 1's iteration with the gradient and data term through it, and X
    after `iters` iterations against the gridded run's (the two differ by the KB error)."""
    N = cfg["N"]
    torch.cuda.synchronize()
    t = time.perf_counter()
    T = mrf.Toeplitz(N, traj_dev)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t
    X = plan.adj(b)
    Y = torch.empty_like(X)
    op_ms = _time(torch, lambda: T.normal(X, Y), 10)
    kb = plan.fwd(X)
    pair_ms = _time(torch, lambda: (plan.fwd(X, kb), plan.adj(kb, Y)), 10)
    del kb, Y
    out = {}
    for name, use in (("toeplitz", True), ("gridded", False)):
        rc = mrf.Recon(plan, d, cfg["p"], cfg["s"], cfg["K"], cfg["r_llr"], lam1_0=cfg["lam1_0"], lam2=cfg["lam2"],
                       beta=cfg["beta"], mu0=cfg["mu0"], lamA=lamA, n_max=100000, tol=-1.0)
        if use:
            rc.set_toeplitz(T)
        rc.init(b)
        torch.cuda.synchronize()
        t = time.perf_counter()
        rc.iterate(iters)
        torch.cuda.synchronize()
        out[name] = ((time.perf_counter() - t) * 1e3 / iters, rc.finish()["X"])
        rc.close()
    dx = float(torch.linalg.vector_norm(out["toeplitz"][1] - out["gridded"][1]) /
               torch.linalg.vector_norm(out["gridded"][1]))
    T.close()
    log("Toeplitz: set-up %.2f s, A^H A %.3f ms (gridded pair %.3f ms), iteration %.3f ms (gridded %.3f ms), "
        "X after %d iterations rel %.2e" % (setup_s, op_ms, pair_ms, out["toeplitz"][0], out["gridded"][0], iters, dx))
    return dict(setup_s=round(setup_s, 3), normal_op_ms=round(op_ms, 4), gridded_pair_ms=round(pair_ms, 4),
                iteration_ms=round(out["toeplitz"][0], 4), gridded_iteration_ms=round(out["gridded"][0], 4),
                x_rel_diff_vs_gridded=dx, iterations=iters)


def bench_radial(torch, mrf, dev, iters=50, n_spokes=13, lam1_0s=(0.1, 0.01, 0.001, 0.0)):
    """Pseudo-radial Cartesian sampling (the paper's third pattern; about 5% of k-space per frame
    with 13 golden-angle-rotated spokes at 256 x 256) at L = 500, the length of its sampling-pattern
    comparison and parameter sweep: MS-LLR for a sweep of lambda1^0 (0.1 is the paper's choice; 0
    is the LLR-only ablation), each run for `iters` iterations (the paper's N_max) from
    X^0 = A^H b; tissue NMSE of T1, T2 and PD against the phantom, the step size, and the time
    per iteration."""
    import mrfgen
    cfg = mrfgen.get_config("C2", L=500)
    atoms, grid = mrfgen.make_dictionary(cfg)
    V, _ = mrfgen.subspace_basis(atoms, cfg["r"])
    ph = mrfgen.make_phantom(cfg, 0)
    X = torch.from_numpy(mrfgen.truth_fingerprints(cfg, ph)).to(dev)
    N, L = cfg["N"], cfg["L"]
    mask = torch.from_numpy(mrfgen.radial_cartesian_mask(N, L, n_spokes)).to(dev)
    plan = mrf.CartPlan(mask)
    bh = plan.fwd(X).cpu().numpy()
    mh = mask.cpu().numpy().reshape(L, N * N).astype(bool)
    sig2 = mrfgen.noise_sigma(np.mean(np.abs(bh[mh]) ** 2), cfg["snr_db"])
    b = torch.from_numpy((bh + mh * mrfgen.complex_noise(bh.shape, sig2, 29)).astype(np.complex64)).to(dev)
    del X
    d = mrf.Dictionary(torch.from_numpy(atoms).to(dev), torch.from_numpy(grid["lut"]).to(dev),
                       torch.from_numpy(V).to(dev))
    tm = ph["mask"] & (ph["PD"] > 0)
    out = dict(N=N, L=L, spokes=n_spokes, sampled_fraction=round(float(mh.mean()), 4), iterations=iters)
    for lam1_0 in lam1_0s:
        name = "llr_only" if lam1_0 == 0.0 else "ms_llr_lam1_0_%g" % lam1_0
        rc = mrf.Recon(plan, d, cfg["p"], cfg["s"], cfg["K"], cfg["r_llr"], lam1_0=lam1_0, lam2=cfg["lam2"],
                       beta=cfg["beta"], mu0=cfg["mu0"], lamA=1.0, n_max=iters, tol=-1.0)
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = rc.run(b)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3 / iters
        maps = r["maps"].cpu().numpy()
        st = r["stats"]
        out[name] = dict(ms_per_iteration=round(ms, 3), mu_last=st["mu"][-1], cost_last=st["cost"][-1],
                         nmse_t1=_nmse(maps[0].ravel(), ph["T1"].ravel(), tm.ravel()),
                         nmse_t2=_nmse(maps[1].ravel(), ph["T2"].ravel(), tm.ravel()),
                         nmse_pd=_nmse(maps[2].ravel(), ph["PD"].ravel(), tm.ravel()))
        rc.close()
        log("radial Cartesian %s: %.3f ms/iteration, tissue NMSE T1 %.3e T2 %.3e PD %.3e" % (
            name, ms, out[name]["nmse_t1"], out[name]["nmse_t2"], out[name]["nmse_pd"]))
    d.close()
    plan.close()
    return out


def bench_batched(torch, mrf, dev, rounds=3):
    """Eight uneven slices (N = 128, 192, 256, 320, each with L = 500 at 2 spiral interleaves per
    frame and L = 1000 at 1), every slice's NUFFT strip width chosen by the autotuner; one round =
    one iteration of every slice. Timed back to back on one stream and batched on 8 streams."""
    import mrfgen
    c5 = mrfgen.get_config("C5")
    dicts = {}
    slices = []
    t0 = time.time()
    for k, sl in enumerate(c5["slices"]):
        N, L, ipf = sl["N"], sl["L"], sl["interleaves_per_frame"]
        cfg = mrfgen.get_config("C5", N=N, L=L)
        if L not in dicts:
            atoms, grid = mrfgen.make_dictionary(cfg)
            V, _ = mrfgen.subspace_basis(atoms, cfg["r"])
            dicts[L] = (mrf.Dictionary(torch.from_numpy(atoms).to(dev), torch.from_numpy(grid["lut"]).to(dev),
                                       torch.from_numpy(V).to(dev)), V)
        ph = mrfgen.make_phantom(cfg, 100 + k)
        X = torch.from_numpy(mrfgen.truth_fingerprints(cfg, ph)).to(dev)
        traj = torch.from_numpy(mrfgen.vds_spiral(N, L, c5["Ns"], c5["n_interleaves"], interleaves_per_frame=ipf)).to(dev)
        tx, times = mrf.autotune(N, traj, reps=2)
        plan = mrf.NufftPlan(N, traj, tile_cols=tx)
        b = plan.fwd(X)
        bh = b.cpu().numpy()
        b = torch.from_numpy(bh + mrfgen.complex_noise(bh.shape, mrfgen.noise_sigma(np.mean(np.abs(bh) ** 2), 40.0),
                                                       200 + k)).to(dev)
        lamA = plan.opnorm(30)
        rc = mrf.Recon(plan, dicts[L][0], cfg["p"], cfg["s"], cfg["K"], cfg["r_llr"], lam1_0=cfg["lam1_0"],
                       lam2=cfg["lam2"], beta=cfg["beta"], mu0=cfg["mu0"], lamA=lamA, n_max=100000, tol=-1.0)
        rc.init(b)
        slices.append(dict(N=N, L=L, Ns=int(traj.shape[1]), tile_cols=tx, autotune_ms={str(a): round(v, 3) for a, v in times.items()},
                           rc=rc, plan=plan, b=b))
        del X
    torch.cuda.synchronize()
    log("C5: 8 slices set up in %.1f s" % (time.time() - t0))
    recons = [x["rc"] for x in slices]
    for rc in recons:
        rc.iterate(1)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(rounds):
        for rc in recons:
            rc.iterate(1)
    torch.cuda.synchronize()
    seq_ms = (time.perf_counter() - t) * 1e3 / rounds
    streams = [torch.cuda.Stream() for _ in recons]
    mrf.recon_batched(recons, streams, 1)
    torch.cuda.synchronize()
    t = time.perf_counter()
    mrf.recon_batched(recons, streams, rounds)
    torch.cuda.synchronize()
    bat_ms = (time.perf_counter() - t) * 1e3 / rounds
    frames = sum(x["L"] for x in slices)
    log("C5: round (one iteration of all 8 slices) %.2f ms back to back, %.2f ms batched" % (seq_ms, bat_ms))
    out = dict(slices=[{k: v for k, v in x.items() if k not in ("rc", "plan", "b")} for x in slices],
               round_ms_sequential=round(seq_ms, 3), round_ms_batched=round(bat_ms, 3),
               frame_pairs_per_s_batched=round(frames / bat_ms * 1e3, 1),
               frame_pairs_per_s_sequential=round(frames / seq_ms * 1e3, 1))
    for x in slices:
        x["rc"].close()
    return out


def cpu_baseline(cfg, frames=32):
    """The oracle's Algorithm 1 iteration (FP64, the host's numpy) at 256 x 256, on a bounded
    sample: the steps whose work grows with L (gradient with one NUFFT pair, projection, per-patch
    SVT and X update, residual, nuclear norm, cost) are timed on the first `frames` frames and
    scaled by L / frames; the graph rebuild (subspace match of the 65 536 voxels and the K-NN
    patch graph), whose work does not depend on L, is timed once at full size. Each step is the
    oracle's own function, called in Algorithm 1's order."""
    import mrfgen
    import scipy.sparse as sp
    from oracle import graph as ograph
    from oracle import match as omatch
    from oracle import nufft as onufft
    from oracle import ops as oops
    from oracle.recon import step_size
    from oracle.patches import coverage
    c = mrfgen.get_config("C2", L=frames)
    atoms, grid = mrfgen.make_dictionary(c)
    V, _ = mrfgen.subspace_basis(atoms, c["r"])
    V = V.astype(np.complex128)
    X = mrfgen.truth_fingerprints(c, mrfgen.make_phantom(c, 0))
    traj = mrfgen.vds_spiral(c["N"], frames, c["Ns"], c["n_interleaves"])
    N, p, s = c["N"], c["p"], c["s"]
    b = onufft.nufft_fwd(X, traj)
    X = onufft.nufft_adj(b, traj, N)
    t = {}
    t0 = time.perf_counter()
    idx, rho, _, _ = omatch.match_subspace(X, atoms, grid["lut"], V)
    g = ograph.knn_laplacian(omatch.maps_from_match(idx, rho, grid["lut"], N), p, s, c["K"], 0.0)
    t["rebuild"] = time.perf_counter() - t0
    Lap = sp.csr_matrix(g["L"])
    lam1 = c["lam1_0"] * g["lmax"]
    mu = step_size(c["mu0"], 65.0, lam1, g["lmax"], float(coverage(N, p, s).max()))
    r = onufft.nufft_fwd(X, traj) - b
    t0 = time.perf_counter()
    grad = onufft.nufft_adj(r, traj, N) + lam1 * oops.laplacian_apply(X, Lap, p, s)
    Z = oops.project(X - mu * grad, V)
    QtP, _ = oops.llr_prox(X, p, s, 1.0 / c["beta"], c["r_llr"])
    X = oops.x_update(Z, QtP, mu, c["lam2"], c["beta"], p, s)
    r = onufft.nufft_fwd(X, traj) - b
    nuc = oops.nuclear_norm(X, p, s)
    oops.cost(r, X, Lap, lam1, c["lam2"], nuc, p, s)
    t["body"] = time.perf_counter() - t0
    per_iter = t["body"] * cfg["L"] / frames + t["rebuild"]
    try:   # the BLAS pool numpy's products and decompositions ran on; the rest is single-threaded
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info() if d.get("user_api") == "blas"] or [1])
    except ImportError:
        threads = 1
    return dict(value=round(1.0 / per_iter, 6), unit="NUFFT pairs/s", cores=threads, kind="oracle",
                seconds_per_iteration=round(per_iter, 2),
                sample="oracle (FP64 numpy) Algorithm 1 iteration at 256x256: the L-proportional steps "
                       "(NUFFT pair, Laplacian, projection, per-patch SVT, X update, residual, nuclear norm, cost) "
                       "on %d of the %d frames, %.1f s, scaled to %d frames; the L-independent graph rebuild "
                       "(subspace match of 65536 voxels, K-NN patch graph) at full size, %.1f s; numpy's BLAS "
                       "on %d host threads" % (frames, cfg["L"], t["body"], cfg["L"], t["rebuild"], threads))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-match-forms", action="store_true", help="skip the precision and learned match components")
    ap.add_argument("--mlp-epochs", type=int, default=20)
    ap.add_argument("--mlp-steps", type=int, default=None,
                    help="train the MLP for this many steps instead (short profiled runs); its quality then drops")
    ap.add_argument("--no-batched", action="store_true", help="skip the 8-slice batched component")
    ap.add_argument("--no-multicoil", action="store_true", help="skip the 8-coil component")
    ap.add_argument("--no-radial", action="store_true", help="skip the pseudo-radial Cartesian component")
    ap.add_argument("--no-toeplitz", action="store_true", help="skip the Toeplitz normal-operator component")
    ap.add_argument("--serial", type=int, default=0,
                    help="recon schedule mask: bit 0 runs the cost terms, bit 1 the rest of an iteration on one "
                         "stream (default 0: independent parts overlap on the recon's two extra streams)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (frames would shard "
              "across GPUs). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2310_05647_amd as mrf

    dev = torch.device("cuda:0")
    cfg, atoms, grid, V, ph, Xtrue, traj = build_workload()
    N, L, Ns = cfg["N"], cfg["L"], cfg["Ns"]
    traj_dev = torch.from_numpy(traj).to(dev)
    plan = mrf.NufftPlan(N, traj_dev)
    lamA = plan.opnorm(30)
    log("lambda_max(A^H A) = %.3f" % lamA)
    d = mrf.Dictionary(torch.from_numpy(atoms).to(dev), torch.from_numpy(grid["lut"]).to(dev),
                       torch.from_numpy(V).to(dev))
    import mrfgen
    b = plan.fwd(torch.from_numpy(Xtrue).to(dev))
    bh = b.cpu().numpy()
    sig2 = mrfgen.noise_sigma(np.mean(np.abs(bh) ** 2), cfg["snr_db"])
    b = torch.from_numpy(bh + mrfgen.complex_noise(bh.shape, sig2, 17)).to(dev)
    rc = mrf.Recon(plan, d, cfg["p"], cfg["s"], cfg["K"], cfg["r_llr"], lam1_0=cfg["lam1_0"], lam2=cfg["lam2"],
                   beta=cfg["beta"], mu0=cfg["mu0"], lamA=lamA, n_max=100000, tol=-1.0, serial=args.serial)
    t = time.time()
    rc.init(b)
    torch.cuda.synchronize()
    log("init (X0 = A^H b, match, graph, cost) %.2f s" % (time.time() - t))
    for i in range(args.warmup):
        rc.iterate(1)
    torch.cuda.synchronize()
    log("warmup done")

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for i in range(args.steps):
        rc.iterate(1)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    log("timed %d iterations: %.3f ms / iteration" % (args.steps, ms))

    # per-kernel times over two more iterations (HIP events on the launch stream), run with the
    # iteration serialised so that no other kernel shares the device with the one being timed
    rc.set_serial(3)
    mrf.timing_enable(True)
    nrep = 2
    for i in range(nrep):
        rc.iterate(1)
    rep = mrf.timing_report()
    mrf.timing_enable(False)
    rc.set_serial(args.serial)
    per_kernel = {k: dict(launches_per_step=v[0] / nrep, ms_per_step=v[1] / nrep, avg_ms=v[1] / v[0])
                  for k, v in rep.items()}

    # Algorithm 1 to its configured 30 iterations: the reconstruction X^ whose maps are reported
    # and whose time courses are the fingerprints of the match forms
    n_done = rc.stats()["iters"]
    rc.iterate(max(0, cfg["iters"] - n_done))
    fin = rc.finish()
    st_all = rc.stats()
    Xhat = fin["X"]
    truth = np.stack([ph["T1"], ph["T2"]])
    tmask = ph["mask"] & (ph["PD"] > 0)
    rmaps = fin["maps"].cpu().numpy()
    recon_quality = dict(iterations=st_all["iters"], nmse_t1=_nmse(rmaps[0].ravel(), truth[0].ravel(), tmask.ravel()),
                         nmse_t2=_nmse(rmaps[1].ravel(), truth[1].ravel(), tmask.ravel()),
                         cost_first=st_all["cost"][0], cost_last=st_all["cost"][-1])
    log("recon after %d iterations: tissue NMSE T1 %.3e T2 %.3e" % (st_all["iters"], recon_quality["nmse_t1"],
                                                                   recon_quality["nmse_t2"]))

    # pure NUFFT pair and plain subspace match throughput
    X = Xhat.clone()
    kb = plan.fwd(X)
    for _ in range(2):
        plan.fwd(X, kb); plan.adj(kb, X)
    e0.record()
    for _ in range(10):
        plan.fwd(X, kb); plan.adj(kb, X)
    e1.record()
    torch.cuda.synchronize()
    pair_ms = e0.elapsed_time(e1) / 10
    alpha = mrf.subspace_coeffs(X, torch.from_numpy(V).to(dev))
    d.match_subspace(alpha)
    e0.record()
    for _ in range(5):
        d.match_subspace(alpha)
    e1.record()
    torch.cuda.synchronize()
    match_ms = e0.elapsed_time(e1) / 5
    del X, kb
    # a plain streaming kernel of known size (256 MiB read, 256 MiB written): the reference that
    # scales the FETCH_SIZE / WRITE_SIZE counters of a profiled run of this same command
    cal = torch.zeros(1 << 26, dtype=torch.float32, device=dev)
    cal_out = torch.empty_like(cal)
    torch.neg(cal, out=cal_out)
    torch.cuda.synchronize()
    del cal, cal_out

    # roofline of the kernels that take the most time per step
    inf = _plan_entries(plan)
    Np = ((N - cfg["p"]) // cfg["s"] + 1) ** 2
    # the Laplacian trace runs as two launches (in-window cell pairs, then the far pairs) that
    # share one algorithmic read of X: priced together under lap_quad
    if "lap_quad_far" in per_kernel and "lap_quad" in per_kernel:
        a, f = per_kernel["lap_quad"], per_kernel.pop("lap_quad_far")
        a["ms_per_step"] += f["ms_per_step"]
        a["avg_ms"] += f["avg_ms"]
    rows = []
    for name in sorted(per_kernel, key=lambda k: -per_kernel[k]["ms_per_step"]):
        w = algorithmic_work(name, cfg, inf, Np)
        if w is None:
            continue
        rows.append(_roof_row(name, w, per_kernel[name]["avg_ms"]))
    dom = max(per_kernel.items(), key=lambda kv: kv[1]["ms_per_step"])[0]
    roof = dict(rows[0]) if rows else None
    if roof is not None:
        roof["dominant_kernel"] = dom
        roof["traffic"] = _counter_traffic(roof["kernel"])

    # match forms on the reconstruction X^ (voxel-major time courses for the full-length match)
    comps_extra = {"recon_30_iterations": recon_quality}
    if not args.no_match_forms:
        import mrfgen
        fpv = mrf.frames_to_voxels(Xhat)
        comps_extra["precision_match"] = bench_precision_match(torch, mrf, dev, fpv, truth, tmask)
        del fpv
        grid_c2 = mrfgen.param_grid(cfg)
        comps_extra["learned_match"] = bench_learned_match(torch, mrf, dev, d, V, Xhat, truth, tmask, grid_c2,
                                                          epochs=args.mlp_epochs, max_steps=args.mlp_steps)
        # the same network trained on off-grid atoms made on the device (EPG), matched against
        # the same grid dictionary
        pool, pool_s = offgrid_pool(torch, mrf, dev, cfg, V)
        comps_extra["learned_match_offgrid"] = bench_learned_match(
            torch, mrf, dev, d, V, Xhat, truth, tmask, grid_c2, epochs=args.mlp_epochs, max_steps=args.mlp_steps,
            train_d=pool)
        comps_extra["learned_match_offgrid"]["pool"] = dict(atoms=pool.M, generation_s=round(pool_s, 3))
        pool.close()
    if not args.no_batched:
        rc.close()
        comps_extra["batched_c5"] = bench_batched(torch, mrf, dev)
    if not args.no_multicoil:
        comps_extra["multicoil"] = bench_multicoil(torch, mrf, dev, plan, d, cfg, Xtrue)
    if not args.no_toeplitz:
        comps_extra["toeplitz"] = bench_toeplitz(torch, mrf, dev, plan, d, cfg, traj_dev, b, lamA)
    if not args.no_radial:
        comps_extra["radial_cartesian"] = bench_radial(torch, mrf, dev)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(cfg)

    out = {
        "metric": METRIC,
        "value": round(1000.0 / ms, 3),
        "unit": "NUFFT pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": "MS-LLR iteration, 256x256 phantom, L=1000 FISP frames, VDS spiral 1/48 "
                               "(2048 samples/frame), 12179-atom dictionary rank-10 subspace, 8x8 patches "
                               "stride 4, K=16, rank cap 10",
                   "N": N, "L": L, "Ns": Ns, "atoms": int(atoms.shape[0]), "r": cfg["r"], "p": cfg["p"],
                   "s": cfg["s"], "K": cfg["K"], "rank_cap": cfg["r_llr"], "lamA": round(lamA, 4)},
        "roofline": roof,
        "cpu_baseline": cpu,
        "components": {
            "nufft_pair_ms": round(pair_ms, 4),
            "nufft_pairs_per_s": round(1000.0 / pair_ms, 2),
            "nufft_frame_pairs_per_s": round(1000.0 * L / pair_ms, 1),
            "match_subspace_fp32_ms": round(match_ms, 4),
            "fingerprints_matched_per_s_subspace_fp32": round(N * N / (match_ms * 1e-3), 1),
            "per_kernel_schedule": "serialised iterations after the timed region",
            "per_kernel_ms_per_step": {k: round(v["ms_per_step"], 4) for k, v in
                                       sorted(per_kernel.items(), key=lambda kv: -kv[1]["ms_per_step"])},
            "roofline_by_kernel": {r["kernel"]: {"bound": r["bound"], "frac": r["frac"], "achieved": r["achieved"],
                                                 "unit": r["unit"]} for r in rows},
            **comps_extra,
        },
    }
    print(json.dumps(out), flush=True)


def _roof_row(name, work, avg_ms):
    bound, amount = work
    avg_s = avg_ms * 1e-3
    if bound == "hbm":
        ach, peak, unit = amount / avg_s / 1e9, HBM_PEAK_GBS, "GB/s"
    elif bound == "fp64":
        ach, peak, unit = amount / avg_s / 1e12, FP64_VECTOR_TFLOPS, "TFLOP/s"
    else:
        ach, peak, unit = amount / avg_s / 1e12, FP32_MFMA_TFLOPS, "TFLOP/s"
    return dict(kernel=name, bound="alu" if bound == "fp64" else bound, achieved=round(ach, 2), peak=peak, unit=unit,
                frac=round(ach / peak, 4), traffic=None, algorithmic_per_launch=amount, avg_launch_ms=round(avg_ms, 4))


def _counter_traffic(kernel):
    """HBM bytes per launch from the committed counter summary of this kernel, or None when there is
    none or the kernel's source file has changed since the counters were taken."""
    from paper_2310_05647_amd import profiling
    return profiling.traffic_bytes(os.path.join(ROOT, "profiles"), kernel)


def _plan_entries(plan):
    # number of (sample, tile) entries of the plan: 4 bytes x (L*ntiles+1) tile pointers
    import ctypes
    from paper_2310_05647_amd._lib import lib
    sz = ctypes.c_size_t()
    lib.mrf_nufft_workspace_size(plan.handle, ctypes.byref(sz))
    N, L = plan.n, plan.L
    T = L * N * 2 * N * 8
    T = (T + 255) & ~255
    return (sz.value - T) // 8


if __name__ == "__main__":
    main()
