"""Writes c2_two_iterations.npz beside this script: two iterations of the oracle's Algorithm 1 on
the full 256 x 256, L = 1000 workload (tests.workloads.c2_workload), for the GPU parity test at
that size. Everything stored comes from oracle/ (the inputs from the seeded generators):

  lamA              the oracle's bound on lambda_max(A^H A) (20 power iterations, seeded start)
  cost, mu, lam1,   Algorithm 1's statistics (cost(0..2); per graph mu, lambda1, sigma^2,
  sigma2, lmax      max(L))
  g{k}_rowptr/col/  graph k (k = 0, 1) in CSR, float64 values
  val
  idx, maps         the final match (subspace) and its T1, T2, PD maps
  xs_pos, xs_val    X after iteration 2 at 8192 seeded positions (flat index into [L][N][N])

Usage: python tests/golden/make_c2_fixture.py   (about 10 minutes and 16 GB of memory)
"""
import os
import sys
import time

import numpy as np
import scipy.sparse as sp

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import mrfgen  # noqa: E402
from oracle import nufft as onufft  # noqa: E402
from oracle import recon as orecon  # noqa: E402
from tests.workloads import c2_workload  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_two_iterations.npz")


def main():
    t0 = time.time()
    w = c2_workload()
    cfg = w["cfg"]
    print("workload %.0f s" % (time.time() - t0), flush=True)
    x0 = mrfgen.complex_noise((cfg["L"], cfg["N"], cfg["N"]), 1.0, 202)
    lamA = onufft.operator_norm(w["traj"], cfg["N"], x0, iters=20)
    print("lamA %.6f at %.0f s" % (lamA, time.time() - t0), flush=True)
    o = orecon.recon(w["b"], w["traj"], w["atoms"], w["grid"]["lut"], w["V"], cfg["N"], cfg["p"], cfg["s"],
                     cfg["K"], cfg["r_llr"], lam1_0=cfg["lam1_0"], lam2=cfg["lam2"], beta=cfg["beta"],
                     mu0=cfg["mu0"], lamA=lamA, n_max=2, keep_graphs=True)
    st = o["stats"]
    print("recon %.0f s: cost %s" % (time.time() - t0, st["cost"]), flush=True)
    rng = np.random.default_rng(2024)
    pos = np.sort(rng.choice(o["X"].size, 8192, replace=False)).astype(np.int64)
    out = dict(lamA=lamA, cost=np.array(st["cost"]), mu=np.array(st["mu"]), lam1=np.array(st["lam1"]),
               sigma2=np.array(st["sigma2"]), lmax=np.array(st["lmax"]), idx=o["idx"].astype(np.int32),
               maps=o["maps"].astype(np.float32), xs_pos=pos, xs_val=o["X"].ravel()[pos])
    for k, Lap in enumerate(st["graphs"]):
        c = sp.csr_matrix(Lap)
        out["g%d_rowptr" % k] = c.indptr.astype(np.int32)
        out["g%d_col" % k] = c.indices.astype(np.int32)
        out["g%d_val" % k] = c.data
    np.savez_compressed(OUT, **out)
    print("wrote %s (%.1f MB) in %.0f s" % (OUT, os.path.getsize(OUT) / 1e6, time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
