"""Synthetic T1/T2/PD phantoms standing in for the paper's simulated maps (Sec. IV-B).

The paper's ground-truth maps come from prior work and are not available. Two
stand-ins with the same structure (tissue inside a head outline, PD = 0 outside):
  "regions": a head ellipse split into n_regions Voronoi cells with constant
             T1 ~ logU[300, 2500] ms, T2 ~ logU[40, min(300, T1)] ms, PD ~ U[0.6, 1.0]
  "smooth":  log T1 and log T2 are sums of seeded Gaussian blobs rescaled to
             [log 300, log 2500] and [log 40, log 300] (T2 <= T1), PD smooth in [0.6, 1.0]
PD is multiplied by pd_scale (the simulated PD of the paper spans [0, 117]).
"""
import numpy as np


def _ellipse_mask(N):
    y, x = np.mgrid[0:N, 0:N].astype(np.float64)
    cy = cx = (N - 1) / 2.0
    return ((x - cx) / (0.45 * N)) ** 2 + ((y - cy) / (0.38 * N)) ** 2 <= 1.0


def _blob_field(N, n_blobs, rng):
    y, x = np.mgrid[0:N, 0:N].astype(np.float64) / N
    f = np.zeros((N, N))
    for _ in range(n_blobs):
        cy, cx = rng.uniform(0.1, 0.9, 2)
        w = rng.uniform(0.05, 0.25)
        a = rng.uniform(-1.0, 1.0)
        f += a * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2 * w * w))
    return f


def _rescale(f, mask, lo, hi):
    v = f[mask]
    return lo + (f - v.min()) / max(v.max() - v.min(), 1e-12) * (hi - lo)


def make_phantom(cfg, seed=0, N=None):
    """Return dict(T1, T2, PD, mask) as float64 [N, N] arrays (zeros outside the head)."""
    N = int(N or cfg["N"])
    rng = np.random.default_rng(seed)
    mask = _ellipse_mask(N)
    T1 = np.zeros((N, N)); T2 = np.zeros((N, N)); PD = np.zeros((N, N))
    if cfg.get("phantom", "regions") == "regions":
        nreg = int(cfg.get("n_regions", 6))
        pts = []
        while len(pts) < nreg:
            py, px = rng.uniform(0, N, 2)
            if mask[int(py), int(px)]:
                pts.append((py, px))
        pts = np.array(pts)
        y, x = np.mgrid[0:N, 0:N].astype(np.float64)
        d = (y[None] - pts[:, 0, None, None]) ** 2 + (x[None] - pts[:, 1, None, None]) ** 2
        lab = np.argmin(d, axis=0)
        for k in range(nreg):
            t1 = float(np.exp(rng.uniform(np.log(300.0), np.log(2500.0))))
            t2 = float(np.exp(rng.uniform(np.log(40.0), np.log(min(300.0, t1)))))
            pd = float(rng.uniform(0.6, 1.0))
            sel = mask & (lab == k)
            T1[sel] = t1; T2[sel] = t2; PD[sel] = pd
    else:
        nb = int(cfg.get("n_blobs", 24))
        lt1 = _rescale(_blob_field(N, nb, rng), mask, np.log(300.0), np.log(2500.0))
        lt2 = _rescale(_blob_field(N, nb, rng), mask, np.log(40.0), np.log(300.0))
        pd = _rescale(_blob_field(N, nb, rng), mask, 0.6, 1.0)
        T1[mask] = np.exp(lt1[mask])
        T2[mask] = np.minimum(np.exp(lt2[mask]), T1[mask])
        PD[mask] = pd[mask]
    PD *= float(cfg.get("pd_scale", 100.0))
    return dict(T1=T1, T2=T2, PD=PD, mask=mask)
