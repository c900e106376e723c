"""Dictionary D and look-up table LUT (eq. (3), Sec. II-B).

Atoms d_m = B(eta_m; theta) with PD = 1, simulated by EPG on a log-spaced (T1, T2)
grid, optionally times a B1 axis. Combinations with T1 < T2 are omitted, as the
paper's discretization does (Sec. IV-A).
"""
import numpy as np

from ._native import epg_fisp
from .sequence import fisp_sequence


def _logspace(lo, hi, n):
    return np.logspace(np.log10(lo), np.log10(hi), int(n))


def param_grid(cfg):
    """Return dict(T1, T2, B1, lut, grid_index, t1_axis, t2_axis, b1_axis).

    lut is [M, nparam] float32 with columns (T1, T2) or (T1, T2, B1).
    grid_index[i1, i2, ib] is the atom index of grid point (i1, i2, ib) or -1 when the
    combination is omitted (T1 < T2). Atom order: B1 outermost, then T1, then T2.
    """
    t1_axis = _logspace(*cfg["t1_grid"])
    t2_axis = _logspace(*cfg["t2_grid"])
    b1_axis = np.asarray(cfg.get("b1_values", (1.0,)), np.float64)
    has_b1 = "b1_values" in cfg
    T1, T2, B1 = [], [], []
    grid_index = -np.ones((t1_axis.size, t2_axis.size, b1_axis.size), np.int32)
    m = 0
    for ib, b1 in enumerate(b1_axis):
        for i1, t1 in enumerate(t1_axis):
            for i2, t2 in enumerate(t2_axis):
                if t2 <= t1:
                    T1.append(t1); T2.append(t2); B1.append(b1)
                    grid_index[i1, i2, ib] = m
                    m += 1
    T1, T2, B1 = np.array(T1), np.array(T2), np.array(B1)
    cols = [T1, T2, B1] if has_b1 else [T1, T2]
    lut = np.stack(cols, axis=1).astype(np.float32)
    return dict(T1=T1, T2=T2, B1=B1, lut=lut, grid_index=grid_index,
                t1_axis=t1_axis, t2_axis=t2_axis, b1_axis=b1_axis, has_b1=has_b1)


def make_dictionary(cfg):
    """Return (atoms complex64 [M, L] with PD = 1, grid dict from param_grid)."""
    grid = param_grid(cfg)
    fa, tr, te = fisp_sequence(cfg["L"], cfg["fa_range"], cfg["fa_period"], cfg["tr_ms"], cfg["te_ms"])
    atoms = epg_fisp(grid["T1"], grid["T2"], fa, tr, te, cfg["epg_states"],
                     b1=grid["B1"] if grid["has_b1"] else None)
    return atoms, grid
