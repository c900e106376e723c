"""FISP acquisition schedule theta = (FA, TR, TE) (Sec. II-B, eq. (2)).

The paper shows its flip-angle and TR patterns only in a figure that is not available;
this generator uses a sinusoidal flip-angle train between fa_range with a constant TR.
"""
import numpy as np


def fisp_sequence(L, fa_range=(5.0, 60.0), fa_period=250, tr_ms=12.0, te_ms=2.0):
    """Return (fa_deg [L], tr_ms [L], te_ms) for an L-frame FISP train."""
    lo, hi = fa_range
    l = np.arange(L, dtype=np.float64)
    fa = lo + (hi - lo) * np.sin(np.pi * l / fa_period) ** 2
    tr = np.full(L, float(tr_ms))
    return fa, tr, float(te_ms)
