"""Oracle: the FISP signal model B(eta; theta) of eqs. (2)-(3) by the extended phase graph, the
step that makes the dictionary atoms d_m (PD = 1) and off-grid training signals.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Model (the FISP train of Sec. IV: per TR one unbalanced dephasing gradient, no RF spoiling).
Magnetisation is kept as configuration states F+_k, F-_k, Z_k (k = 0 .. K-1; Weigel, J. Magn.
Reson. Imaging 2015). Start: an ideal inversion (Z_0 = -1) and one TR of recovery. Frame l:
  1. RF rotation about x by a_l = FA_l * B1 (in radians), the same 3 x 3 mixing for every k:
       F+' = cos^2(a/2) F+ + sin^2(a/2) F- - i sin(a) Z
       F-' = sin^2(a/2) F+ + cos^2(a/2) F- + i sin(a) Z
       Z'  = -(i/2) sin(a) F+ + (i/2) sin(a) F- + cos(a) Z
  2. the signal of frame l is F+_0' exp(-TE/T2);
  3. relaxation over TR_l: F *= exp(-TR/T2), Z *= exp(-TR/T1), Z_0 += 1 - exp(-TR/T1);
  4. dephasing: F+_k <- F+_{k-1}, F-_k <- F-_{k+1}, F-_{K-1} <- 0, F+_0 <- conj(F-_0).
With K >= L + 1 no state is ever dropped and the model is exact for the spin ensemble it
describes; smaller K drops the highest orders (the dictionaries use K = 24).

Pins (tests/test_oracle_epg.py): an isochromat (Bloch) simulation of the same train, the first
frame's closed form, B1 as a flip-angle scale, and the input generator's C simulator.
"""
import numpy as np


def epg_fisp(t1, t2, fa_deg, tr_ms, te_ms, n_states=24, b1=None):
    """Signals complex128 [M, L] for parameters t1, t2 (and b1) [M] (ms) and the train fa_deg,
    tr_ms [L], te_ms."""
    t1 = np.asarray(t1, np.float64)[:, None]
    t2 = np.asarray(t2, np.float64)[:, None]
    scale = np.ones_like(t1) if b1 is None else np.asarray(b1, np.float64)[:, None]
    fa = np.asarray(fa_deg, np.float64)
    tr = np.asarray(tr_ms, np.float64)
    M, L, K = t1.shape[0], fa.size, int(n_states)
    Fp = np.zeros((M, K), np.complex128)
    Fm = np.zeros((M, K), np.complex128)
    Z = np.zeros((M, K), np.complex128)
    e1 = np.exp(-tr[0] / t1[:, 0])
    Z[:, 0] = -e1 + (1.0 - e1)                       # inversion, one TR of recovery
    out = np.empty((M, L), np.complex128)
    ete = np.exp(-float(te_ms) / t2)
    for l in range(L):
        a = np.deg2rad(fa[l]) * scale                # [M, 1]
        c2, s2, sa, ca = np.cos(a / 2) ** 2, np.sin(a / 2) ** 2, np.sin(a), np.cos(a)
        Fp, Fm, Z = (c2 * Fp + s2 * Fm - 1j * sa * Z,
                     s2 * Fp + c2 * Fm + 1j * sa * Z,
                     -0.5j * sa * Fp + 0.5j * sa * Fm + ca * Z)
        out[:, l] = Fp[:, 0] * ete[:, 0]
        E1 = np.exp(-tr[l] / t1)
        E2 = np.exp(-tr[l] / t2)
        Fp, Fm, Z = Fp * E2, Fm * E2, Z * E1
        Z[:, 0] += 1.0 - E1[:, 0]
        Fp = np.concatenate([np.zeros((M, 1), np.complex128), Fp[:, :-1]], axis=1)
        Fm = np.concatenate([Fm[:, 1:], np.zeros((M, 1), np.complex128)], axis=1)
        Fp[:, 0] = np.conj(Fm[:, 0])
    return out


def isochromat_fisp(t1, t2, fa_deg, tr_ms, te_ms, n_iso, b1=1.0):
    """The same train for an ensemble of n_iso spins whose phases the per-TR gradient advances by
    2 pi j / n_iso (j = 0 .. n_iso - 1): rotations and relaxation of each spin's (Mx, My, Mz),
    the signal the ensemble mean of Mx + i My times exp(-TE/T2). One parameter set; [L]."""
    fa = np.asarray(fa_deg, np.float64)
    tr = np.asarray(tr_ms, np.float64)
    phi = 2 * np.pi * np.arange(n_iso) / n_iso
    M = np.zeros((3, n_iso))
    e1 = np.exp(-tr[0] / t1)
    M[2] = -e1 + (1.0 - e1)
    out = np.empty(fa.size, np.complex128)
    for l in range(fa.size):
        a = np.deg2rad(fa[l]) * b1
        # rotation about x by a, in the sense of the EPG mixing above (F+ = Mx + i My: Z feeds
        # F+ with -i sin(a), i.e. My' = cos(a) My - sin(a) Mz)
        Rx = np.array([[1, 0, 0], [0, np.cos(a), -np.sin(a)], [0, np.sin(a), np.cos(a)]])
        M = Rx @ M
        out[l] = np.mean(M[0] + 1j * M[1]) * np.exp(-te_ms / t2)
        E1, E2 = np.exp(-tr[l] / t1), np.exp(-tr[l] / t2)
        M[0] *= E2; M[1] *= E2; M[2] = M[2] * E1 + (1.0 - E1)
        c, s = np.cos(phi), np.sin(phi)                 # precession by the gradient's twist
        M[0], M[1] = c * M[0] - s * M[1], s * M[0] + c * M[1]
    return out


def random_params(n, seed, t1_range, t2_range, b1_range=(1.0, 1.0)):
    """Off-grid parameter sets [n, 3] = (T1, T2, B1): for set i, Philox4x32-10 (oracle.mlp) with
    counter (i, 0x45504731, 0, 0) and key (seed low, seed high) gives u1, u2, u3 in (0, 1);
    T1 = exp(log t1_lo + u1 (log t1_hi - log t1_lo)), T2 = exp(log t2_lo + u2 (log min(t2_hi, T1)
    - log t2_lo)) so that T2 <= T1, B1 = b1_lo + u3 (b1_hi - b1_lo)."""
    from .mlp import _u01, philox4x32_10
    i = np.arange(n, dtype=np.uint64)
    ctr = np.stack([i, np.full(n, 0x45504731, np.uint64), np.zeros(n, np.uint64), np.zeros(n, np.uint64)], -1)
    key = np.stack([np.full(n, seed & 0xFFFFFFFF, np.uint64), np.full(n, (seed >> 32) & 0xFFFFFFFF, np.uint64)], -1)
    u = philox4x32_10(ctr, key)
    a1, b1_ = np.log(t1_range[0]), np.log(t1_range[1])
    T1 = np.exp(a1 + _u01(u[:, 0]) * (b1_ - a1))
    a2, b2 = np.log(t2_range[0]), np.log(np.minimum(t2_range[1], T1))
    T2 = np.exp(a2 + _u01(u[:, 1]) * (b2 - a2))
    B1 = b1_range[0] + _u01(u[:, 2]) * (b1_range[1] - b1_range[0])
    return np.stack([T1, T2, B1], -1)
