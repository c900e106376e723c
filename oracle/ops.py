"""Oracle: the per-iteration operators of the MS-LLR solve (Sec. III-B, III-C).

TEST INFRASTRUCTURE ONLY.

  laplacian_apply  S_L X = Q*(Q(X) L)                       manifold gradient, eq. (15)
  project          P_S(X) = X V V^H per voxel time course    eq. (17)
  llr_prox         per-patch SVT of Q_q(X), then Q*          eqs. (20), (22)
  x_update         (Z + mu lam2 beta Q*(P)) / (1 + mu lam2 beta c)   eqs. (21), (23)
  cost             (1/2)||AX - b||^2 + lam1 Tr(Q L Q^H) + lam2 sum ||Q_q X||_*  (Algorithm 1)

Readings:
  * SVT acts on Q_q(X^n) as eq. (22) states (not on Z^n); its threshold is 1/beta;
    at most r_llr singular values are kept (rank cap); the nuclear norm of the cost
    uses all singular values;
  * eq. (23) divides by the scalar 1 + mu lam2 beta, which is the minimiser of
    eq. (21) only when patches do not overlap; the exact minimiser divides per pixel
    by 1 + mu lam2 beta c(v) with c the patch coverage, and reduces to eq. (23) when
    p = s (pin: the gradient of eq. (21) vanishes at the output);
  * the trace term of the cost is Re<X, S_L X> = Tr(Q(X) L Q(X)^H).
"""
import numpy as np
import scipy.sparse as sp

from .patches import Q, Qadj, coverage


def laplacian_apply(X, Lap, p, s):
    """Y = Q*(Q(X) L). X [L, N, N]; Lap dense or scipy.sparse [Np, Np]."""
    X = np.asarray(X, np.complex128)
    Lf, N, _ = X.shape
    P = Q(X, p, s)                                   # [Np, p^2, L]
    Np = P.shape[0]
    flat = P.reshape(Np, -1)                         # row j = vec(patch j)
    Lt = Lap.T if sp.issparse(Lap) else np.asarray(Lap).T
    Yp = (Lt @ flat).reshape(P.shape)                # patch i = sum_j L[j, i] patch j
    return Qadj(Yp, N, p, s)


def project(U, V):
    """P_S(U) = U V V^H applied to every voxel's time course. U [L, N, N], V [L, r]."""
    U = np.asarray(U, np.complex128)
    V = np.asarray(V, np.complex128)
    Lf = U.shape[0]
    rows = U.reshape(Lf, -1).T                       # [Nv, L], one row per voxel
    out = (rows @ V) @ V.conj().T
    return out.T.reshape(U.shape)


def svt(P, tau, r_cap):
    """Singular value thresholding of one Casorati matrix (eq. (22)) via numpy's SVD.

    Returns (P', sum of all singular values)."""
    U, S, Vh = np.linalg.svd(P, full_matrices=False)
    St = np.maximum(S - tau, 0.0)
    St[r_cap:] = 0.0
    return (U * St[None, :]) @ Vh, float(S.sum())


def llr_prox(X, p, s, tau, r_cap):
    """Q*(P') with P'_i = SVT(Q_{q_i}(X)); returns (Q*(P') [L, N, N], sum_i ||Q_i X||_*)."""
    X = np.asarray(X, np.complex128)
    N = X.shape[1]
    P = Q(X, p, s)
    out = np.empty_like(P)
    nuc = 0.0
    for i in range(P.shape[0]):
        out[i], n_i = svt(P[i], tau, r_cap)
        nuc += n_i
    return Qadj(out, N, p, s), nuc


def nuclear_norm(X, p, s):
    """sum_i ||Q_{q_i}(X)||_* (eq. (13))."""
    P = Q(np.asarray(X, np.complex128), p, s)
    return float(sum(np.linalg.svd(P[i], compute_uv=False).sum() for i in range(P.shape[0])))


def x_update(Z, QtP, mu, lam2, beta, p, s):
    """Exact minimiser of eq. (21): (Z + k Q*(P)) / (1 + k c), k = mu lam2 beta."""
    k = mu * lam2 * beta
    N = Z.shape[1]
    c = coverage(N, p, s)
    return (np.asarray(Z, np.complex128) + k * np.asarray(QtP, np.complex128)) / (1.0 + k * c)[None]


def cost(resid, X, Lap, lam1, lam2, nuc, p, s):
    """Algorithm 1's cost: (1/2)||r||^2 + lam1 Re<X, S_L X> + lam2 * nuc."""
    X = np.asarray(X, np.complex128)
    data = 0.5 * float(np.vdot(resid, resid).real)
    tr = float(np.vdot(X, laplacian_apply(X, Lap, p, s)).real)
    return data + lam1 * tr + lam2 * nuc, (data, tr, nuc)
