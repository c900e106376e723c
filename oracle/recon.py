"""Oracle: Algorithm 1, the MS-LLR reconstruction (Sec. III-C, III-D).

TEST INFRASTRUCTURE ONLY.

  X^0 = A^H b,  M^0 = Phi_D(X^0),  L^0 from M^0,  lambda1 = lambda1^0 max(L^0)
  repeat for n = 0 .. N_max - 1:
    Z^n     = P_S(X^n - mu [A^H(A X^n - b) + lambda1 Q*(Q(X^n) L^n)])          eq. (15)
    P^{n+1} = SVT_{1/beta}(Q_q(X^n)) for every patch                            eq. (22)
    X^{n+1} = (Z^n + mu lam2 beta Q*(P^{n+1})) / (1 + mu lam2 beta c)          eq. (23)
    cost(n+1) = (1/2)||A X^{n+1} - b||^2 + lambda1 Tr(Q L^n Q^H) + lam2 sum ||Q_q X^{n+1}||_*
    stop if cost(n)/cost(n+1) - 1 < tol
    M^{n+1} = Phi_D(X^{n+1}),  L^{n+1} from M^{n+1},  lambda1 = lambda1^0 max(L^{n+1})
  output X, Phi_D(X)

Readings (beyond those of the operator modules):
  * cost(0) is evaluated on X^0 with L^0 so that the first stopping test has a
    predecessor; a tolerance of None runs exactly N_max iterations;
  * step size mu = min(mu0, 1 / (lamA + 2 c_max lambda1 max(L))): lamA bounds
    lambda_max(A^H A) and 2 c_max max(L) bounds the Laplacian term (Gershgorin), so the
    paper's mu = 1 is kept whenever it is stable; lamA <= 0 keeps mu = mu0;
  * the per-iteration match uses the subspace form with the projection basis V.
Pins: with lambda1 = lambda2 = 0 and V = I the loop is a Landweber iteration that
converges to the least-squares solution (numpy.linalg.lstsq on a tiny dense operator).
"""
import numpy as np
import scipy.sparse as sp

from . import cartesian, graph, match, nufft, ops
from . import toeplitz as toep
from .patches import coverage


def step_size(mu0, lamA, lam1, lmax, cmax):
    if lamA is None or lamA <= 0:
        return float(mu0)
    return float(min(mu0, 1.0 / (lamA + 2.0 * cmax * lam1 * lmax)))


def recon(b, traj, atoms, lut, V, N, p, s, K, r_llr, lam1_0=0.1, lam2=0.1, beta=0.2,
          mu0=1.0, lamA=0.0, sigma2=0.0, n_max=10, tol=None, osf=2, W=6, X0=None, keep_graphs=False,
          smaps=None, mask=None, toeplitz=False):
    """Return dict(X, maps, idx, rho, stats). keep_graphs: stats["graphs"] lists every Laplacian
    used (scipy CSR [Np, Np]; graph k serves iteration k + 1). The Laplacian is applied from
    sparse storage (the same entries; only the non-zeros enter the sums). smaps [Nc, N, N]: the
    acquisition is eq. (1)'s multi-coil F_u C (b [Nc, L, Ns]); None: a single coil. mask [L, N, N]:
    Cartesian sampling (oracle.cartesian; traj unused, b [L, N, N] or [Nc, L, N, N]). toeplitz:
    the data term's gradient A^H A X - A^H b and its cost value through the Toeplitz normal
    operator (oracle.toeplitz; single coil, non-Cartesian), with no forward transform in the loop."""
    b = np.asarray(b, np.complex128)
    V = np.asarray(V, np.complex128)
    tau = 1.0 / beta
    cmax = float(coverage(N, p, s).max())

    def fwd(X):
        if mask is not None:
            return cartesian.cart_fwd_mc(X, mask, smaps) if smaps is not None else cartesian.cart_fwd(X, mask)
        if smaps is not None:
            return nufft.nufft_fwd_mc(X, traj, smaps, osf, W)
        return nufft.nufft_fwd(X, traj, osf, W)

    def adj(r):
        if mask is not None:
            return cartesian.cart_adj_mc(r, mask, smaps) if smaps is not None else cartesian.cart_adj(r, mask)
        if smaps is not None:
            return nufft.nufft_adj_mc(r, traj, N, smaps, osf, W)
        return nufft.nufft_adj(r, traj, N, osf, W)

    def rebuild(X):
        idx, rho, _, _ = match.match_subspace(X, atoms, lut, V)
        maps = match.maps_from_match(idx, rho, lut, N)
        g = graph.knn_laplacian(maps, p, s, K, sigma2)
        return g

    if toeplitz:
        Khat = toep.kernel_spectrum(toep.psf_circulant(traj, N, osf, W))
        AHb = adj(b)
        bn2 = float(np.vdot(b, b).real)

    def data_state(X):   # what the data term's gradient and value need: r = A X - b, or A^H A X
        return toep.toeplitz_normal(X, Khat) if toeplitz else fwd(X) - b

    def data_grad(st):
        return st - AHb if toeplitz else adj(st)

    def cost_of(st, X, Lap, lam1, nuc):
        if not toeplitz:
            return ops.cost(st, X, Lap, lam1, lam2, nuc, p, s)
        c, (_, tr, _) = ops.cost(np.zeros(1), X, Lap, lam1, lam2, nuc, p, s)
        data = toep.data_term(X, st, AHb, bn2)
        return c + data, (data, tr, nuc)

    X = adj(b) if X0 is None else np.asarray(X0, np.complex128)
    g = rebuild(X)
    Lap, lam1 = sp.csr_matrix(g["L"]), lam1_0 * g["lmax"]
    mu = step_size(mu0, lamA, lam1, g["lmax"], cmax)
    r = data_state(X)
    nuc = ops.nuclear_norm(X, p, s)
    c_prev, terms = cost_of(r, X, Lap, lam1, nuc)
    stats = dict(cost=[c_prev], terms=[terms], mu=[mu], lam1=[lam1], sigma2=[g["sigma2"]],
                 lmax=[g["lmax"]], iters=0, stop="max_iter")
    if keep_graphs:
        stats["graphs"] = [Lap]
    for n in range(n_max):
        grad = data_grad(r) + lam1 * ops.laplacian_apply(X, Lap, p, s)
        Z = ops.project(X - mu * grad, V)
        QtP, _ = ops.llr_prox(X, p, s, tau, r_llr)
        X = ops.x_update(Z, QtP, mu, lam2, beta, p, s)
        r = data_state(X)
        nuc = ops.nuclear_norm(X, p, s)
        c, terms = cost_of(r, X, Lap, lam1, nuc)
        stats["cost"].append(c); stats["terms"].append(terms)
        stats["iters"] = n + 1
        if tol is not None and c_prev / c - 1.0 < tol:
            stats["stop"] = "tolerance"
            break
        c_prev = c
        if n + 1 < n_max:
            g = rebuild(X)
            Lap, lam1 = sp.csr_matrix(g["L"]), lam1_0 * g["lmax"]
            mu = step_size(mu0, lamA, lam1, g["lmax"], cmax)
            stats["mu"].append(mu); stats["lam1"].append(lam1)
            stats["sigma2"].append(g["sigma2"]); stats["lmax"].append(g["lmax"])
            if keep_graphs:
                stats["graphs"].append(Lap)
    idx, rho, score, params = match.match_subspace(X, atoms, lut, V)
    maps = match.maps_from_match(idx, rho, lut, N)
    return dict(X=X, maps=maps, idx=idx, rho=rho, score=score, stats=stats)
