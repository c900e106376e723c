"""Oracle: the learned matcher (20 -> 256 -> 256 -> 256 -> 2 MLP) and its training step.

TEST INFRASTRUCTURE ONLY. The paper cites learned signal-to-parameter mapping as related
work; this form of it (architecture, inputs, training batches, gate) is the project's
own and is defined here:

  features  alpha = x V (r complex coefficients), alpha / ||alpha||, rotated so that
            alpha_0 is real and >= 0; z = (Re alpha, Im alpha) in R^{2r}
  network   h1 = relu(W1 z + b1), h2 = relu(W2 h1 + b2), h3 = relu(W3 h2 + b3),
            y = W4 h3 + b4; y is (log T1, log T2) standardised by (mean, std)
  loss      mean over the batch and the two outputs of (y - t)^2
  optimiser Adam (beta1, beta2, eps) with bias correction
  batches   sample i of step t draws (Philox4x32-10, key = seed, counter = (i, t, c, 0)):
            atom m = mulhi32(u, M), phase phi = 2 pi (u + 1/2) 2^-32, SNR ~ U[snr_lo, snr_hi] dB,
            noise n ~ CN(0, sigma^2 I_r) by Box-Muller with sigma^2 = 10^(-SNR/10) / L,
            alpha = exp(i phi) d_m V / ||d_m|| + n
  gate      k* = the kept grid atom (T2 <= T1) nearest to the prediction in Euclidean distance on
            (log T1, log T2), ties to the lower atom index;
            residual = 1 - |<d_k* V/||d_k*||, alpha/||alpha||>|;
            voxels whose residual exceeds theta fall back to the exhaustive match.
Pins: Philox against the published known-answer vectors; central finite differences
against the analytic backward; one Adam step against its closed form; the gate's grid atom
against hand-worked cases on a small grid (boundary of the kept region, unequal axis
spacings) and against per-axis rounding where the rounded grid point is kept.
"""
import numpy as np

# ---------------------------------------------------------------- Philox4x32-10
_M0, _M1 = 0xD2511F53, 0xCD9E8D57
_W0, _W1 = 0x9E3779B9, 0xBB67AE85
_MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds (Salmon et al., SC'11). ctr [..., 4], key [..., 2] uint64 -> [..., 4]."""
    c = [np.asarray(ctr[..., i], np.uint64) for i in range(4)]
    k0 = np.asarray(key[..., 0], np.uint64)
    k1 = np.asarray(key[..., 1], np.uint64)
    for rnd in range(10):
        p0 = np.uint64(_M0) * c[0]
        p1 = np.uint64(_M1) * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(_MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(_MASK)
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
        if rnd < 9:
            k0 = (k0 + np.uint64(_W0)) & np.uint64(_MASK)
            k1 = (k1 + np.uint64(_W1)) & np.uint64(_MASK)
    return np.stack(c, axis=-1)


def _u01(u):
    """uint32 -> (0, 1): (u + 1/2) 2^-32."""
    return (u.astype(np.float64) + 0.5) * 2.0 ** -32


def synth_batch(Dr_unit, seed, step, batch, snr_lo, snr_hi, L):
    """Training batch in the subspace: returns (alpha [B, r] complex, atom index [B])."""
    M, r = Dr_unit.shape
    i = np.arange(batch, dtype=np.uint64)
    key = np.stack([np.full(batch, seed & _MASK, np.uint64),
                    np.full(batch, (seed >> 32) & _MASK, np.uint64)], -1)

    def draw(c):
        ctr = np.stack([i, np.full(batch, step, np.uint64), np.full(batch, c, np.uint64),
                        np.zeros(batch, np.uint64)], -1)
        return philox4x32_10(ctr, key)

    u = draw(0)
    m = ((u[:, 0] * np.uint64(M)) >> np.uint64(32)).astype(np.int64)
    phi = 2.0 * np.pi * _u01(u[:, 1])
    snr = snr_lo + (snr_hi - snr_lo) * _u01(u[:, 2])
    sigma = np.sqrt(10.0 ** (-snr / 10.0) / L)
    gauss = []
    for c in range(1, (2 * r + 3) // 4 + 1):         # 4 uniforms -> 4 normals per call
        v = draw(c)
        for a, b in ((0, 1), (2, 3)):
            rad = np.sqrt(-2.0 * np.log(_u01(v[:, a])))
            ang = 2.0 * np.pi * _u01(v[:, b])
            gauss += [rad * np.cos(ang), rad * np.sin(ang)]
    g = np.stack(gauss[:2 * r], axis=1)              # [B, 2r]
    noise = (g[:, :r] + 1j * g[:, r:]) * (sigma / np.sqrt(2.0))[:, None]
    alpha = np.exp(1j * phi)[:, None] * np.asarray(Dr_unit, np.complex128)[m] + noise
    return alpha, m


# ---------------------------------------------------------------- features
def features(alpha):
    """alpha [B, r] complex -> z [B, 2r] (unit norm, alpha_0 real >= 0)."""
    a = np.asarray(alpha, np.complex128)
    n = np.linalg.norm(a, axis=1, keepdims=True)
    a = np.where(n > 0, a / np.where(n > 0, n, 1.0), 0.0)
    ph = np.angle(a[:, :1])
    a = a * np.exp(-1j * ph)
    return np.concatenate([a.real, a.imag], axis=1)


def bf16_round(x):
    """Round float values to bfloat16 (nearest, ties to even), returned as float64."""
    f = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    lsb = (f >> np.uint64(16)) & np.uint64(1)
    f = (f + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return f.astype(np.uint32).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------- network
def init_params(sizes, seed):
    """He-normal weights (seeded), zero biases. Returns list of (W [out, in], b [out])."""
    rng = np.random.default_rng(seed)
    params = []
    for fan_in, fan_out in zip(sizes[:-1], sizes[1:]):
        params.append((rng.standard_normal((fan_out, fan_in)) * np.sqrt(2.0 / fan_in), np.zeros(fan_out)))
    return params


def forward(params, z, act_round=None):
    """Returns (y, cache). act_round, if given, rounds the input and hidden activations
    (e.g. bf16_round) where the GPU rounds them before each product."""
    rnd = act_round or (lambda v: v)
    h = rnd(np.asarray(z, np.float64))
    cache = [h]
    for li, (W, b) in enumerate(params):
        pre = h @ W.T + b
        if li < len(params) - 1:
            h = rnd(np.maximum(pre, 0.0))
            cache.append(h)
        else:
            h = pre
    return h, cache


def loss_and_grads(params, z, t, act_round=None):
    """MSE loss and its gradients [(dW, db), ...]."""
    y, cache = forward(params, z, act_round)
    B = y.shape[0]
    diff = y - t
    loss = float(np.mean(diff * diff))
    g = 2.0 * diff / diff.size                       # dL/dy
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        h_in = cache[li]
        grads[li] = (g.T @ h_in, g.sum(axis=0))
        if li > 0:
            g = (g @ W) * (h_in > 0)
    return loss, grads


def adam_step(params, grads, state, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected). state: dict(t, m, v) (created when empty)."""
    if not state:
        state.update(t=0, m=[(np.zeros_like(W), np.zeros_like(b)) for W, b in params],
                     v=[(np.zeros_like(W), np.zeros_like(b)) for W, b in params])
    state["t"] += 1
    t = state["t"]
    new = []
    for li, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
        out = []
        for j, (w, g) in enumerate(((W, gW), (b, gb))):
            m = b1 * state["m"][li][j] + (1 - b1) * g
            v = b2 * state["v"][li][j] + (1 - b2) * g * g
            state["m"][li] = tuple(m if jj == j else state["m"][li][jj] for jj in range(2))
            state["v"][li] = tuple(v if jj == j else state["v"][li][jj] for jj in range(2))
            mh = m / (1 - b1 ** t)
            vh = v / (1 - b2 ** t)
            out.append(w - lr * mh / (np.sqrt(vh) + eps))
        new.append(tuple(out))
    return new


# ---------------------------------------------------------------- inference + gate
def target_stats(lut):
    lg = np.log(np.asarray(lut, np.float64)[:, :2])
    return lg.mean(axis=0), lg.std(axis=0)


def nearest_grid_atom(logt, t1_axis, t2_axis, grid_index, chunk=2048):
    """k* for predicted (log T1, log T2) [B, 2]: the kept grid atom (B1 index 0) at the least
    Euclidean distance in (log T1, log T2); ties go to the lower atom index."""
    logt = np.asarray(logt, np.float64)
    l1 = np.log(np.asarray(t1_axis, np.float64))
    l2 = np.log(np.asarray(t2_axis, np.float64))
    gi = np.asarray(grid_index)[:, :, 0]
    a, b = np.nonzero(gi >= 0)
    atom = gi[a, b]
    order = np.argsort(atom, kind="stable")
    a, b, atom = a[order], b[order], atom[order]
    out = np.empty(logt.shape[0], np.int64)
    for c0 in range(0, logt.shape[0], chunk):
        t = logt[c0:c0 + chunk]
        d2 = (t[:, :1] - l1[a][None, :]) ** 2 + (t[:, 1:2] - l2[b][None, :]) ** 2
        out[c0:c0 + chunk] = atom[np.argmin(d2, axis=1)]     # argmin keeps the first (lowest) index
    return out


def learned_match(alpha, params, stats, Dr_unit, atom_norms, t1_axis, t2_axis, grid_index, theta,
                  act_round=None):
    """Returns dict(T1, T2, k, residual, fallback mask, rho) for alpha [Nv, r]."""
    a = np.asarray(alpha, np.complex128)
    y, _ = forward(params, features(a), act_round)
    mean, std = stats
    logt = y * std + mean
    k = nearest_grid_atom(logt, t1_axis, t2_axis, grid_index)
    n = np.linalg.norm(a, axis=1)
    ip = np.sum(np.asarray(Dr_unit, np.complex128)[k].conj() * a, axis=1)
    resid = 1.0 - np.abs(ip) / np.where(n > 0, n, 1.0)
    rho = np.maximum(ip.real / atom_norms[k], 0.0)
    return dict(T1=np.exp(logt[:, 0]), T2=np.exp(logt[:, 1]), k=k, residual=resid,
                fallback=resid > theta, rho=rho)
