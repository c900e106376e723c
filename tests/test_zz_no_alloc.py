"""mrf_subspace_coeffs_noalloc (partial sums in the library's static scratch array) against
mrf_subspace_coeffs (caller workspace): the same kernels, so the coefficients must agree bit for
bit, on two calls in a row (the second smaller, so it runs over what the first left in the
array), and with the oracle's X V to rel-L2 1e-5. Sizes whose partial sums exceed the array are
refused before anything is enqueued."""
import numpy as np
import pytest
import torch

from tests.gpu_util import rel_l2, say, to_dev

pytestmark = pytest.mark.gpu


def _case(rng, L, N, r):
    X = (rng.standard_normal((L, N, N)) + 1j * rng.standard_normal((L, N, N))).astype(np.complex64)
    q, _ = np.linalg.qr(rng.standard_normal((L, r)) + 1j * rng.standard_normal((L, r)))
    return X, q.astype(np.complex64)


def test_noalloc_coeffs_equal_workspace_coeffs_on_two_calls():
    from paper_2310_05647_amd import subspace_coeffs, subspace_coeffs_noalloc
    rng = np.random.default_rng(31)
    for L, N, r in ((1000, 256, 10), (100, 64, 7)):
        X, V = _case(rng, L, N, r)
        Xd, Vd = to_dev(X), to_dev(V)
        out = torch.full((N * N, r), float("nan"), dtype=torch.complex64, device=Xd.device)
        subspace_coeffs_noalloc(Xd, Vd, out)
        ref = subspace_coeffs(Xd, Vd)
        torch.cuda.synchronize()
        a, b = out.cpu().numpy(), ref.cpu().numpy()
        e = rel_l2(a, X.reshape(L, -1).T.astype(np.complex128) @ V.astype(np.complex128))
        say(f"noalloc coeffs L={L} N={N} r={r}: bitwise equal {np.array_equal(a, b)}, oracle rel-L2 {e:.2e}")
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
        assert e <= 1e-5
        del Xd, out, ref


def test_noalloc_coeffs_refuse_oversized_partial_sums():
    from paper_2310_05647_amd import subspace_coeffs_noalloc
    from paper_2310_05647_amd._lib import MrfError
    rng = np.random.default_rng(32)
    # one frame chunk x 10 x 262 144 x 8 bytes = 21 MB > 16 MiB (V need not be orthonormal here)
    X = (rng.standard_normal((1, 512, 512)) + 1j * rng.standard_normal((1, 512, 512))).astype(np.complex64)
    V = (rng.standard_normal((1, 10)) + 1j * rng.standard_normal((1, 10))).astype(np.complex64)
    out = torch.empty((512 * 512, 10), dtype=torch.complex64, device="cuda:0")
    with pytest.raises(MrfError) as ei:
        subspace_coeffs_noalloc(to_dev(X), to_dev(V), out)
    assert ei.value.status == 3   # MRF_WORKSPACE
