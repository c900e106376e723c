"""Pins of the patch extractor Q and its adjoint."""
import numpy as np
import pytest

from oracle import patches


@pytest.mark.parametrize("N,p,s", [(16, 4, 2), (20, 6, 3), (17, 4, 2), (12, 4, 4)])
def test_adjoint_identity(N, p, s):
    rng = np.random.default_rng(N + p)
    L = 3
    X = rng.standard_normal((L, N, N)) + 1j * rng.standard_normal((L, N, N))
    Np = len(patches.patch_origins(N, p, s))
    P = rng.standard_normal((Np, p * p, L)) + 1j * rng.standard_normal((Np, p * p, L))
    lhs = np.vdot(patches.Q(X, p, s), P)
    rhs = np.vdot(X, patches.Qadj(P, N, p, s))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("N,p,s", [(16, 4, 2), (64, 4, 2), (256, 8, 4), (12, 4, 4)])
def test_coverage_closed_form(N, p, s):
    nmax = (N - p) // s          # aligned configurations
    v = np.arange(N)
    hi = np.minimum(v // s, nmax)
    lo = np.maximum(-((p - 1 - v) // s), 0)      # ceil((v - p + 1) / s)
    c1 = hi - lo + 1
    np.testing.assert_array_equal(patches.coverage(N, p, s), np.outer(c1, c1))


def test_patch_layout_raster_order():
    X = np.arange(2 * 6 * 6).reshape(2, 6, 6).astype(float)
    P = patches.Q(X, 4, 2)
    assert P.shape == (4, 16, 2)
    # patch 1 has origin (0, 2); its row 5 is pixel (1, 3)
    assert P[1, 5, 0] == X[0, 1, 3] and P[1, 5, 1] == X[1, 1, 3]
