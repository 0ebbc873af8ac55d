"""Pins of the oracle's univariate B-splines (Sec. 2.1) against facts that do
not come from the oracle itself: partition of unity, the closed-form pieces
of the uniform cubic B-spline, the truncated-power formula of the cardinal
B-spline and its derivatives, and affine reproduction from Greville
abscissae."""
import math

import numpy as np
import pytest

from oracle import bspline


def cardinal_cubic(u, r=0):
    """r-th derivative of the cardinal cubic B-spline on [0, 4] by truncated
    powers: M(u) = (1/3!) sum_k (-1)^k binom(4, k) (u - k)_+^3."""
    u = np.asarray(u, dtype=np.float64)
    out = np.zeros_like(u)
    for k in range(5):
        z = np.maximum(u - k, 0.0)
        out += (-1) ** k * math.comb(4, k) * (math.factorial(3) / math.factorial(3 - r)) * z ** (3 - r)
    return out / math.factorial(3)


@pytest.mark.parametrize("N,lo,hi", [(4, 0.0, 1.0), (32, -2.0, 3.5), (7, 0.25, 0.5)])
def test_partition_of_unity(N, lo, hi):
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.uniform(lo, hi, 2000), [lo, hi], lo + (hi - lo) * np.arange(N + 1) / N])
    V = bspline.basis_dense(x, lo, hi, N, 3)
    assert np.abs(V.sum(axis=1) - 1.0).max() < 1e-14
    assert V.min() >= -1e-16


def test_closed_form_cubic_pieces():
    rng = np.random.default_rng(1)
    lo, hi, N = -1.0, 2.0, 12
    h = (hi - lo) / N
    x = rng.uniform(lo, hi, 5000)
    c, V = bspline.basis_local(x, lo, hi, N, 3)
    t = (x - lo) / h - c
    ref = np.stack([(1 - t) ** 3 / 6, (3 * t ** 3 - 6 * t ** 2 + 4) / 6,
                    (-3 * t ** 3 + 3 * t ** 2 + 3 * t + 1) / 6, t ** 3 / 6], axis=1)
    assert np.abs(V - ref).max() < 1e-14


@pytest.mark.parametrize("r", [0, 1, 2])
def test_truncated_power_formula(r):
    """B_j(x) = M((x - t_j) / h), D^r B_j = h^-r M^(r)((x - t_j)/h)."""
    rng = np.random.default_rng(2 + r)
    lo, hi, N = 0.5, 1.75, 9
    h = (hi - lo) / N
    x = rng.uniform(lo, hi, 3000)
    V = bspline.basis_dense(x, lo, hi, N, 3, r)
    t = bspline.uniform_knots(lo, hi, N, 3)
    for j in range(N + 3):
        ref = cardinal_cubic((x - t[j]) / h, r) / h ** r
        assert np.abs(V[:, j] - ref).max() < 1e-9 * max(1.0, h ** -r)


@pytest.mark.parametrize("N", [2, 5, 64])
def test_greville_affine_reproduction(N):
    rng = np.random.default_rng(3)
    lo, hi = -0.3, 1.9
    x = rng.uniform(lo, hi, 4000)
    V = bspline.basis_dense(x, lo, hi, N, 3)
    xi = bspline.greville(lo, hi, N, 3)
    h = (hi - lo) / N
    assert np.allclose(xi, lo + (np.arange(N + 3) - 1) * h, atol=1e-14)
    assert np.abs(V @ xi - x).max() < 1e-13
    assert np.abs(V @ (2.0 - 3.0 * xi) - (2.0 - 3.0 * x)).max() < 1e-13


def test_cell_convention_at_knots_and_ends():
    lo, hi, N = 0.0, 1.0, 8
    c = bspline.cell_index([0.0, 0.125, 0.5, 1.0], lo, hi, N)
    assert list(c) == [0, 1, 4, 7]
    # continuity: both sides of an interior knot give the same values
    xk = np.array([0.375])
    left = bspline.basis_dense(xk - 1e-13, lo, hi, N, 3)
    right = bspline.basis_dense(xk, lo, hi, N, 3)
    assert np.abs(left - right).max() < 1e-11
