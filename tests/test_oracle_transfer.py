"""Pins of the oracle's grid transfer (Sec. 2.4, eq. 2.5/2.6; Sec. 3.2.3):
subdivision exactness at random points, the Galerkin identity, and the shape
of the 1D subdivision matrix."""
import numpy as np
import pytest

from oracle import system


@pytest.mark.parametrize("d,Nc", [(1, 2), (1, 16), (2, 4), (3, 2)])
def test_subdivision_exact_at_random_points(d, Nc):
    rng = np.random.default_rng(20 + d)
    lo, hi = list(rng.uniform(-1, 0, d)), list(rng.uniform(1, 3, d))
    x = np.stack([rng.uniform(lo[p], hi[p], 500) for p in range(d)], axis=1)
    x[0] = lo
    x[1] = hi
    ac = rng.standard_normal((Nc + 3) ** d)
    sc = system.phi_matrix(x, lo, hi, Nc) @ ac
    sf = system.phi_matrix(x, lo, hi, 2 * Nc) @ (system.prolongation(d, Nc) @ ac)
    assert np.abs(sc - sf).max() < 1e-13 * max(1.0, np.abs(sc).max())


def test_prolongation_1d_shape():
    I = system.prolongation_1d(8)
    assert I.shape == (19, 11)
    # interior columns carry the mask [1, 4, 6, 4, 1] / 8 at rows 2j-3 .. 2j+1
    for j in range(2, 9):
        assert np.allclose(I[2 * j - 3:2 * j + 2, j], np.array([1, 4, 6, 4, 1]) / 8)
        assert np.count_nonzero(I[:, j]) == 5
    # rows: even i has parents (1/2, 1/2), odd i has (1/8, 3/4, 1/8)
    assert np.allclose(I[4, 2:4], [0.5, 0.5])
    assert np.allclose(I[5, 2:5], [0.125, 0.75, 0.125])


@pytest.mark.parametrize("d,N,n", [(2, 8, 800), (3, 4, 600)])
def test_galerkin_identity(d, N, n):
    rng = np.random.default_rng(30 + d)
    lo, hi = [0.0] * d, [1.0] * d
    x = rng.random((n, d))
    y = rng.standard_normal(n)
    Af, _, _, _ = system.system(x, y, lo, hi, N, 0.05)
    Ac, _, _, _ = system.system(x, y, lo, hi, N // 2, 0.05)
    P = system.prolongation(d, N // 2)
    G = (P.T @ Af @ P).toarray()
    assert np.abs(G - Ac.toarray()).max() < 1e-12 * np.abs(Ac.toarray()).max()
