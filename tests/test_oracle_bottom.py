"""The recurrence by which the library assembles the V-cycle's lower levels
as one dense operator, checked against the oracle's V-cycle (Alg. 7) run on
every unit vector: from B_c = A_c^-1,
  M1  = sum_{j < nu1} (I - W A_g)^j W,
  X   = M1 + I_g B_{g-1} I_g' (I - A_g M1),
  B_g = X + W (I - A_g X)   (nu2 times),
with W = omega_g D_g^-1, gives the map b -> alpha of one V-cycle from zero
on level g. Dense matrices on tiny grids; no GPU."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import mg


def _dense(A):
    return A.toarray() if sp.issparse(A) else np.asarray(A)


def _case(d, n, N, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, (n, d))
    y = np.sin(2 * np.pi * x.sum(axis=1)) + 0.1 * rng.standard_normal(n)
    return x, y, [0.0] * d, [1.0] * d, N


@pytest.mark.parametrize("d,n,N", [(1, 300, 32), (2, 2000, 16)])
@pytest.mark.parametrize("nu", [(1, 1), (2, 2), (2, 1), (0, 1), (1, 0), (3, 3)])
def test_recurrence_is_the_vcycle(d, n, N, nu):
    x, y, lo, hi, N = _case(d, n, N, 80 + d)
    M = mg.MG(x, y, lo, hi, N, 1e-3, nu1=nu[0], nu2=nu[1])
    B = np.linalg.inv(_dense(M.levels[M.c]["A"]))
    for g in range(M.c + 1, M.G + 1):
        A = _dense(M.levels[g]["A"])
        K = A.shape[0]
        W = M.omega[g] * M.Dinv[g]
        P = _dense(M.levels[g]["P"])
        M1 = np.zeros((K, K))
        if nu[0] >= 1:
            M1 = np.diag(W)
            for _ in range(1, nu[0]):
                M1 = M1 + W[:, None] * (np.eye(K) - A @ M1)
        X = M1 + P @ (B @ (P.T @ (np.eye(K) - A @ M1)))
        for _ in range(nu[1]):
            X = X + W[:, None] * (np.eye(K) - A @ X)
        B = X
        ref = np.stack([M.vcycle(e, g) for e in np.eye(K)], axis=1)
        assert np.abs(B - ref).max() <= 1e-10 * np.abs(ref).max(), (g, nu)
        if nu[0] == nu[1]:   # symmetric smoothing: B_g symmetric
            assert np.abs(B - B.T).max() <= 1e-10 * np.abs(B).max()
