"""Pins of the oracle's solves (eq. 2.4, Alg. 7, Alg. 8): exact reproduction
of data from the penalty's null space, the two limits in lambda, dense brute
force normal equations, MGCG against the direct solve, the V-cycle's
symmetry and special cases, and the Lanczos damping estimate."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import bspline, mg, system


@pytest.mark.parametrize("lam", [1e-6, 1.0, 1e3])
def test_affine_data_reproduced_exactly(lam):
    rng = np.random.default_rng(40)
    d, N, n = 2, 8, 600
    lo, hi = [0.0, -1.0], [1.0, 2.0]
    x = np.stack([rng.uniform(lo[p], hi[p], n) for p in range(d)], axis=1)
    a0, bv = 0.7, np.array([-1.3, 2.1])
    y = a0 + x @ bv
    A, b, _, _ = system.system(x, y, lo, hi, N, lam)
    alpha = mg.solve_direct(A, b)
    J = N + 3
    ref = a0 * np.ones(J * J)
    for p in range(d):
        xi = bspline.greville(lo[p], hi[p], N, 3)
        ref += bv[p] * np.kron(xi if p == 0 else np.ones(J), xi if p == 1 else np.ones(J))
    assert np.abs(alpha - ref).max() < 1e-9 * np.abs(ref).max()


def test_lambda_to_infinity_gives_affine_least_squares():
    """The fit tends to the least-squares hyperplane as O(1/lambda) (Sec. 2.2)."""
    rng = np.random.default_rng(41)
    d, N, n = 2, 8, 2000
    x = rng.random((n, d))
    y = np.sin(3 * x[:, 0]) + x[:, 1] ** 2 + 0.1 * rng.standard_normal(n)
    X = np.column_stack([np.ones(n), x])
    ref = X @ np.linalg.lstsq(X, y, rcond=None)[0]
    errs = []
    for lam in (1e3, 1e5, 1e7):
        A, b, Phi, _ = system.system(x, y, [0, 0], [1, 1], N, lam)
        errs.append(np.abs(Phi @ mg.solve_direct(A, b) - ref).max())
    assert errs[2] < 1e-5
    assert errs[1] < errs[0] / 50 and errs[2] < errs[1] / 50


def test_lambda_to_zero_gives_least_squares_spline():
    rng = np.random.default_rng(42)
    d, N, n = 2, 4, 5000
    x = rng.random((n, d))
    y = np.cos(2 * x.sum(axis=1)) + 0.1 * rng.standard_normal(n)
    A, b, Phi, _ = system.system(x, y, [0, 0], [1, 1], N, 1e-12)
    alpha = mg.solve_direct(A, b)
    ref = np.linalg.lstsq(Phi.toarray(), y, rcond=None)[0]
    assert np.linalg.norm(alpha - ref) < 1e-6 * np.linalg.norm(ref)


def test_dense_brute_force_normal_equations():
    rng = np.random.default_rng(43)
    for d, N, n in [(1, 6, 40), (2, 2, 60), (3, 2, 200)]:
        x = rng.random((n, d))
        y = rng.standard_normal(n)
        A, b, Phi, Lam = system.system(x, y, [0.0] * d, [1.0] * d, N, 0.1)
        Pd = Phi.toarray()
        ref = np.linalg.solve(Pd.T @ Pd + 0.1 * Lam.toarray(), Pd.T @ y)
        assert np.abs(mg.solve_direct(A, b) - ref).max() < 1e-10 * np.abs(ref).max()


@pytest.fixture(scope="module")
def small_mg():
    rng = np.random.default_rng(44)
    n, d, N = 3000, 2, 16
    x = rng.random((n, d))
    y = np.sin(2 * np.pi * x[:, 0]) * np.cos(2 * np.pi * x[:, 1]) + 0.1 * rng.standard_normal(n)
    return mg.MG(x, y, [0, 0], [1, 1], N, 1e-3)


def test_mgcg_converges_to_direct_solution(small_mg):
    lev = small_mg.levels[small_mg.G]
    A, b = lev["A"], lev["b"]
    ref = mg.solve_direct(A, b)
    alpha, it, hist = mg.pcg(A, b, small_mg.vcycle, tol=1e-14)
    assert np.linalg.norm(alpha - ref) < 1e-10 * np.linalg.norm(ref)
    assert it < 200
    _, it_cg, _ = mg.cg(A, b, tol=1e-8)
    _, it_mg, _ = mg.pcg(A, b, small_mg.vcycle, tol=1e-8)
    assert it_mg < it_cg


def test_vcycle_symmetric_positive_definite(small_mg):
    rng = np.random.default_rng(45)
    u, v = rng.standard_normal((2, small_mg.levels[small_mg.G]["A"].shape[0]))
    Bu, Bv = small_mg.vcycle(u), small_mg.vcycle(v)
    assert abs(v @ Bu - u @ Bv) < 1e-12 * abs(v @ Bu)
    assert u @ Bu > 0 and v @ Bv > 0


def test_vcycle_special_cases():
    rng = np.random.default_rng(46)
    x = rng.random((800, 2))
    y = rng.standard_normal(800)
    # G = 1: the V-cycle is the exact coarse solve
    m1 = mg.MG(x, y, [0, 0], [1, 1], 2, 1e-2)
    A1 = m1.levels[1]["A"].toarray()
    r = rng.standard_normal(A1.shape[0])
    assert np.allclose(m1.vcycle(r), np.linalg.solve(A1, r), rtol=1e-10, atol=1e-12)
    # two grids, no smoothing: B = I A_1^-1 I'
    m2 = mg.MG(x, y, [0, 0], [1, 1], 4, 1e-2, nu1=0, nu2=0)
    P = m2.levels[2]["P"].toarray()
    A1 = m2.levels[1]["A"].toarray()
    r = rng.standard_normal(P.shape[0])
    assert np.allclose(m2.vcycle(r), P @ np.linalg.solve(A1, P.T @ r), rtol=1e-10, atol=1e-12)


def test_lanczos_estimate_bounds_spectral_radius(small_mg):
    for g in range(2, small_mg.G + 1):
        A = small_mg.levels[g]["A"]
        Dm = 1.0 / np.sqrt(A.diagonal())
        S = A.multiply(Dm[:, None]).multiply(Dm[None, :]).tocsr()
        rho = spla.eigsh(S, k=1, which="LA", return_eigenvectors=False)[0]
        theta = mg.lanczos_rho(A)
        assert theta <= rho * (1 + 1e-10)
        assert theta >= 0.95 * rho


def test_singular_when_data_lie_on_a_line():
    """An affine function vanishing at every point makes A singular (no unique fit)."""
    rng = np.random.default_rng(47)
    t = rng.random(500)
    x = np.column_stack([t, t])          # x1 - x2 = 0 at every point
    A, _, _, _ = system.system(x, rng.standard_normal(500), [0, 0], [1, 1], 2, 1e-2)
    ev = np.linalg.eigvalsh(A.toarray())
    assert ev.min() < 1e-12 * ev.max()
