"""Pins of the oracle's general form (Sec. 2.1: degree q_p and knots per
dimension; Sec. 3.2.1: the grid hierarchy): B-splines of degree q != 3,
anisotropic and non-power-of-two grids. Each pin is a property the
mathematics fixes independently of the code: partition of unity, exact
reproduction of affine functions, exactness of the subdivision
prolongation, the Galerkin identity and the null space of Lambda."""
import numpy as np
import pytest

from oracle import bspline, mg, system


@pytest.mark.parametrize("q", [1, 2, 4, 5])
@pytest.mark.parametrize("N,lo,hi", [(3, 0.0, 1.0), (12, -1.0, 2.5)])
def test_partition_of_unity_any_degree(q, N, lo, hi):
    x = np.random.default_rng(q * 10 + N).uniform(lo, hi, 500)
    x[:2] = [lo, hi]
    _, V = bspline.basis_local(x, lo, hi, N, q)
    assert np.abs(V.sum(axis=1) - 1.0).max() <= 1e-14
    assert V.min() >= -1e-15


@pytest.mark.parametrize("q", [1, 2, 4, 5])
def test_greville_reproduces_x_any_degree(q):
    lo, hi, N = -0.5, 1.5, 7
    x = np.random.default_rng(q).uniform(lo, hi, 300)
    B = bspline.basis_dense(x, lo, hi, N, q)
    assert np.abs(B @ bspline.greville(lo, hi, N, q) - x).max() <= 1e-13


@pytest.mark.parametrize("Nc,q", [((2, 4), (2, 3)), ((3, 2), (4, 1)), ((4,), (5,)), ((2, 3, 2), (2, 2, 4))])
def test_subdivision_exact_anisotropic(Nc, q):
    """eq. 2.5/2.6 per dimension: the coarse spline with coefficients a equals
    the fine spline (every interval halved) with coefficients I a."""
    d = len(Nc)
    lo, hi = [0.0] * d, [1.0] * d
    rng = np.random.default_rng(sum(Nc) + sum(q))
    Kc = system.num_coeffs(list(Nc), list(q), d)
    a = rng.standard_normal(Kc)
    x = rng.random((400, d))
    Nf = [2 * n for n in Nc]
    coarse = system.phi_matrix(x, lo, hi, list(Nc), list(q)) @ a
    fine = system.phi_matrix(x, lo, hi, Nf, list(q)) @ (system.prolongation(d, list(Nc), list(q)) @ a)
    assert np.abs(coarse - fine).max() <= 1e-13 * np.abs(coarse).max()


@pytest.mark.parametrize("N,q", [((8, 4), (3, 3)), ((6, 12), (2, 3)), ((12,), (4,))])
def test_galerkin_identity_general(N, q):
    """A_g = I' A_{g+1} I (Sec. 3.2.3) on general grids and degrees."""
    d = len(N)
    rng = np.random.default_rng(sum(N))
    x = rng.random((700, d))
    y = rng.standard_normal(700)
    lev = system.hierarchy(x, y, [0.0] * d, [1.0] * d, list(N), 1e-2, list(q))
    G = max(lev)
    assert G >= 2
    for g in range(2, G + 1):
        P = lev[g]["P"]
        Ac = (P.T @ lev[g]["A"] @ P).toarray()
        ref = lev[g - 1]["A"].toarray()
        assert np.abs(Ac - ref).max() <= 1e-12 * np.abs(ref).max(), g


@pytest.mark.parametrize("N,q", [((5, 3), (2, 3)), ((4, 6), (4, 2)), ((3, 2, 4), (3, 2, 2))])
def test_lambda_null_space_is_affine_general(N, q):
    """Lambda alpha = 0 for the coefficients of any affine function (Greville
    abscissae per dimension), and exactly d + 1 zero eigenvalues."""
    d = len(N)
    lo, hi = [0.0] * d, [1.0] * d
    L = system.lambda_matrix(d, lo, hi, list(N), list(q)).toarray()
    grids = [bspline.greville(lo[p], hi[p], N[p], q[p]) for p in range(d)]
    ones = [np.ones(N[p] + q[p]) for p in range(d)]
    for p in range(d):
        v = np.ones(1)
        for r in range(d):
            v = np.kron(v, grids[r] if r == p else ones[r])
        assert np.abs(L @ v).max() <= 1e-9 * np.abs(L).max()
    ev = np.linalg.eigvalsh(L)
    assert np.sum(np.abs(ev) <= 1e-10 * ev.max()) == d + 1


def test_num_levels_rule():
    assert system.num_levels(32) == 5 and system.num_levels([32, 32]) == 5
    assert system.num_levels([64, 32, 16]) == 5          # coarsest (4, 2, 1)
    assert system.num_levels([24, 12]) == 3              # coarsest (6, 3)
    assert system.num_levels([6, 6]) == 2 and system.num_levels([3, 5]) == 1


def test_mgcg_general_grid_reaches_direct_solution():
    """MGCG (Alg. 8) on an anisotropic, non-power-of-two grid with mixed
    degrees converges to the direct solution."""
    rng = np.random.default_rng(5)
    x = rng.random((3000, 2))
    y = np.sin(3 * x[:, 0]) * x[:, 1] + 0.05 * rng.standard_normal(3000)
    N, q = [24, 12], [3, 2]
    M = mg.MG(x, y, [0.0, 0.0], [1.0, 1.0], N, 1e-3, q=q, levels=system.hierarchy(x, y, [0, 0], [1, 1], N, 1e-3, q))
    lev = M.levels[M.G]
    a, its, _ = mg.pcg(lev["A"], lev["b"], M.vcycle, tol=1e-12, maxiter=500)
    ref = mg.solve_direct(lev["A"], lev["b"])
    assert np.linalg.norm(a - ref) <= 1e-8 * np.linalg.norm(ref), its
