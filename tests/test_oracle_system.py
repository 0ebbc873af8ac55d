"""Pins of the oracle's assembled system (Sec. 2.2, 2.4): Gram stencils from
the B-spline autocorrelation identity, the null space of Lambda, the penalty
as an integrated squared Hessian, symmetry and definiteness of A, Phi against
a dense Kronecker brute force, the diagonal formula, Table 1, and the
matrix-free oracle against the assembled one."""
import itertools
import math
import os

import numpy as np
import pytest

from oracle import bspline, matfree, system

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def cardinal(v, deg, r=0):
    """r-th derivative of the cardinal B-spline of degree deg on [0, deg+1]."""
    v = np.asarray(v, dtype=np.float64)
    out = np.zeros_like(v)
    for k in range(deg + 2):
        z = np.maximum(v - k, 0.0)
        out += (-1) ** k * math.comb(deg + 1, k) * (math.factorial(deg) / math.factorial(deg - r)) * z ** (deg - r)
    return out / math.factorial(deg)


def test_gram_interior_rows_golden_and_autocorrelation():
    lo, hi, N = 0.0, 2.0, 16
    h = (hi - lo) / N
    rows = [l.split() for l in open(os.path.join(GOLDEN, "gram_interior_stencils.txt"))
            if l.strip() and not l.startswith("#")]
    for row in rows:
        r = int(row[0])
        nums = np.array([float(v) for v in row[2:9]])
        den = float(row[9])
        golden = nums / den * h ** (1 - 2 * r)
        # autocorrelation identity with the degree-7 cardinal B-spline
        k = np.arange(-3, 4)
        auto = (-1) ** r * cardinal(4 + k, 7, 2 * r) * h ** (1 - 2 * r)
        assert np.allclose(golden, auto, rtol=1e-12, atol=1e-12 * abs(auto).max())
        G = system.gram_1d(lo, hi, N, 3, r)
        for j in range(3, N):           # rows unaffected by the ends of the box
            assert np.allclose(G[j, j - 3:j + 4], golden, rtol=1e-12, atol=1e-12 * abs(golden).max())


@pytest.mark.parametrize("d,N", [(1, 8), (2, 4), (3, 2)])
def test_lambda_null_space_is_affine(d, N):
    lo, hi = [0.0] * d, [1.0] * d
    L = system.lambda_matrix(d, lo, hi, N).toarray()
    J = N + 3
    xi = bspline.greville(0.0, 1.0, N, 3)
    ones = np.ones(J ** d)
    assert np.abs(L @ ones).max() < 1e-10 * np.abs(L).max()
    for p in range(d):
        v = np.ones(1)
        for q in range(d):
            v = np.kron(v, xi if q == p else np.ones(J))
        assert np.abs(L @ v).max() < 1e-10 * np.abs(L).max()
    ev = np.linalg.eigvalsh(L)
    assert np.sum(np.abs(ev) < 1e-10 * ev.max()) == d + 1
    assert ev.min() > -1e-10 * ev.max()


def _hessian_energy(alpha, lo, hi, N, frobenius=True):
    """int over [lo,hi]^2 of ||Hess s||_F^2 (or of (sum of its entries)^2) by
    Gauss-Legendre with 6 nodes per interval, derivatives of the 1D bases."""
    nodes, weights = np.polynomial.legendre.leggauss(6)
    A = alpha.reshape(N + 3, N + 3)
    total = 0.0
    for cx in range(N):
        for cy in range(N):
            ax, bx = lo[0] + cx * (hi[0] - lo[0]) / N, lo[0] + (cx + 1) * (hi[0] - lo[0]) / N
            ay, by = lo[1] + cy * (hi[1] - lo[1]) / N, lo[1] + (cy + 1) * (hi[1] - lo[1]) / N
            xs = 0.5 * (ax + bx) + 0.5 * (bx - ax) * nodes
            ys = 0.5 * (ay + by) + 0.5 * (by - ay) * nodes
            wx = 0.5 * (bx - ax) * weights
            wy = 0.5 * (by - ay) * weights
            Bx = [bspline.basis_dense(xs, lo[0], hi[0], N, 3, r) for r in range(3)]
            By = [bspline.basis_dense(ys, lo[1], hi[1], N, 3, r) for r in range(3)]
            sxx = Bx[2] @ A @ By[0].T
            syy = Bx[0] @ A @ By[2].T
            sxy = Bx[1] @ A @ By[1].T
            if frobenius:
                f = sxx ** 2 + syy ** 2 + 2 * sxy ** 2
            else:
                f = (sxx + syy + 2 * sxy) ** 2
            total += np.einsum("i,j,ij->", wx, wy, f)
    return total


def test_penalty_is_integrated_squared_hessian():
    rng = np.random.default_rng(5)
    lo, hi, N = [0.0, -1.0], [2.0, 0.5], 4
    L = system.lambda_matrix(2, lo, hi, N)
    for _ in range(3):
        a = rng.standard_normal((N + 3) ** 2)
        e = _hessian_energy(a, lo, hi, N)
        assert abs(a @ (L @ a) - e) < 1e-10 * abs(e)
        # the literal square-of-the-sum integrand is a different quantity
        assert abs(a @ (L @ a) - _hessian_energy(a, lo, hi, N, frobenius=False)) > 1e-3 * abs(e)


@pytest.mark.parametrize("d,N,n", [(1, 8, 60), (2, 4, 150), (3, 2, 120)])
def test_phi_equals_dense_kronecker_brute_force(d, N, n):
    rng = np.random.default_rng(6)
    lo, hi = list(rng.uniform(-1, 0, d)), list(rng.uniform(1, 2, d))
    x = np.stack([rng.uniform(lo[p], hi[p], n) for p in range(d)], axis=1)
    Phi = system.phi_matrix(x, lo, hi, N).toarray()
    for i in range(n):
        row = np.ones(1)
        for p in range(d):
            row = np.kron(row, bspline.basis_dense(x[i:i + 1, p], lo[p], hi[p], N, 3)[0])
        assert np.abs(Phi[i] - row).max() < 1e-15


@pytest.mark.parametrize("d,N,n,lam", [(2, 8, 400, 1e-3), (3, 4, 600, 1e-2)])
def test_system_symmetric_positive_definite(d, N, n, lam):
    rng = np.random.default_rng(7)
    x = rng.random((n, d))
    y = rng.standard_normal(n)
    A, b, Phi, Lam = system.system(x, y, [0.0] * d, [1.0] * d, N, lam)
    u, v = rng.standard_normal((2, A.shape[0]))
    assert abs(u @ (A @ v) - v @ (A @ u)) < 1e-12 * abs(u @ (A @ v)) + 1e-14
    np.linalg.cholesky(A.toarray())
    assert np.allclose(b, Phi.T @ y)


def test_diagonal_formula():
    """diag(A) = sum_i Phi[i,k]^2 (Alg. 5) + lambda * sum_r (2/r!) prod_p diag(Psi^p)."""
    rng = np.random.default_rng(8)
    d, N, n, lam = 3, 4, 500, 0.3
    lo, hi = [0.0] * d, [1.0, 2.0, 0.5]
    x = np.stack([rng.uniform(lo[p], hi[p], n) for p in range(d)], axis=1)
    A, _, Phi, _ = system.system(x, np.zeros(n), lo, hi, N, lam)
    data = np.asarray(Phi.multiply(Phi).sum(axis=0)).ravel()
    diags = [[np.diag(system.gram_1d(lo[p], hi[p], N, 3, r)) for r in range(3)] for p in range(d)]
    lamd = np.zeros_like(data)
    for r in itertools.product(range(3), repeat=d):
        if sum(r) != 2:
            continue
        v = np.ones(1)
        for p in range(d):
            v = np.kron(v, diags[p][r[p]])
        lamd += 2.0 / np.prod([math.factorial(q) for q in r]) * v
    assert np.allclose(A.diagonal(), data + lam * lamd, rtol=1e-13)


def test_table1_num_coeffs():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "table1_num_coeffs.txt"))
            if l.strip() and not l.startswith("#")]
    for P, K in rows:
        assert system.num_coeffs(32, 3, int(P)) == int(K)


@pytest.mark.parametrize("d,N,n", [(2, 8, 300), (3, 4, 400), (4, 2, 300)])
def test_matrix_free_matches_assembled(d, N, n):
    rng = np.random.default_rng(9)
    lo, hi = [0.0] * d, [1.0] * d
    x = rng.random((n, d))
    y = rng.standard_normal(n)
    lam = 0.01
    A, b, _, _ = system.system(x, y, lo, hi, N, lam)
    c = rng.standard_normal(A.shape[0])
    ref = A @ c
    assert np.abs(matfree.apply(x, c, lo, hi, N, lam) - ref).max() < 1e-12 * np.abs(ref).max()
    assert np.abs(matfree.rhs(x, y, lo, hi, N) - b).max() < 1e-12 * np.abs(b).max()
    ks = rng.integers(0, A.shape[0], 12)
    assert np.abs(matfree.apply_rows(x, c, lo, hi, N, lam, ks) - ref[ks]).max() < 1e-12 * np.abs(ref).max()


def test_planted_mistakes_are_caught(monkeypatch):
    """The pins above fail on plausible mistakes planted in the oracle."""
    lo, hi, N = [0.0, -1.0], [2.0, 0.5], 4
    a = np.random.default_rng(10).standard_normal((N + 3) ** 2)
    e = _hessian_energy(a, lo, hi, N)
    # (1) cross terms weighted 1 instead of 2/r! = 2
    orig_factorial = math.factorial
    monkeypatch.setattr(system.math, "factorial", lambda k: 2 if k == 1 else orig_factorial(k))
    L_bad = system.lambda_matrix(2, lo, hi, N)
    monkeypatch.undo()
    assert abs(a @ (L_bad @ a) - e) > 1e-3 * abs(e)
    # (2) Kronecker factors in the wrong order (dimension 1 most significant)
    rng = np.random.default_rng(11)
    x = rng.random((50, 2)) * [1.0, 1.0]
    Phi = system.phi_matrix(x, [0, 0], [1, 1], 4).toarray()
    row_swapped = np.kron(bspline.basis_dense(x[:1, 1], 0, 1, 4, 3)[0],
                          bspline.basis_dense(x[:1, 0], 0, 1, 4, 3)[0])
    assert np.abs(Phi[0] - row_swapped).max() > 1e-3
