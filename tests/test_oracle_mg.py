"""Pins of the oracle's multigrid (Alg. 6-8, Sec. 3.2) beyond MGCG reaching the
direct solution (test_oracle_solve): the V-cycle against the recursion for its
iteration matrix C_MG printed in Sec. 3.2.5, the SSOR sweep against the
closed-form SSOR preconditioner, the operator form of the hierarchy against
the assembled one, and plain CG on the paper's test data against the
iteration counts of Table 2."""
import os

import numpy as np
import pytest

from oracle import matfree, mg, system
from paper_1901_00654_amd import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table2_iterations.txt")


def _small(d, N, n, lam, seed):
    rng = np.random.default_rng(seed)
    x = rng.random((n, d))
    y = np.sin(2 * np.pi * x.sum(axis=1)) + 0.1 * rng.standard_normal(n)
    return x, y, [0.0] * d, [1.0] * d, N, lam


@pytest.mark.parametrize("d,N,smoother,nu1,nu2,coarsest", [
    (2, 8, "jacobi", 1, 1, 1), (2, 8, "jacobi", 2, 2, 1), (2, 8, "jacobi", 0, 3, 1),
    (2, 16, "jacobi", 2, 2, 2), (3, 4, "jacobi", 2, 2, 1), (2, 8, "ssor", 1, 1, 1), (2, 8, "ssor", 2, 2, 2)])
def test_vcycle_equals_iteration_matrix_recursion(d, N, smoother, nu1, nu2, coarsest):
    """Sec. 3.2.5: one V-cycle from zero is z = B r with I - B A = C_MG,G,
    C_MG,c = 0 and C_MG,g = S^nu2 (I - I (I - C_MG,g-1) A_{g-1}^-1 I' A_g) S^nu1.
    The recursion is built from dense matrices, independently of the
    recursive vcycle code; a dropped smoothing step, a wrong sign of the
    correction or a transposed transfer changes B."""
    x, y, lo, hi, N, lam = _small(d, N, 600 if d == 2 else 900, 1e-2, 7)
    M = mg.MG(x, y, lo, hi, N, lam, nu1=nu1, nu2=nu2, smoother=smoother, coarsest=coarsest)
    A = M.levels[M.G]["A"].toarray()
    B_rec = (np.eye(A.shape[0]) - M.iteration_matrix()) @ np.linalg.inv(A)
    B = M.matrix()
    assert np.abs(B - B_rec).max() <= 1e-10 * np.abs(B).max()
    if nu1 == nu2:
        assert np.abs(B - B.T).max() <= 1e-12 * np.abs(B).max()


def test_vcycle_exact_on_coarsest_level():
    x, y, lo, hi, N, lam = _small(2, 8, 500, 1e-2, 8)
    M = mg.MG(x, y, lo, hi, N, lam, coarsest=3)
    A = M.levels[3]["A"].toarray()
    r = np.random.default_rng(1).standard_normal(A.shape[0])
    assert np.abs(A @ M.vcycle(r) - r).max() <= 1e-10 * np.abs(r).max()


@pytest.mark.parametrize("omega", [1.0, 1.4])
def test_ssor_step_matches_closed_form(omega):
    """One forward and backward sweep over the colour classes equals
    x + M^-1 (b - A x) with M = (D/w + L) ((2-w)/w D)^-1 (D/w + U) for the
    class-by-class order of the unknowns."""
    x, y, lo, hi, N, lam = _small(2, 8, 500, 1e-2, 9)
    A, _, _, _ = system.system(x, y, lo, hi, N, lam)
    classes = mg.color_classes(N + 3, 2)
    rng = np.random.default_rng(2)
    x0, b = rng.standard_normal((2, A.shape[0]))
    x1 = mg.ssor(A, A.diagonal(), omega, x0, b, 1, classes)
    M = mg.ssor_matrix(A, omega, classes)
    ref = x0 + np.linalg.solve(M, b - A @ x0)
    assert np.abs(x1 - ref).max() <= 1e-11 * np.abs(ref).max()


def test_color_classes_do_not_couple():
    """Rows of one colour class have no coupling in A (a cubic B-spline's
    support spans four cells), which makes the simultaneous class update a
    Gauss-Seidel sweep."""
    x, y, lo, hi, N, lam = _small(3, 4, 800, 1e-2, 10)
    A, _, _, _ = system.system(x, y, lo, hi, N, lam)
    A = A.toarray()
    classes = mg.color_classes(N + 3, 3)
    assert sorted(np.concatenate(classes).tolist()) == list(range(A.shape[0]))
    for rows in classes:
        sub = A[np.ix_(rows, rows)]
        assert np.count_nonzero(sub - np.diag(np.diag(sub))) == 0


def test_operator_hierarchy_matches_assembled():
    """The operator levels (sparse Phi, Kronecker Lambda, cell-block dense
    coarse matrix) give the same A_g products, diagonals, coarse matrix,
    right-hand side and V-cycle as the assembled hierarchy."""
    x, y, lo, hi, N, lam = _small(3, 8, 1500, 1e-2, 11)
    lev_a = system.hierarchy(x, y, lo, hi, N, lam)
    lev_o = matfree.operator_hierarchy(x, y, lo, hi, N, lam)
    rng = np.random.default_rng(3)
    for g in (2, 3):
        c = rng.standard_normal(lev_a[g]["A"].shape[0])
        ref = lev_a[g]["A"] @ c
        assert np.abs(lev_o[g]["A"] @ c - ref).max() <= 1e-12 * np.abs(ref).max()
        assert np.allclose(lev_o[g]["A"].diagonal(), lev_a[g]["A"].diagonal(), rtol=1e-13, atol=0)
    A1 = lev_a[1]["A"].toarray()
    assert np.abs(lev_o[1]["A"] - A1).max() <= 1e-13 * np.abs(A1).max()
    assert np.allclose(lev_o[3]["b"], lev_a[3]["b"], rtol=1e-13, atol=1e-14)
    Ma = mg.MG(x, y, lo, hi, N, lam, levels=lev_a)
    Mo = mg.MG(x, y, lo, hi, N, lam, levels=lev_o)
    r = rng.standard_normal(lev_a[3]["A"].shape[0])
    za, zo = Ma.vcycle(r), Mo.vcycle(r)
    assert np.abs(za - zo).max() <= 1e-9 * np.abs(za).max()


def test_lambda_diagonal_is_diag_of_lambda():
    lo, hi = [0.0, -1.0, 0.5], [1.0, 2.0, 0.75]
    L = system.lambda_matrix(3, lo, hi, 4)
    assert np.allclose(matfree.lambda_diagonal(3, lo, hi, 4), L.diagonal(), rtol=1e-13, atol=0)
    assert np.abs(system.lambda_dense(3, lo, hi, 4) - L.toarray()).max() <= 1e-13 * abs(L).max()


def _table2():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    return {int(r[0]): (int(r[1]), int(r[2])) for r in rows}


@pytest.mark.parametrize("P", [1, 2, 3])
def test_plain_cg_counts_match_table2(P):
    """Plain CG (the comparison method of Sec. 4) depends only on A, b and the
    stopping rule. On the paper's test data with lambda read off Table 3 and
    the stopping tolerance ||r|| / ||b|| <= 1e-5, our A reproduces Table 2's
    CG counts 22 / 73 / 367 to within 1 % (22 / 74 / 369 here). A change of the
    knot convention, of the penalty's weights or of the sigmoid moves them by
    far more; this also pins the paper's unstated tolerance near 1e-5."""
    ref_cg, _ = _table2()[P]
    w = workloads.paper_sigmoid(P, N=32)
    A, b, _, _ = system.system(w["x"], w["y"], w["lo"], w["hi"], w["N"], w["lam"])
    _, its, _ = mg.cg(A, b, tol=1e-5)
    assert abs(its - ref_cg) <= max(1, 0.01 * ref_cg), (its, ref_cg)


@pytest.mark.parametrize("P", [1, 2, 3])
def test_mgcg_counts_near_table2(P):
    """MGCG with the Jacobi V-cycle at the same tolerance: Table 2 prints
    2 / 4 / 14 for P = 1 / 2 / 3; the damping and smoothing counts it used are
    not given; with nu = 2 and omega_g = 1.5 / theta_g the oracle needs
    3 / 5 / 14, within one iteration of the paper (the faster default for the
    data-dominated workloads, nu = 1 and 1.8 / theta_g, needs 7 / 7 / 18)."""
    _, ref_mg = _table2()[P]
    w = workloads.paper_sigmoid(P, N=32)
    M = mg.MG(w["x"], w["y"], w["lo"], w["hi"], w["N"], w["lam"], nu1=2, nu2=2, omega_scale=1.5)
    lev = M.levels[M.G]
    _, its, _ = mg.pcg(lev["A"], lev["b"], M.vcycle, tol=1e-5)
    assert abs(its - ref_mg) <= 1, (its, ref_mg)
