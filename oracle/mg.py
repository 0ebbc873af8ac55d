"""Assembled-matrix multigrid, MGCG, CG and the direct solve (test oracle, FP64).

The V-cycle follows Alg. 7 of arXiv:1901.00654 step by step on explicitly
assembled sparse matrices A_g (from ``system.hierarchy``), or on level
operators with ``@`` and ``diagonal()`` where assembly is too large
(``matfree.operator_hierarchy``): damped Jacobi (Alg. 6) or SSOR
(Sec. 3.2.2), residual r = A_g alpha - b, restriction by the transposed
prolongation (Sec. 3.2.3), recursion with a zero start, correction
alpha <- alpha - I e, post-smoothing; the coarsest level c (g = 1 unless
chosen otherwise) is solved exactly with a dense Cholesky factor
(Sec. 3.2.4). MGCG follows Alg. 8. ``iteration_matrix`` is the recursion
for C_MG of Sec. 3.2.5, the independent check of ``MG.matrix``.

Readings where the paper is silent or inconsistent:
- Alg. 8 takes the step length as ||r||^2 / p'v but the direction update
  with r'z; the preconditioned step r'z / p'v is used (standard PCG).
- The start is alpha = 0 and the stop is ||r_k||_2 / ||b||_2 <= tol on the
  recursively updated residual; neither is stated.
- SSOR needs an order of the unknowns, which the paper does not give. The
  rows are split into 4^d colour classes by (j_1 mod 4, ..., j_d mod 4)
  (class index in C order); rows of one class never couple in A (the support
  of a cubic B-spline spans four cells), so one forward sweep updates the
  classes in order, each class at once, and the backward sweep takes them in
  reverse. This is point SSOR in the class-by-class ordering (pinned against
  the closed form M = (D/w + L) ((2-w)/w D)^-1 (D/w + U)).
- The Jacobi damping omega and the smoothing counts are not given. omega_g
  is taken as omega_scale / theta_g, where theta_g is the largest Ritz value
  of a fixed number of plain Lanczos steps on D_g^-1/2 A_g D_g^-1/2 from a
  fixed start vector (``lanczos_rho``). theta_g <= rho(D_g^-1 A_g) and is
  within a few per cent of it after 16 steps, so omega_scale < 2 keeps
  omega_g rho < 2 as long as theta_g is within omega_scale / 2 of rho: damped
  Jacobi stays A-norm contractive and the symmetric V-cycle SPD, as CG needs.
  Defaults nu1 = nu2 = 1, omega_scale = 1.8 (the fastest setting measured on
  the workloads); the comparisons with the paper's Table 2 take nu = 2,
  omega_scale = 1.5, closer to its counts.
"""

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import system


def start_vector(K):
    """Deterministic Lanczos start u[k] = frac(k * 2654435761 / 2^32) - 1/2.

    Knuth's multiplicative hash of the index; any fixed vector with
    components along every eigenvector would do.
    """
    k = np.arange(K, dtype=np.int64)
    return ((k * 2654435761) % (1 << 32)).astype(np.float64) / float(1 << 32) - 0.5


def lanczos_rho(A, steps=16):
    """Largest Ritz value of m = min(steps, K) plain Lanczos steps on D^-1/2 A D^-1/2.

    v_1 = u / ||u||; w = S v_j - beta_{j-1} v_{j-1}; alpha_j = w'v_j;
    w -= alpha_j v_j; beta_j = ||w||; v_{j+1} = w / beta_j. The result is the
    largest eigenvalue of the tridiagonal T_m (it never exceeds rho(D^-1 A)).
    Stops early when beta_j <= 1e-12 * |alpha_j| (invariant subspace).
    """
    K = A.shape[0]
    dis = 1.0 / np.sqrt(A.diagonal())
    v = start_vector(K)
    v = v / np.linalg.norm(v)
    v_prev = np.zeros(K)
    beta_prev = 0.0
    alphas, betas = [], []
    for j in range(min(steps, K)):
        w = dis * (A @ (dis * v)) - beta_prev * v_prev
        a = w @ v
        w = w - a * v
        alphas.append(a)
        b = np.linalg.norm(w)
        if j == min(steps, K) - 1 or b <= 1e-12 * abs(a):
            break
        betas.append(b)
        v_prev, v, beta_prev = v, w / b, b
    return float(sla.eigvalsh_tridiagonal(np.array(alphas), np.array(betas)).max())


def jacobi_omega(A, omega_scale=1.8, steps=16):
    """omega_g = omega_scale / lanczos_rho(A_g) (reading; the paper gives none)."""
    return omega_scale / lanczos_rho(A, steps)


def jac(A, Dinv, omega, alpha, b, nu):
    """Alg. 6: nu damped Jacobi sweeps alpha <- alpha + omega D^-1 (b - A alpha)."""
    for _ in range(nu):
        r = b - A @ alpha
        alpha = alpha + omega * Dinv * r
    return alpha


def color_classes(J, d):
    """Row sets of the SSOR colour classes on a grid of J^d coefficients.

    Class c (c = sum_p c_p 4^(d-1-p)) holds the multi-indices with
    j_p = c_p (mod 4) in every dimension p, as flat C-order indices.
    """
    idx = np.indices((J,) * d).reshape(d, -1)
    cls = np.zeros(J ** d, dtype=np.int64)
    for p in range(d):
        cls = cls * 4 + idx[p] % 4
    return [np.flatnonzero(cls == c) for c in range(4 ** d)]


def ssor(A, diag, omega, alpha, b, nu, classes):
    """nu SSOR steps: each a forward sweep over the colour classes, then a
    backward one; per class alpha_R <- alpha_R + omega (b_R - (A alpha)_R) / D_R."""
    alpha = alpha.copy()
    for _ in range(nu):
        for rows in list(classes) + list(classes)[::-1]:
            alpha[rows] += omega * (b[rows] - _rows_product(A, rows, alpha)) / diag[rows]
    return alpha


def _rows_product(A, rows, x):
    if sp.issparse(A):
        return A[rows] @ x
    if isinstance(A, np.ndarray):
        return A[rows] @ x
    return (A @ x)[rows]


def ssor_matrix(A, omega, classes):
    """The SSOR preconditioner M = (D/w + L) ((2-w)/w D)^-1 (D/w + U), written
    for the class-by-class order of the unknowns and mapped back; one SSOR
    step from x is x + M^-1 (b - A x). Dense; for checks on tiny grids."""
    A = A.toarray() if sp.issparse(A) else np.asarray(A)
    perm = np.concatenate(classes)
    Ap = A[np.ix_(perm, perm)]
    D = np.diag(np.diag(Ap))
    L = np.tril(Ap, -1)
    U = np.triu(Ap, 1)
    Mp = (D / omega + L) @ np.linalg.inv((2.0 - omega) / omega * D) @ (D / omega + U)
    M = np.empty_like(Mp)
    M[np.ix_(perm, perm)] = Mp
    return M


class MG:
    """Hierarchy plus smoother data; ``vcycle(b)`` is Alg. 7 from zero.

    ``levels`` may be given prebuilt (a dict g -> {"A", "b", "P"} as from
    ``system.hierarchy``, with "A" a sparse matrix or an operator with ``@``
    and ``diagonal()``, and a dense or sparse "A" on the coarsest level);
    otherwise the levels are assembled. ``smoother`` is "jacobi" (Alg. 6,
    damping omega_scale / theta_g or omega_fixed) or "ssor" (relaxation
    ssor_omega) on every level above the coarsest one ``coarsest``.
    """

    def __init__(self, x, y, lo, hi, N, lam, q=3, nu1=1, nu2=1, omega_scale=1.8,
                 G=None, lanczos_steps=16, levels=None, coarsest=1, smoother="jacobi",
                 ssor_omega=1.0, omega_fixed=None):
        self.levels = levels if levels is not None else system.hierarchy(x, y, lo, hi, N, lam, q, G)
        self.G = max(self.levels)
        self.c = coarsest
        self.nu1, self.nu2 = nu1, nu2
        self.smoother = smoother
        self.ssor_omega = ssor_omega
        self.omega = {}
        self.Dinv = {}
        self.diag = {}
        self.classes = {}
        d = np.atleast_2d(x).shape[1]
        for g, lev in self.levels.items():
            if g <= self.c:
                continue
            A = lev["A"]
            self.diag[g] = np.asarray(A.diagonal(), dtype=np.float64)
            self.Dinv[g] = 1.0 / self.diag[g]
            self.omega[g] = (omega_fixed if omega_fixed is not None
                             else jacobi_omega(A, omega_scale, lanczos_steps))
            if smoother == "ssor":
                self.classes[g] = color_classes(int(round(A.shape[0] ** (1.0 / d))), d)
        Ac = self.levels[self.c]["A"]
        Ac = Ac.toarray() if sp.issparse(Ac) else np.asarray(Ac)
        self.coarse = sla.cho_factor(Ac, lower=True)

    def coarse_solve(self, b):
        return sla.cho_solve(self.coarse, b)

    def smooth(self, g, alpha, b, nu):
        A = self.levels[g]["A"]
        if self.smoother == "ssor":
            return ssor(A, self.diag[g], self.ssor_omega, alpha, b, nu, self.classes[g])
        return jac(A, self.Dinv[g], self.omega[g], alpha, b, nu)

    def vcycle(self, b, g=None):
        if g is None:
            g = self.G
        if g == self.c:
            return self.coarse_solve(b)
        lev = self.levels[g]
        A = lev["A"]
        alpha = np.zeros_like(b)
        alpha = self.smooth(g, alpha, b, self.nu1)
        r = A @ alpha - b
        r = lev["P"].T @ r
        e = self.vcycle(r, g - 1)
        alpha = alpha - lev["P"] @ e
        alpha = self.smooth(g, alpha, b, self.nu2)
        return alpha

    def matrix(self):
        """The V-cycle as an explicit matrix B (columns = V-cycles of unit vectors)."""
        K = self.levels[self.G]["A"].shape[0]
        B = np.zeros((K, K))
        for k in range(K):
            e = np.zeros(K)
            e[k] = 1.0
            B[:, k] = self.vcycle(e)
        return B

    def smoother_matrix(self, g):
        """C_smooth of level g (dense): I - omega D^-1 A or I - M_SSOR^-1 A."""
        A = self.levels[g]["A"]
        A = A.toarray() if sp.issparse(A) else np.asarray(A)
        if self.smoother == "ssor":
            return np.eye(A.shape[0]) - np.linalg.solve(ssor_matrix(A, self.ssor_omega, self.classes[g]), A)
        return np.eye(A.shape[0]) - self.omega[g] * self.Dinv[g][:, None] * A

    def iteration_matrix(self, g=None):
        """C_MG,g of Sec. 3.2.5 by its recursion (dense, tiny grids only):
        C_MG,c = 0 and C_MG,g = S^nu2 (I - I_g (I - C_MG,g-1) A_{g-1}^-1 I_g' A_g) S^nu1."""
        if g is None:
            g = self.G
        K = self.levels[g]["A"].shape[0]
        if g == self.c:
            return np.zeros((K, K))
        A = self.levels[g]["A"]
        A = A.toarray() if sp.issparse(A) else np.asarray(A)
        Ac = self.levels[g - 1]["A"]
        Ac = Ac.toarray() if sp.issparse(Ac) else np.asarray(Ac)
        Pg = self.levels[g]["P"].toarray()
        Cc = self.iteration_matrix(g - 1)
        S = self.smoother_matrix(g)
        inner = np.eye(K) - Pg @ (np.eye(Ac.shape[0]) - Cc) @ np.linalg.solve(Ac, Pg.T @ A)
        return np.linalg.matrix_power(S, self.nu2) @ inner @ np.linalg.matrix_power(S, self.nu1)


def pcg(A, b, precond, tol=1e-10, maxiter=1000):
    """Alg. 8 (MGCG) with the preconditioned step length r'z / p'v.

    Returns (alpha, iterations, history of ||r_k|| / ||b||).
    """
    alpha = np.zeros_like(b)
    r = b.copy()
    bnorm = np.linalg.norm(b)
    hist = [np.linalg.norm(r) / bnorm]
    z = precond(r)
    p = z.copy()
    it = 0
    while hist[-1] > tol and it < maxiter:
        v = A @ p
        w = (r @ z) / (p @ v)
        alpha = alpha + w * p
        r_old, z_old = r, z
        r = r - w * v
        it += 1
        hist.append(np.linalg.norm(r) / bnorm)
        if hist[-1] <= tol:
            break
        z = precond(r)
        beta = (r @ z) / (r_old @ z_old)
        p = z + beta * p
    return alpha, it, hist


def cg(A, b, tol=1e-10, maxiter=100000):
    """Unpreconditioned CG (the comparison method of Sec. 4)."""
    return pcg(A, b, lambda r: r, tol, maxiter)


def solve_direct(A, b):
    """alpha* solving A alpha = b by sparse LU (SuperLU); A is SPD."""
    lu = spla.splu(sp.csc_matrix(A), permc_spec="MMD_AT_PLUS_A")
    return lu.solve(np.asarray(b, dtype=np.float64))
