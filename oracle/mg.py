"""Assembled-matrix multigrid, MGCG, CG and the direct solve (test oracle, FP64).

The V-cycle follows Alg. 7 of arXiv:1901.00654 step by step on explicitly
assembled sparse matrices A_g (from ``system.hierarchy``): damped Jacobi
(Alg. 6), residual r = A_g alpha - b, restriction by the transposed
prolongation (Sec. 3.2.3), recursion with a zero start, correction
alpha <- alpha - I e, post-smoothing; the coarsest level g = 1 is solved
exactly with a dense Cholesky factor (Sec. 3.2.4). MGCG follows Alg. 8.

Readings where the paper is silent or inconsistent:
- Alg. 8 takes the step length as ||r||^2 / p'v but the direction update
  with r'z; the preconditioned step r'z / p'v is used (standard PCG).
- The start is alpha = 0 and the stop is ||r_k||_2 / ||b||_2 <= tol on the
  recursively updated residual; neither is stated.
- The Jacobi damping omega and the smoothing counts are not given. omega_g
  is taken as omega_scale / theta_g, where theta_g is the largest Ritz value
  of a fixed number of plain Lanczos steps on D_g^-1/2 A_g D_g^-1/2 from a
  fixed start vector (``lanczos_rho``). theta_g <= rho(D_g^-1 A_g) and is
  within a few per cent of it after 16 steps, so omega_scale = 1.5 keeps
  omega_g rho < 2: damped Jacobi stays A-norm contractive and the symmetric
  V-cycle stays SPD, as CG needs.
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


def jacobi_omega(A, omega_scale=1.5, steps=16):
    """omega_g = omega_scale / lanczos_rho(A_g) (reading; the paper gives none)."""
    return omega_scale / lanczos_rho(A, steps)


def jac(A, Dinv, omega, alpha, b, nu):
    """Alg. 6: nu damped Jacobi sweeps alpha <- alpha + omega D^-1 (b - A alpha)."""
    for _ in range(nu):
        r = b - A @ alpha
        alpha = alpha + omega * Dinv * r
    return alpha


class MG:
    """Assembled hierarchy plus smoother data; ``vcycle(b)`` is Alg. 7 from zero."""

    def __init__(self, x, y, lo, hi, N, lam, q=3, nu1=2, nu2=2, omega_scale=1.5,
                 G=None, lanczos_steps=16):
        self.levels = system.hierarchy(x, y, lo, hi, N, lam, q, G)
        self.G = max(self.levels)
        self.nu1, self.nu2 = nu1, nu2
        self.omega = {}
        self.Dinv = {}
        for g, lev in self.levels.items():
            self.Dinv[g] = 1.0 / lev["A"].diagonal()
            self.omega[g] = jacobi_omega(lev["A"], omega_scale, lanczos_steps)
        A1 = self.levels[1]["A"].toarray()
        self.coarse = sla.cho_factor(A1, lower=True)

    def coarse_solve(self, b):
        return sla.cho_solve(self.coarse, b)

    def vcycle(self, b, g=None):
        if g is None:
            g = self.G
        if g == 1:
            return self.coarse_solve(b)
        lev = self.levels[g]
        A = lev["A"]
        alpha = np.zeros_like(b)
        alpha = jac(A, self.Dinv[g], self.omega[g], alpha, b, self.nu1)
        r = A @ alpha - b
        r = lev["P"].T @ r
        e = self.vcycle(r, g - 1)
        alpha = alpha - lev["P"] @ e
        alpha = jac(A, self.Dinv[g], self.omega[g], alpha, b, self.nu2)
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
