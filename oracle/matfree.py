"""Matrix-free CPU apply and sampled outputs (test oracle, FP64).

For sizes where assembling A is too large, this computes the same products
as ``system`` without forming Phi or Lambda: the Khatri-Rao products of
Alg. 3 / Alg. 4 (s = Phi c, then Phi' s, one point at a time in vectorised
form) and the Kronecker structure of Lambda (Sec. 2.4) through the 1D Gram
matrices of ``system.gram_1d``.

``apply_rows`` returns selected entries (A c)[k] exactly, using only the
points whose cell lies in the support of phi_k; it serves as the oracle for
full-size problems, where the complete product is too slow on a CPU.

``LevelOperator`` is A_g as an operator for the multigrid oracle at sizes
where the Kronecker products of Lambda are too large to assemble: Phi_g as a
sparse matrix, Lambda_g through its 1D factors. ``lambda_diagonal`` is the
diagonal of Lambda from the diagonals of the 1D factors (the diagonal of a
Kronecker product is the Kronecker product of the diagonals, Sec. 3.1.3).

Pinned by tests/test_oracle_system.py (matrix-free products and rows,
LevelOperator and lambda_diagonal) against the assembled ``system`` on small
problems.
"""
import itertools
import math

import numpy as np

from . import bspline, system


def _point_basis(x, lo, hi, N, q):
    d = x.shape[1]
    cells, vals = [], []
    for p in range(d):
        c, V = bspline.basis_local(x[:, p], lo[p], hi[p], N, q)
        cells.append(c)
        vals.append(V)
    return cells, vals


def phi_apply(x, c, lo, hi, N, q=3):
    """s = Phi c (Alg. 4, the transposed Khatri-Rao product)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    n, d = x.shape
    J = N + q
    cells, vals = _point_basis(x, lo, hi, N, q)
    s = np.zeros(n)
    for a in itertools.product(range(q + 1), repeat=d):
        col = np.zeros(n, dtype=np.int64)
        val = np.ones(n)
        for p in range(d):
            col = col * J + (cells[p] + a[p])
            val = val * vals[p][:, a[p]]
        s += val * c[col]
    return s


def phit_apply(x, s, lo, hi, N, q=3):
    """w = Phi' s (Alg. 3, the Khatri-Rao product)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    n, d = x.shape
    J = N + q
    cells, vals = _point_basis(x, lo, hi, N, q)
    w = np.zeros(J ** d)
    for a in itertools.product(range(q + 1), repeat=d):
        col = np.zeros(n, dtype=np.int64)
        val = np.ones(n)
        for p in range(d):
            col = col * J + (cells[p] + a[p])
            val = val * vals[p][:, a[p]]
        w += np.bincount(col, weights=val * s, minlength=J ** d)
    return w


def _grams(d, lo, hi, N, q):
    return [[system.gram_1d(lo[p], hi[p], N, q, r) for r in range(3)]
            for p in range(d)]


def _terms(d):
    for r in itertools.product(range(3), repeat=d):
        if sum(r) == 2:
            yield r, 2.0 / np.prod([math.factorial(rp) for rp in r])


def lambda_apply(c, d, lo, hi, N, q=3):
    """Lambda c through the Kronecker factors, one dimension at a time (Alg. 2)."""
    J = N + q
    grams = _grams(d, lo, hi, N, q)
    out = np.zeros(J ** d)
    for r, coef in _terms(d):
        T = c.reshape((J,) * d)
        for p in range(d):
            T = np.moveaxis(np.tensordot(grams[p][r[p]], T, axes=([1], [p])), 0, p)
        out += coef * T.ravel()
    return out


def apply(x, c, lo, hi, N, lam, q=3):
    """(Phi'Phi + lam Lambda) c without assembly."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    d = x.shape[1]
    s = phi_apply(x, c, lo, hi, N, q)
    return phit_apply(x, s, lo, hi, N, q) + lam * lambda_apply(c, d, lo, hi, N, q)


def rhs(x, y, lo, hi, N, q=3):
    """b = Phi' y."""
    return phit_apply(x, np.asarray(y, dtype=np.float64), lo, hi, N, q)


def apply_rows(x, c, lo, hi, N, lam, ks, q=3):
    """(A c)[k] for each flat coefficient index k in ``ks``.

    Uses only points in cells j_p - q .. j_p of the support of phi_k.
    """
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    n, d = x.shape
    J = N + q
    grams = _grams(d, lo, hi, N, q)
    cells = np.stack([bspline.cell_index(x[:, p], lo[p], hi[p], N)
                      for p in range(d)], axis=1)
    out = np.zeros(len(ks))
    C = c.reshape((J,) * d)
    for idx, k in enumerate(ks):
        jk = np.array(np.unravel_index(int(k), (J,) * d))
        sel = np.all((cells >= jk - q) & (cells <= jk), axis=1)
        xs = x[sel]
        if xs.shape[0]:
            s = phi_apply(xs, c, lo, hi, N, q)
            vk = np.ones(xs.shape[0])
            for p in range(d):
                vk *= bspline.basis_dense(xs[:, p], lo[p], hi[p], N, q)[:, jk[p]]
            out[idx] = vk @ s
        # Lambda row k: sum over terms of prod_p Psi^p[j_p, :] contracted with C
        lam_k = 0.0
        for r, coef in _terms(d):
            T = C
            for p in range(d):
                T = np.tensordot(grams[p][r[p]][jk[p]], T, axes=([0], [0]))
            lam_k += coef * float(T)
        out[idx] += lam * lam_k
    return out


def evaluate(alpha, xq, lo, hi, N, q=3):
    """s(x_q) = sum_k alpha_k phi_k(x_q) without assembly."""
    return phi_apply(np.atleast_2d(xq), np.asarray(alpha, dtype=np.float64),
                     lo, hi, N, q)


def lambda_diagonal(d, lo, hi, N, q=3):
    """diag(Lambda) = sum over |r| = 2 of (2/r!) kron_p diag(Psi^p_{r_p})."""
    grams = _grams(d, lo, hi, N, q)
    out = np.zeros((N + q) ** d)
    for r, coef in _terms(d):
        v = np.ones(1)
        for p in range(d):
            v = np.kron(v, np.diag(grams[p][r[p]]))
        out += coef * v
    return out


class LevelOperator:
    """A_g = Phi_g'Phi_g + lam Lambda_g as an operator (``@``, ``diagonal()``).

    Phi_g is assembled sparse (n x K, (q+1)^d nonzeros per row, Sec. 2.4) and
    applied as Phi_g'(Phi_g c); Lambda_g c goes through the 1D factors
    (``lambda_apply``). The diagonal is the column sums of Phi_g squared
    (Alg. 5) plus lam times ``lambda_diagonal``.
    """

    def __init__(self, x, lo, hi, N, lam, q=3):
        x = np.atleast_2d(np.asarray(x, dtype=np.float64))
        self.d = x.shape[1]
        self.lo, self.hi, self.N, self.lam, self.q = lo, hi, N, lam, q
        self.Phi = system.phi_matrix(x, lo, hi, N, q).tocsr()
        self.PhiT = self.Phi.T.tocsr()
        K = (N + q) ** self.d
        self.shape = (K, K)
        self._diag = (np.asarray(self.Phi.multiply(self.Phi).sum(axis=0)).ravel()
                      + lam * lambda_diagonal(self.d, lo, hi, N, q))

    def __matmul__(self, c):
        c = np.asarray(c, dtype=np.float64)
        return (self.PhiT @ (self.Phi @ c)
                + self.lam * lambda_apply(c, self.d, self.lo, self.hi, self.N, self.q))

    def diagonal(self):
        return self._diag


def operator_hierarchy(x, y, lo, hi, N, lam, q=3, G=None, coarsest=1):
    """Levels c..G for ``mg.MG(levels=...)`` without assembling A_g above c.

    Level g > c holds a ``LevelOperator``; level c holds the dense A_c
    (``system.normal_matrix_dense``); the finest level holds b = Phi'y; every
    level above c holds the prolongation from the level below (eq. 2.6).
    """
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    d = x.shape[1]
    if G is None:
        G = int(round(math.log2(N)))
    levels = {}
    for g in range(coarsest, G + 1):
        Ng = N >> (G - g)
        if g == coarsest:
            lev = {"N": Ng, "A": system.normal_matrix_dense(x, lo, hi, Ng, lam, q)}
        else:
            lev = {"N": Ng, "A": LevelOperator(x, lo, hi, Ng, lam, q),
                   "P": system.prolongation(d, Ng // 2, q)}
        if g == G:
            op = lev["A"]
            lev["b"] = (op.PhiT @ np.asarray(y, dtype=np.float64) if isinstance(op, LevelOperator)
                        else system.phi_matrix(x, lo, hi, Ng, q).T @ np.asarray(y, dtype=np.float64))
        levels[g] = lev
    return levels
