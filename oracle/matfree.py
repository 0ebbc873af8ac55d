"""Matrix-free CPU apply and sampled outputs (test oracle, FP64).

For sizes where assembling A is too large, this computes the same products
as ``system`` without forming Phi or Lambda: the Khatri-Rao products of
Alg. 3 / Alg. 4 (s = Phi c, then Phi' s, one point at a time in vectorised
form) and the Kronecker structure of Lambda (Sec. 2.4) through the 1D Gram
matrices of ``system.gram_1d``.

``apply_rows`` returns selected entries (A c)[k] exactly, using only the
points whose cell lies in the support of phi_k; it serves as the oracle for
full-size problems, where the complete product is too slow on a CPU.

Pinned by tests/test_oracle_matfree.py against the assembled ``system`` on
small problems.
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
