"""Assembled FP64 smoothing system (test oracle).

Everything here is a direct transcription of a definition in arXiv:1901.00654,
assembled with scipy.sparse:

- Phi[i, k] = phi_k(x_i), the tensor-product B-spline basis with multi-indices
  ordered "descending lexicographically" (Sec. 2.1, eq. 2.2). Reading: j_1 is
  the most significant digit and j_P the least (C order), the only order under
  which Phi' is the Khatri-Rao product of the Phi_p' and Psi_r, I are Kronecker
  products in the natural factor order (Sec. 2.4).
- Psi^p_r[j, l] = <D^r phi_j, D^r phi_l>_{L2(Omega_p)} (Sec. 2.4), integrated
  over Omega_p = [lo, hi] by Gauss-Legendre with q+1 nodes per knot interval,
  exact for the degree-2q integrands.
- Lambda = sum_{|r|=2} (2/r!) Psi_r, Psi_r = kron_p Psi^p_{r_p} (Sec. 2.2 and
  2.4). Reading: the matrix form is taken as the definition of the penalty
  (it is the integrated squared Frobenius norm of the Hessian); the displayed
  integrand of eq. 2.3 squares the *sum* of the second derivatives instead,
  which disagrees with the matrix form for P >= 2.
- A = Phi'Phi + lambda Lambda and b = Phi'y (eq. 2.4).
- The 1D prolongation I[i, j] = 2^-q binom(q+1, i - 2j + q + 1) (1-based, from
  the subdivision formula eq. 2.5) and its Kronecker product (eq. 2.6).
  Reading: entries whose row would fall outside 1..J^h are dropped; those fine
  B-splines vanish on Omega.
- Grid hierarchy N_g = 2^g intervals per dimension, K_g = (2^g + q)^P
  (Sec. 3.2.1), A_g = Phi_g'Phi_g + lambda Lambda_g with Phi_g evaluated at
  the same data points on every level.

Pins live in tests/test_oracle_system.py and tests/test_oracle_transfer.py.
"""
import itertools
import math

import numpy as np
import scipy.sparse as sp

from . import bspline


def per_dim(v, d):
    """A scalar N or q for every dimension, or the per-dimension list itself
    (Sec. 2.1 defines q_p, J_p and the knots dimension by dimension)."""
    if np.ndim(v) == 0:
        return [int(v)] * d
    v = [int(a) for a in v]
    if len(v) != d:
        raise ValueError("expected %d per-dimension values" % d)
    return v


def num_coeffs(N, q, d):
    """K = prod_p J_p with J_p = N_p + q_p (Sec. 2.1; Table 1 for J_p = 35)."""
    return int(np.prod([Np + qp for Np, qp in zip(per_dim(N, d), per_dim(q, d))]))


def phi_matrix(x, lo, hi, N, q=3):
    """Sparse Phi (n x K) for points x (n x d) on [lo, hi]^d with N_p
    intervals and degree q_p in dimension p (scalars: the same for all).

    Row i is the Kronecker product over dimensions of the 1D rows
    Phi_p[i, :] (the Khatri-Rao identity of Sec. 2.4), built entry by entry.
    """
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    n, d = x.shape
    Ns, qs = per_dim(N, d), per_dim(q, d)
    Js = [Np + qp for Np, qp in zip(Ns, qs)]
    cells, vals = [], []
    for p in range(d):
        c, V = bspline.basis_local(x[:, p], lo[p], hi[p], Ns[p], qs[p])
        cells.append(c)
        vals.append(V)
    rows, cols, data = [], [], []
    for a in itertools.product(*[range(qp + 1) for qp in qs]):
        col = np.zeros(n, dtype=np.int64)
        val = np.ones(n)
        for p in range(d):
            col = col * Js[p] + (cells[p] + a[p])
            val = val * vals[p][:, a[p]]
        rows.append(np.arange(n))
        cols.append(col)
        data.append(val)
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    data = np.concatenate(data)
    return sp.csr_matrix((data, (rows, cols)), shape=(n, int(np.prod(Js))))


def gram_1d(lo, hi, N, q, r):
    """Dense Psi_r (J x J) on [lo, hi]: integral of D^r B_j * D^r B_l."""
    J = N + q
    h = (hi - lo) / N
    nodes, weights = np.polynomial.legendre.leggauss(q + 1)
    G = np.zeros((J, J))
    for c in range(N):
        a, b = lo + c * h, lo + (c + 1) * h
        xq = 0.5 * (a + b) + 0.5 * (b - a) * nodes
        wq = 0.5 * (b - a) * weights
        D = bspline.basis_dense(xq, lo, hi, N, q, r)   # (q+1 nodes) x J
        G += D.T @ (wq[:, None] * D)
    return G


def lambda_matrix(d, lo, hi, N, q=3):
    """Lambda = sum over multi-indices r with |r| = 2 of (2/r!) kron_p Psi^p_{r_p}."""
    Ns, qs = per_dim(N, d), per_dim(q, d)
    psi = [[sp.csr_matrix(gram_1d(lo[p], hi[p], Ns[p], qs[p], rp)) for rp in range(3)]
           for p in range(d)]
    K = num_coeffs(Ns, qs, d)
    L = sp.csr_matrix((K, K))
    for r in itertools.product(range(3), repeat=d):
        if sum(r) != 2:
            continue
        coef = 2.0 / np.prod([math.factorial(rp) for rp in r])
        term = psi[0][r[0]]
        for p in range(1, d):
            term = sp.kron(term, psi[p][r[p]], format="csr")
        L = L + coef * term
    return L.tocsr()


def lambda_dense(d, lo, hi, N, q=3):
    """Lambda as a dense array: the same sum of Kronecker products as
    ``lambda_matrix``, with dense 1D factors (for K up to a few 10^4)."""
    psi = [[gram_1d(lo[p], hi[p], N, q, rp) for rp in range(3)] for p in range(d)]
    K = (N + q) ** d
    L = np.zeros((K, K))
    for r in itertools.product(range(3), repeat=d):
        if sum(r) != 2:
            continue
        coef = 2.0 / np.prod([math.factorial(rp) for rp in r])
        term = psi[0][r[0]]
        for p in range(1, d):
            term = np.kron(term, psi[p][r[p]])
        L += coef * term
    return L


def system(x, y, lo, hi, N, lam, q=3):
    """(A, b, Phi, Lambda) with A = Phi'Phi + lam Lambda, b = Phi'y (eq. 2.4)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    d = x.shape[1]
    Phi = phi_matrix(x, lo, hi, N, q)
    Lam = lambda_matrix(d, lo, hi, N, q)
    A = (Phi.T @ Phi + lam * Lam).tocsr()
    b = Phi.T @ np.asarray(y, dtype=np.float64)
    return A, b, Phi, Lam


def prolongation_1d(Nc, q=3):
    """I_{2h}^h (J^h x J^{2h}) from the subdivision formula (eq. 2.5).

    1-based: I[i, j] = 2^-q binom(q+1, i - 2j + q + 1) for 0 <= i-2j+q+1 <= q+1.
    """
    Jc, Jf = Nc + q, 2 * Nc + q
    I = np.zeros((Jf, Jc))
    for i in range(1, Jf + 1):
        for j in range(1, Jc + 1):
            m = i - 2 * j + q + 1
            if 0 <= m <= q + 1:
                I[i - 1, j - 1] = math.comb(q + 1, m) / 2.0 ** q
    return I


def prolongation(d, Nc, q=3):
    """Multivariate I_{2h}^h = kron_p I_p (eq. 2.6), sparse; Nc and q per
    dimension or scalars."""
    Ns, qs = per_dim(Nc, d), per_dim(q, d)
    P = sp.csr_matrix(prolongation_1d(Ns[0], qs[0]))
    for p in range(1, d):
        P = sp.kron(P, sp.csr_matrix(prolongation_1d(Ns[p], qs[p])), format="csr")
    return P


def level_intervals(N, G):
    """N_g for g = 1..G given the finest N = N_G (Sec. 3.2.1: N_g = 2^g);
    N may be per dimension (then a list per level)."""
    if np.ndim(N) == 0:
        return [N >> (G - g) for g in range(1, G + 1)]
    return [[Np >> (G - g) for Np in N] for g in range(1, G + 1)]


def num_levels(N):
    """Levels of the hierarchy for the finest intervals N (per dimension or
    a scalar): every dimension is halved from one level to the next (the
    subdivision of eq. 2.5 applies per dimension) while all N_p are even and
    not all equal to 2; powers of two N give G = log2(N) with N_1 = 2
    (Sec. 3.2.1)."""
    Ns = [int(N)] if np.ndim(N) == 0 else [int(a) for a in N]
    G = 1
    while all(Np % 2 == 0 for Np in Ns) and not all(Np == 2 for Np in Ns):
        Ns = [Np // 2 for Np in Ns]
        G += 1
    return G


def hierarchy(x, y, lo, hi, N, lam, q=3, G=None):
    """Per-level assembled data, finest level G: N_G = N, N_g = N / 2^(G-g)
    (per dimension when N is a list).

    Returns a dict g -> {"N", "A", "b", "Phi", "Lam", "P"} where P is the
    prolongation from level g-1 to g (absent at g = 1).
    """
    if G is None:
        G = num_levels(N) if np.ndim(N) else int(round(math.log2(N)))
    d = np.atleast_2d(x).shape[1]
    levels = {}
    for g, Ng in zip(range(1, G + 1), level_intervals(N, G)):
        A, b, Phi, Lam = system(x, y, lo, hi, Ng, lam, q)
        lev = {"N": Ng, "A": A, "b": b, "Phi": Phi, "Lam": Lam}
        if g > 1:
            Nc = [a // 2 for a in per_dim(Ng, d)]
            lev["P"] = prolongation(d, Nc, q)
        levels[g] = lev
    return levels


def evaluate(alpha, xq, lo, hi, N, q=3):
    """s(x) = sum_k alpha_k phi_k(x) at query points (eq. 2.2)."""
    return phi_matrix(xq, lo, hi, N, q) @ np.asarray(alpha, dtype=np.float64)


def normal_matrix_dense(x, lo, hi, N, lam, q=3):
    """Dense A = Phi'Phi + lam Lambda with Phi'Phi summed cell by cell.

    The points of one knot cell share their (q+1)^d nonzero basis indices, so
    Phi'Phi = sum over cells of B_c' B_c with B_c the dense (points x (q+1)^d)
    block of those rows, added into the rows and columns of the cell's patch
    (the per-cell Gram blocks of the survey's oracle recipe). Same matrix as
    ``system`` (pinned there); practical where K is a few thousand.
    """
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    n, d = x.shape
    J = N + q
    cells, vals = [], []
    for p in range(d):
        c, V = bspline.basis_local(x[:, p], lo[p], hi[p], N, q)
        cells.append(c)
        vals.append(V)
    flat_cell = np.zeros(n, dtype=np.int64)
    for p in range(d):
        flat_cell = flat_cell * N + cells[p]
    A = lambda_dense(d, lo, hi, N, q) * lam
    order = np.argsort(flat_cell, kind="stable")
    bounds = np.flatnonzero(np.diff(flat_cell[order])) + 1
    offsets = list(itertools.product(range(q + 1), repeat=d))
    for grp in np.split(order, bounds):
        if grp.size == 0:
            continue
        i0 = grp[0]
        B = np.ones((grp.size, len(offsets)))
        idx = np.zeros(len(offsets), dtype=np.int64)
        for m, a in enumerate(offsets):
            k = 0
            for p in range(d):
                k = k * J + cells[p][i0] + a[p]
                B[:, m] *= vals[p][grp, a[p]]
            idx[m] = k
        A[np.ix_(idx, idx)] += B.T @ B
    return A
