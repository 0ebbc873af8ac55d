"""Univariate B-splines on uniform extended knots (test oracle, FP64).

Follows Sec. 2.1 of arXiv:1901.00654: the spline space of degree q on the
knots a = k_0 < ... < k_{m+1} = b has dimension J = m + q + 1 and the
B-spline basis phi_{j,q} of de Boor. The paper does not spell out the knot
vector at the ends; the reading taken here is the uniform *extended*
(non-clamped) knot vector t_j = lo + (j - q) h, j = 0 .. N + 2q, with
N = m + 1 intervals of width h = (hi - lo) / N. That is the only choice under
which the subdivision formula (eq. 2.5) holds for every basis function and
J = N + q, K_g = (2^g + q)^P (Sec. 3.2.1) come out as printed.

Basis values come from the Cox-de Boor recursion
    B_{j,0} = 1 on [t_j, t_{j+1}),
    B_{j,k}(x) = (x - t_j) / (t_{j+k} - t_j) B_{j,k-1}(x)
               + (t_{j+k+1} - x) / (t_{j+k+1} - t_{j+1}) B_{j+1,k-1}(x),
restricted to the q+1 functions that do not vanish on the cell of x, and
derivatives from the standard derivative recursion
    D B_{j,k} = k [ B_{j,k-1} / (t_{j+k} - t_j) - B_{j+1,k-1} / (t_{j+k+1} - t_{j+1}) ].

Pinned (tests/test_oracle_basis.py) against: partition of unity, the closed
form of the uniform cubic pieces, the truncated-power formula of the cardinal
B-spline, and reproduction of affine functions from Greville abscissae.
"""
import numpy as np


def uniform_knots(lo, hi, N, q):
    """Extended uniform knot vector t_j = lo + (j - q) h, j = 0..N+2q."""
    h = (hi - lo) / N
    return lo + (np.arange(N + 2 * q + 1, dtype=np.float64) - q) * h


def cell_index(x, lo, hi, N):
    """Knot interval of each x: c = min(floor((x - lo) / h), N - 1).

    A point on an interior knot belongs to the interval on its right; the
    right end point hi belongs to the last interval (the basis is continuous
    there for q >= 1, so either side gives the same values).
    """
    x = np.asarray(x, dtype=np.float64)
    h = (hi - lo) / N
    c = np.floor((x - lo) / h).astype(np.int64)
    return np.clip(c, 0, N - 1)


def _raise_degree(vals, k, x, c, t, q, derivative):
    """From the degree-(k-1) functions alive on cell c to degree k.

    ``vals[:, m]`` holds B_{j,k-1} for j = c + q - (k-1) + m, m = 0..k-1.
    Returns an (n, k+1) array holding, for j = c + q - k + m, either
    B_{j,k}(x) (Cox-de Boor) or k * [F_{j,k-1}/(t_{j+k}-t_j)
    - F_{j+1,k-1}/(t_{j+k+1}-t_{j+1})] when ``derivative`` is set, where F is
    whatever ``vals`` holds (values or lower derivatives).
    """
    n = x.shape[0]
    out = np.zeros((n, k + 1))
    for m in range(k + 1):
        j = c + q - k + m
        # B_{j,k-1} sits at old column m-1, B_{j+1,k-1} at old column m.
        if m - 1 >= 0:
            den = t[j + k] - t[j]
            if derivative:
                out[:, m] += k * vals[:, m - 1] / den
            else:
                out[:, m] += (x - t[j]) / den * vals[:, m - 1]
        if m <= k - 1:
            den = t[j + k + 1] - t[j + 1]
            if derivative:
                out[:, m] -= k * vals[:, m] / den
            else:
                out[:, m] += (t[j + k + 1] - x) / den * vals[:, m]
    return out


def basis_local(x, lo, hi, N, q, r=0):
    """r-th derivative of the q+1 B-splines alive at each x.

    Returns ``(c, V)`` with ``c`` the cell index of every point and
    ``V[i, a] = D^r B_{c_i + a, q}(x_i)`` for a = 0..q (basis indices are
    0-based, j = 0..N+q-1).
    """
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    t = uniform_knots(lo, hi, N, q)
    c = cell_index(x, lo, hi, N)
    vals = np.ones((x.shape[0], 1))
    for k in range(1, q - r + 1):
        vals = _raise_degree(vals, k, x, c, t, q, derivative=False)
    for k in range(q - r + 1, q + 1):
        vals = _raise_degree(vals, k, x, c, t, q, derivative=True)
    return c, vals


def basis_dense(x, lo, hi, N, q, r=0):
    """Dense (n, J) matrix of D^r B_{j,q}(x_i), J = N + q (Phi_p of Sec. 2.4)."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    c, V = basis_local(x, lo, hi, N, q, r)
    out = np.zeros((x.shape[0], N + q))
    rows = np.arange(x.shape[0])
    for a in range(q + 1):
        out[rows, c + a] = V[:, a]
    return out


def greville(lo, hi, N, q):
    """Greville abscissae xi_j = (t_{j+1} + ... + t_{j+q}) / q.

    sum_j xi_j B_{j,q}(x) = x on [lo, hi] (affine reproduction).
    """
    t = uniform_knots(lo, hi, N, q)
    J = N + q
    return np.array([t[j + 1:j + q + 1].mean() for j in range(J)])
