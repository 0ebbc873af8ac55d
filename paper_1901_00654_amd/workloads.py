"""Seeded synthetic inputs shaped like the smoothing workloads.

This module only draws data: points x (n x d, float64, row-major), responses
y, the box [lo, hi]^d, the number of knot intervals per dimension and the
smoothing weight. It holds none of the method's arithmetic and imports
nothing else from the package, so the GPU tests, the CPU oracle checks and
the benchmark all draw identical inputs from it.

Workloads (all cubic, uniform knots on [0, 1]^d):

- ``c1``  d=2, 32x32 intervals, 10,000 uniform points,
          y = sin(2 pi x1) cos(2 pi x2) + N(0, 0.1^2), lambda = 1e-4.
- ``c2``  d=3, 64^3 intervals, 2,000,000 points from an 8-component Gaussian
          mixture truncated to the unit cube by rejection (clustered, with
          empty cells), y = exp(-|x - 0.5|^2 / 0.05) + 0.3 x1 x2 + N(0, 0.05^2),
          lambda = 1e-5.
- ``c3``  d=4, 32^4 intervals, 10,000,000 uniform points,
          y = sum_k sin(2 pi k x_k) / k + N(0, 0.1^2), lambda = 1e-4.
- ``c4``  d=5, 16^5 (or 8^5) intervals, 16M scrambled Sobol points plus 4M
          points clustered in the corner at the origin,
          y = prod_k (1 + 0.5 cos(pi x_k)) + N(0, 0.1^2), lambda = 1e-3.
- ``paper_sigmoid``  the test data of the paper's Sec. 4 (P = 1..4,
          100,000 uniform points, sigmoid of ||x||^2 / P plus noise).
- ``serving_trace``  a Poisson stream of requests with d in {2,3,4},
          intervals in {16,32,64} (at most 2e6 coefficients), 1e4..1e6
          uniform points, y = sin(2 pi sum_k x_k) + N(0, 0.1^2),
          lambda log-uniform in [1e-6, 1e-2].

Every function takes optional ``n`` / ``N`` overrides so tests can draw the
same recipe at sizes a CPU oracle handles; the recipe (distribution, noise,
lambda) is unchanged by the override.
"""
import math

import numpy as np


def _box(d):
    return [0.0] * d, [1.0] * d


def _pack(name, x, y, N, lam):
    d = x.shape[1]
    lo, hi = _box(d)
    return {"name": name, "d": d, "x": np.ascontiguousarray(x, dtype=np.float64),
            "y": np.ascontiguousarray(y, dtype=np.float64), "lo": lo, "hi": hi,
            "N": int(N), "lam": float(lam)}


def c1(n=10_000, N=32, seed=1):
    rng = np.random.default_rng(seed)
    x = rng.random((n, 2))
    y = np.sin(2 * np.pi * x[:, 0]) * np.cos(2 * np.pi * x[:, 1])
    y = y + 0.1 * rng.standard_normal(n)
    return _pack("c1", x, y, N, 1e-4)


def _gaussian_mixture(rng, n, d, k=8):
    means = rng.uniform(0.15, 0.85, size=(k, d))
    chols = []
    for _ in range(k):
        sig = np.exp(rng.uniform(np.log(0.03), np.log(0.12), size=d))
        Q, R = np.linalg.qr(rng.standard_normal((d, d)))
        Q = Q * np.sign(np.diag(R))
        chols.append(Q * sig)          # cov = Q diag(sig^2) Q'
    out = np.empty((0, d))
    while out.shape[0] < n:
        m = n - out.shape[0]
        comp = rng.integers(0, k, size=2 * m)
        z = rng.standard_normal((2 * m, d))
        pts = means[comp] + np.einsum("nij,nj->ni", np.stack(chols)[comp], z)
        keep = np.all((pts >= 0.0) & (pts <= 1.0), axis=1)
        out = np.concatenate([out, pts[keep]])
    return out[:n]


def c2(n=2_000_000, N=64, seed=2):
    rng = np.random.default_rng(seed)
    x = _gaussian_mixture(rng, n, 3)
    r2 = np.sum((x - 0.5) ** 2, axis=1)
    y = np.exp(-r2 / 0.05) + 0.3 * x[:, 0] * x[:, 1]
    y = y + 0.05 * rng.standard_normal(n)
    return _pack("c2", x, y, N, 1e-5)


def c3(n=10_000_000, N=32, seed=3):
    rng = np.random.default_rng(seed)
    x = rng.random((n, 4))
    y = sum(np.sin(2 * np.pi * k * x[:, k - 1]) / k for k in range(1, 5))
    y = y + 0.1 * rng.standard_normal(n)
    return _pack("c3", x, y, N, 1e-4)


def c4(n=20_000_000, N=16, seed=4):
    from scipy.stats import qmc
    rng = np.random.default_rng(seed)
    n_sobol = (4 * n) // 5
    n_corner = n - n_sobol
    m = max(1, math.ceil(math.log2(max(n_sobol, 1))))
    sob = qmc.Sobol(5, scramble=True, seed=seed).random_base2(m)[:n_sobol]
    corner = np.abs(0.1 * rng.standard_normal((n_corner, 5)))
    bad = np.any(corner > 1.0, axis=1)
    while bad.any():
        corner[bad] = np.abs(0.1 * rng.standard_normal((int(bad.sum()), 5)))
        bad = np.any(corner > 1.0, axis=1)
    x = np.concatenate([sob, corner])
    y = np.prod(1.0 + 0.5 * np.cos(np.pi * x), axis=1)
    y = y + 0.1 * rng.standard_normal(n)
    return _pack("c4", x, y, N, 1e-3)


def paper_sigmoid(P, n=100_000, N=32, lam=0.2, seed=11):
    """The test data of Sec. 4: n uniform points in [0,1]^P and the
    normalised multivariable sigmoid of ||x||^2 / P plus N(0, 0.1^2) noise.
    The printed formula has a pole (a minus sign in the denominator); the
    logistic form 1 / (1 + exp(-16 (||x||^2 / P - 0.5))), which maps into
    [0, 1] as the paper states, is used. The paper gives no lambda; 0.2 is
    where kappa(A) for P = 2, G = 5 meets its Table 3 value."""
    rng = np.random.default_rng(seed)
    x = rng.random((n, P))
    f = 1.0 / (1.0 + np.exp(-16.0 * (np.sum(x * x, axis=1) / P - 0.5)))
    y = f + 0.1 * rng.standard_normal(n)
    return _pack("sigmoid%d" % P, x, y, N, lam)


CONFIGS = {"c1": c1, "c2": c2, "c3": c3, "c4": c4}


def serving_request(i, seed=5, n=None):
    """Request i of the serving trace (its own stream, seed 5000 + i)."""
    rng = np.random.default_rng(1000 * seed + i)
    d = int(rng.integers(2, 5))
    while True:
        N = int(rng.choice([16, 32, 64]))
        if (N + 3) ** d <= 2_000_000:
            break
    if n is None:
        n = int(round(10.0 ** rng.uniform(4.0, 6.0)))
    lam = 10.0 ** rng.uniform(-6.0, -2.0)
    x = rng.random((n, d))
    y = np.sin(2 * np.pi * x.sum(axis=1)) + 0.1 * rng.standard_normal(n)
    req = _pack("req%d" % i, x, y, N, lam)
    req["index"] = i
    return req


def poisson_arrivals(count, rate, seed=5):
    """Arrival times (s) of a Poisson process with the given rate (1/s)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))
