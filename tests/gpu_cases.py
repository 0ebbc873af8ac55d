"""Shared helpers of the GPU parity tests: seeded cases and oracle references.

Inputs come from paper_1901_00654_amd.workloads (seeded, no method
arithmetic); every expected value comes from the oracle package."""
import itertools
import math

import numpy as np

from oracle import matfree, mg, system
from paper_1901_00654_amd import workloads


def case(recipe, n, N, seed=None):
    """Seeded inputs of a workload recipe at a reduced size."""
    fn = workloads.CONFIGS[recipe]
    w = fn(n=n, N=N) if seed is None else fn(n=n, N=N, seed=seed)
    return w


def uniform_case(d, n, N, lam, seed):
    rng = np.random.default_rng(seed)
    lo = list(np.round(rng.uniform(-1.0, 0.0, d), 3))
    hi = list(np.round(rng.uniform(1.0, 2.0, d), 3))
    x = np.stack([rng.uniform(lo[p], hi[p], n) for p in range(d)], axis=1)
    y = np.sin(2 * np.pi * x.sum(axis=1)) + 0.1 * rng.standard_normal(n)
    return {"name": "u%dd" % d, "d": d, "x": x, "y": y, "lo": lo, "hi": hi, "N": N, "lam": lam}


def assemblable(d, Ng):
    return (Ng + 3) ** d <= 20000 and not (d == 5 and Ng >= 4)


def level_matrix(w, Ng):
    A, b, Phi, Lam = system.system(w["x"], w["y"], w["lo"], w["hi"], Ng, w["lam"])
    return A, b, Phi


def oracle_apply(w, Ng, c):
    if assemblable(w["d"], Ng):
        A, _, _ = level_matrix(w, Ng)
        return A @ c
    return matfree.apply(w["x"], c, w["lo"], w["hi"], Ng, w["lam"])


def lambda_diag(d, lo, hi, N):
    diags = [[np.diag(system.gram_1d(lo[p], hi[p], N, 3, r)) for r in range(3)] for p in range(d)]
    out = np.zeros((N + 3) ** d)
    for r in itertools.product(range(3), repeat=d):
        if sum(r) != 2:
            continue
        v = np.ones(1)
        for p in range(d):
            v = np.kron(v, diags[p][r[p]])
        out += 2.0 / np.prod([math.factorial(q) for q in r]) * v
    return out


def oracle_diag(w, Ng):
    Phi = system.phi_matrix(w["x"], w["lo"], w["hi"], Ng)
    data = np.asarray(Phi.multiply(Phi).sum(axis=0)).ravel()
    return data + w["lam"] * lambda_diag(w["d"], w["lo"], w["hi"], Ng)


class MatFreeOp:
    """A_g as an object with ``@`` and ``diagonal()`` for the oracle's Lanczos."""

    def __init__(self, w, Ng):
        self.w, self.Ng = w, Ng
        self.shape = ((Ng + 3) ** w["d"],) * 2
        self._diag = oracle_diag(w, Ng)

    def __matmul__(self, c):
        return matfree.apply(self.w["x"], c, self.w["lo"], self.w["hi"], self.Ng, self.w["lam"])

    def diagonal(self):
        return self._diag


def oracle_omega(w, Ng, omega_scale=1.8, steps=16):
    if assemblable(w["d"], Ng):
        A, _, _ = level_matrix(w, Ng)
    else:
        A = MatFreeOp(w, Ng)
    return omega_scale / mg.lanczos_rho(A, steps)


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
