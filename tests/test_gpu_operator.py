"""GPU parity of the operator pieces through the C ABI against the oracle:
A_g c on every level (FP64 and FP32), Phi'y, diag(A_g), omega_g, the grid
transfer, the coarse solve and the evaluation of a fit."""
import numpy as np
import pytest

import gpu_cases as gc
from oracle import matfree, system
from paper_1901_00654_amd import tsmg

pytestmark = pytest.mark.gpu

CASES = {
    "d1": lambda: gc.uniform_case(1, 701, 16, 1e-3, 1),
    "c1": lambda: gc.case("c1", 10000, 32),
    "d2": lambda: gc.uniform_case(2, 3001, 16, 1e-4, 2),
    "c2s": lambda: gc.case("c2", 20011, 8),
    "d3": lambda: gc.uniform_case(3, 5003, 8, 1e-2, 3),
    "c3s": lambda: gc.case("c3", 8009, 4),
    "c4s": lambda: gc.case("c4", 6007, 4),
    "d5": lambda: gc.uniform_case(5, 2503, 2, 1e-3, 5),
}


@pytest.fixture(scope="module", params=list(CASES))
def prob(request, lib):
    w = CASES[request.param]()
    print("case", request.param, "d", w["d"], "N", w["N"], "n", len(w["y"]), flush=True)
    S = tsmg.Smoother(w["x"], w["y"], w["N"], w["lam"], lo=w["lo"], hi=w["hi"])
    yield w, S
    S.close()


def levels(S):
    return range(1, S.G + 1)


def test_apply_fp64_every_level(prob):
    w, S = prob
    rng = np.random.default_rng(100)
    for g in levels(S):
        Ng = w["N"] >> (S.G - g)
        c = rng.standard_normal(S.K(g))
        out = S.apply(g, c).cpu().numpy()
        assert gc.rel(out, gc.oracle_apply(w, Ng, c)) < 1e-12, g


@pytest.mark.parametrize("mode", [tsmg.TS_STENCIL_NONE, tsmg.TS_STENCIL_ALL])
def test_apply_every_level_matrix_free_and_stencil(prob, mode):
    """Both ways of applying A_g (point pass + Lambda passes, or the stencil
    assembled at setup) against the oracle on every level, FP64 and FP32."""
    w, _ = prob
    S = tsmg.Smoother(w["x"], w["y"], w["N"], w["lam"], lo=w["lo"], hi=w["hi"], stencil_mode=mode)
    try:
        rng = np.random.default_rng(105)
        for g in levels(S):
            Ng = w["N"] >> (S.G - g)
            c = rng.standard_normal(S.K(g))
            ref = gc.oracle_apply(w, Ng, c)
            assert gc.rel(S.apply(g, c).cpu().numpy(), ref) < 1e-12, (mode, g)
            c32 = c.astype(np.float32)
            ref32 = gc.oracle_apply(w, Ng, c32.astype(np.float64))
            assert gc.rel(S.apply(g, c32, fp32=True).cpu().numpy(), ref32) < 3e-5, (mode, g)
    finally:
        S.close()


@pytest.mark.parametrize("d,N", [(3, 16), (3, 32), (4, 16), (5, 8)])
def test_apply_lambda_dominated(lib, d, N):
    """lambda so large that lambda*Lambda dominates A_g: the fused Lambda
    kernel's column tiles, halos and runs of planes (J = 11, 19 and 35 span
    several of each, with ragged last ones), at d >= 4 after the banded
    passes over the leading dimensions, against the oracle on every level,
    FP64 and FP32."""
    w = gc.uniform_case(d, 3001 if d == 3 else 2003, N, 1e3, 7 if d == 3 else 8 + d)
    S = tsmg.Smoother(w["x"], w["y"], w["N"], w["lam"], lo=w["lo"], hi=w["hi"], stencil_mode=tsmg.TS_STENCIL_NONE)
    try:
        rng = np.random.default_rng(106)
        for g in levels(S):
            Ng = w["N"] >> (S.G - g)
            c = rng.standard_normal(S.K(g))
            ref = gc.oracle_apply(w, Ng, c)
            assert gc.rel(S.apply(g, c).cpu().numpy(), ref) < 1e-12, g
            c32 = c.astype(np.float32)
            ref32 = gc.oracle_apply(w, Ng, c32.astype(np.float64))
            assert gc.rel(S.apply(g, c32, fp32=True).cpu().numpy(), ref32) < 3e-5, g
    finally:
        S.close()


def test_apply_fp32_finest_and_coarsest(prob):
    w, S = prob
    rng = np.random.default_rng(101)
    for g in sorted({1, S.G}):
        Ng = w["N"] >> (S.G - g)
        c = rng.standard_normal(S.K(g)).astype(np.float32)
        out = S.apply(g, c, fp32=True).cpu().numpy()
        assert gc.rel(out, gc.oracle_apply(w, Ng, c.astype(np.float64))) < 3e-5, g


def test_rhs(prob):
    w, S = prob
    b = S.rhs().cpu().numpy()
    ref = matfree.rhs(w["x"], w["y"], w["lo"], w["hi"], w["N"])
    assert gc.rel(b, ref) < 1e-12


def test_diag_every_level(prob):
    w, S = prob
    for g in levels(S):
        Ng = w["N"] >> (S.G - g)
        assert gc.rel(S.diag(g).cpu().numpy(), gc.oracle_diag(w, Ng)) < 1e-12, g


def test_omega_every_level(prob):
    w, S = prob
    assert S.omega(1) == 0.0
    for g in range(2, S.G + 1):
        Ng = w["N"] >> (S.G - g)
        ref = gc.oracle_omega(w, Ng)
        assert abs(S.omega(g) - ref) < 1e-9 * ref, g


def test_transfer_every_level(prob):
    w, S = prob
    rng = np.random.default_rng(102)
    for g in range(2, S.G + 1):
        Nc = w["N"] >> (S.G - g + 1)
        P = system.prolongation(w["d"], Nc)
        e = rng.standard_normal(S.K(g - 1))
        assert gc.rel(S.prolong(g, e).cpu().numpy(), P @ e) < 1e-14
        r = rng.standard_normal(S.K(g))
        assert gc.rel(S.restrict(g, r).cpu().numpy(), P.T @ r) < 1e-14


def test_coarse_solve(prob):
    """Sec. 3.2.4. Two FP64 solves of A_1 x = b agree only to about
    kappa(A_1) eps, and kappa(A_1) reaches 1e16 here at d = 5 (the five
    B-splines of a two-interval grid are nearly dependent on the box). The
    check is the normwise backward error, which a backward-stable FP64
    solver keeps near eps whatever the conditioning; the forward differences
    are printed."""
    w, S = prob
    A1, _, _ = gc.level_matrix(w, w["N"] >> (S.G - 1))
    A1 = A1.toarray()
    b = np.random.default_rng(103).standard_normal(S.K(1))
    ref = np.linalg.solve(A1, b)
    x = S.coarse_solve(b).cpu().numpy()
    back = np.linalg.norm(A1 @ x - b) / (np.linalg.norm(A1, 2) * np.linalg.norm(x) + np.linalg.norm(b))
    e = x - ref
    energy = np.sqrt(abs(e @ A1 @ e) / (ref @ A1 @ ref))
    print("coarse solve: backward error %.2e, energy-norm difference %.2e, kappa(A_1) %.1e"
          % (back, energy, np.linalg.cond(A1)), flush=True)
    assert back <= 1e-14


def test_evaluate(prob):
    w, S = prob
    rng = np.random.default_rng(104)
    d = w["d"]
    alpha = rng.standard_normal(S.K())
    xq = np.stack([rng.uniform(w["lo"][p], w["hi"][p], 997) for p in range(d)], axis=1)
    xq[0], xq[1] = w["lo"], w["hi"]
    import torch
    yq = S.evaluate(torch.as_tensor(alpha).cuda(), xq).cpu().numpy()
    ref = system.evaluate(alpha, xq, w["lo"], w["hi"], w["N"])
    assert gc.rel(yq, ref) < 1e-13


def _on_knots_case(d, N, n, seed):
    """Uniform points with a third of the coordinates moved exactly onto knots
    lo + j h (j = 0..N, so also onto hi), where the cell index switches."""
    w = gc.uniform_case(d, n, N, 1e-2, seed)
    rng = np.random.default_rng(seed + 100)
    x = w["x"].copy()
    for p in range(d):
        pick = rng.random(n) < 1.0 / 3.0
        j = rng.integers(0, N + 1, size=n)
        h = (w["hi"][p] - w["lo"][p]) / N
        knots = np.where(j == N, w["hi"][p], w["lo"][p] + j * h)
        x[pick, p] = knots[pick]
    w["x"] = x
    return w


@pytest.mark.parametrize("d,N", [(2, 16), (3, 8), (5, 4)])
def test_apply_points_on_knots_and_hi(lib, d, N):
    """Points exactly on interior knots and on the upper bound hi (reading
    R12: cell = min(floor((x - lo) / h), N - 1)) on every level: A_g c, Phi'y,
    diag(A_g) and the fit at those points, against the oracle."""
    w = _on_knots_case(d, N, 3001 if d < 5 else 4001, 40 + d)
    assert np.any(w["x"] == np.asarray(w["hi"])[None, :])
    S = tsmg.Smoother(w["x"], w["y"], w["N"], w["lam"], lo=w["lo"], hi=w["hi"])
    try:
        rng = np.random.default_rng(107)
        for g in levels(S):
            Ng = w["N"] >> (S.G - g)
            c = rng.standard_normal(S.K(g))
            assert gc.rel(S.apply(g, c).cpu().numpy(), gc.oracle_apply(w, Ng, c)) < 1e-12, g
            assert gc.rel(S.diag(g).cpu().numpy(), gc.oracle_diag(w, Ng)) < 1e-12, g
        b = matfree.rhs(w["x"], w["y"], w["lo"], w["hi"], w["N"])
        assert gc.rel(S.rhs().cpu().numpy(), b) < 1e-12
        alpha = rng.standard_normal(S.K())
        yq = S.evaluate(S._dev(alpha, S.torch.float64), w["x"]).cpu().numpy()
        ref = matfree.evaluate(alpha, w["x"], w["lo"], w["hi"], w["N"])
        assert gc.rel(yq, ref) < 1e-13
    finally:
        S.close()


@pytest.mark.parametrize("recipe,n,N", [("c3", 60013, 8), ("c4", 40009, 4)])
def test_apply_fullsize_layout(lib, recipe, n, N):
    """The work split the full workloads take: 512 points per workgroup with
    the packed work lists of d >= 4, and for the c4 recipe the corner cluster
    (most of 8,000 points in one cell of N = 4), whose tile is cut into
    several chunks. Every entry of A_G c, Phi'y and diag(A_G) is compared."""
    w = gc.case(recipe, n, N)
    S = tsmg.Smoother(w["x"], w["y"], w["N"], w["lam"], lo=w["lo"], hi=w["hi"], points_per_block=512,
                      stencil_mode=tsmg.TS_STENCIL_NONE)
    try:
        op = matfree.LevelOperator(w["x"], w["lo"], w["hi"], w["N"], w["lam"])
        rng = np.random.default_rng(108)
        c = rng.standard_normal(S.K())
        assert gc.rel(S.apply(S.G, c).cpu().numpy(), op @ c) < 1e-12
        c32 = c.astype(np.float32)
        assert gc.rel(S.apply(S.G, c32, fp32=True).cpu().numpy(), op @ c32.astype(np.float64)) < 3e-5
        assert gc.rel(S.rhs().cpu().numpy(), op.PhiT @ w["y"]) < 1e-12
        assert gc.rel(S.diag(S.G).cpu().numpy(), op.diagonal()) < 1e-12
    finally:
        S.close()
