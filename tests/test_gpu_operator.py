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
    w, S = prob
    A1, _, _ = gc.level_matrix(w, w["N"] >> (S.G - 1))
    A1 = A1.toarray()
    b = np.random.default_rng(103).standard_normal(S.K(1))
    ref = np.linalg.solve(A1, b)
    x = S.coarse_solve(b).cpu().numpy()
    kappa = np.linalg.cond(A1)
    # two FP64 solvers agree to the conditioning of A_1 (it reaches 1e7 and
    # more for small lambda at d >= 3)
    assert np.linalg.norm(x - ref) <= max(1e-12, 1e-13 * kappa) * np.linalg.norm(ref)
    assert np.linalg.norm(A1 @ x - b) <= 1e-13 * kappa * np.linalg.norm(b)


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
