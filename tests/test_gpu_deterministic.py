"""The reproducible mode (ts_options.deterministic): the point pass without
atomics (fixed-order sums of each round's items in LDS, patches stored per
chunk and added per coefficient in a fixed order) and one block per cell in
the setup's moment sums. Checked against the oracle on every level, for bit
equality between runs of the same problem, and against the default mode."""
import numpy as np
import pytest

import gpu_cases as gc
from oracle import matfree
from paper_1901_00654_amd import tsmg

pytestmark = pytest.mark.gpu

CASES = {
    "d1": lambda: gc.uniform_case(1, 701, 16, 1e-3, 1),
    "d2": lambda: gc.uniform_case(2, 3001, 16, 1e-4, 2),
    "c2s": lambda: gc.case("c2", 20011, 8),
    "c3s": lambda: gc.case("c3", 8009, 4),
    "c4s": lambda: gc.case("c4", 6007, 4),
    "d5g2": lambda: gc.uniform_case(5, 20011, 4, 1.0, 51),
}


def _smoother(w, **opts):
    return tsmg.Smoother(w["x"], w["y"], w["N"], w["lam"], lo=w["lo"], hi=w["hi"], deterministic=1, **opts)


@pytest.mark.parametrize("name", ["d1", "d2", "c2s", "c3s", "c4s"])
@pytest.mark.parametrize("mode", [tsmg.TS_STENCIL_AUTO, tsmg.TS_STENCIL_NONE])
def test_pieces_match_oracle(lib, name, mode):
    """Phi'y, diag(A_g) and A_g c (FP64 and FP32) on every level."""
    w = CASES[name]()
    print("case", name, "d", w["d"], "N", w["N"], "n", len(w["y"]), "stencil mode", mode, flush=True)
    S = _smoother(w, stencil_mode=mode)
    try:
        b = S.rhs().cpu().numpy()
        assert gc.rel(b, matfree.rhs(w["x"], w["y"], w["lo"], w["hi"], w["N"])) < 1e-12
        rng = np.random.default_rng(400)
        for g in range(1, S.G + 1):
            Ng = w["N"] >> (S.G - g)
            assert gc.rel(S.diag(g).cpu().numpy(), gc.oracle_diag(w, Ng)) < 1e-12, g
            c = rng.standard_normal(S.K(g))
            assert gc.rel(S.apply(g, c).cpu().numpy(), gc.oracle_apply(w, Ng, c)) < 1e-12, g
            c32 = c.astype(np.float32)
            ref32 = gc.oracle_apply(w, Ng, c32.astype(np.float64))
            assert gc.rel(S.apply(g, c32, fp32=True).cpu().numpy(), ref32) < 3e-5, g
    finally:
        S.close()


def _solve(w, precision, deterministic=1):
    S = tsmg.Smoother(w["x"], w["y"], w["N"], w["lam"], lo=w["lo"], hi=w["hi"], deterministic=deterministic)
    try:
        S.set_options(tol=1e-10, precision=precision, max_iter=20000)
        a, status, info = S.solve()
        assert status == tsmg.TS_OK, info
        rng = np.random.default_rng(401)
        c = rng.standard_normal(S.K())
        return a.cpu().numpy(), S.apply(S.G, c).cpu().numpy(), info
    finally:
        S.close()


@pytest.mark.parametrize("name", ["c2s", "c3s", "d5g2"])
@pytest.mark.parametrize("precision", [tsmg.TS_FP64, tsmg.TS_MIXED_FP32, tsmg.TS_MIXED_FP32_VCYCLE])
def test_bitwise_repeatable(lib, name, precision):
    """Two problems built from the same data give the same bits: the
    operator apply, the iteration count and the solution."""
    w = CASES[name]()
    a1, v1, i1 = _solve(w, precision)
    a2, v2, i2 = _solve(w, precision)
    print(name, "precision", precision, "iterations", i1["iterations"], i2["iterations"], flush=True)
    assert np.array_equal(v1, v2)
    assert i1["iterations"] == i2["iterations"] and i1["refinements"] == i2["refinements"]
    assert np.array_equal(a1, a2)


@pytest.mark.parametrize("name", ["c2s", "c3s", "d5g2"])
def test_solves_the_same_system(lib, name):
    """The reproducible solution meets the tolerance against the default
    mode's operator and right-hand side (b - A alpha recomputed there)."""
    w = CASES[name]()
    a_det, _, info = _solve(w, tsmg.TS_FP64)
    S = tsmg.Smoother(w["x"], w["y"], w["N"], w["lam"], lo=w["lo"], hi=w["hi"])
    try:
        b = S.rhs().cpu().numpy()
        r = b - S.apply(S.G, a_det).cpu().numpy()
    finally:
        S.close()
    rel = np.linalg.norm(r) / np.linalg.norm(b)
    print(name, "iterations", info["iterations"], "residual in the default mode %.2e" % rel, flush=True)
    assert rel <= 2e-10


def test_rejects_the_general_form(lib):
    w = gc.uniform_case(2, 501, 8, 1e-3, 9)
    with pytest.raises(tsmg.TsmgError) as ei:
        tsmg.Smoother(w["x"], w["y"], [8, 4], w["lam"], lo=w["lo"], hi=w["hi"], deterministic=1)
    assert ei.value.status == tsmg.TS_EINVAL
    with pytest.raises(tsmg.TsmgError):
        tsmg.Smoother(w["x"], w["y"], 8, w["lam"], lo=w["lo"], hi=w["hi"], deterministic=2)
