"""V-cycles replayed from a captured HIP graph inside ts_solve (ts_options
vcycle_graph = 1) against the same solves with every kernel launched one by
one (vcycle_graph = 0, the default).

In the reproducible mode (deterministic = 1) both run the same kernels in the
same order on the same data, so the solutions and iteration counts must agree
bit for bit. A solve replays its graph once per iteration, with the program's
own eager kernels (operator apply, inner products, CG step), host reads of
the residual and device synchronisations between the replays, so the final
solution checks every replay. The graph is captured again when the options
it bakes in change, and reused across solves otherwise."""
import numpy as np
import pytest

import gpu_cases as gc
from paper_1901_00654_amd import tsmg

pytestmark = pytest.mark.gpu

CASES = {
    "d2": lambda: gc.uniform_case(2, 3001, 16, 1e-3, 12),
    "c2s": lambda: gc.case("c2", 20011, 8),
    "d3g4": lambda: gc.uniform_case(3, 60013, 16, 1.0, 32),
    "d4g3": lambda: gc.uniform_case(4, 40009, 8, 1.0, 41),
}


def _smoother(w, **opts):
    return tsmg.Smoother(w["x"], w["y"], w["N"], w["lam"], lo=w["lo"], hi=w["hi"], **opts)


def _solve(S, device=False, **opts):
    S.set_options(**opts)
    a, status, info = S.solve()
    assert status == tsmg.TS_OK, info
    return (a if device else a.cpu().numpy()), info


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", [tsmg.TS_FP64, tsmg.TS_MIXED_FP32, tsmg.TS_MIXED_FP32_VCYCLE])
def test_bitwise_same_as_eager(lib, name, precision):
    w = CASES[name]()
    S = _smoother(w, deterministic=1)
    try:
        kw = dict(tol=1e-10, precision=precision, max_iter=20000)
        a1, i1 = _solve(S, vcycle_graph=1, **kw)
        a0, i0 = _solve(S, vcycle_graph=0, **kw)
        a2, i2 = _solve(S, vcycle_graph=1, **kw)   # the graph captured by the first solve, replayed again
        print(name, "precision", precision, "iterations", i1["iterations"], i0["iterations"], i2["iterations"],
              "applies", i1["applies"], i0["applies"], flush=True)
        assert i1["iterations"] == i0["iterations"] == i2["iterations"]
        assert i1["applies"] == i0["applies"] == i2["applies"]
        assert np.array_equal(a1, a0) and np.array_equal(a2, a0)
    finally:
        S.close()


@pytest.mark.parametrize("kw", [dict(nu1=2, nu2=2), dict(smoother=tsmg.TS_SMOOTH_SSOR), dict(nu1=1, nu2=1)])
def test_recaptured_when_the_options_change(lib, kw):
    """A solve with other smoothing counts or smoother after a first solve:
    the graph is captured again and gives the eager result."""
    w = CASES["d3g4"]()
    S = _smoother(w, deterministic=1)
    try:
        _solve(S, tol=1e-10, vcycle_graph=1)
        a1, i1 = _solve(S, vcycle_graph=1, **kw)
        a0, i0 = _solve(S, vcycle_graph=0, **kw)
        print(kw, "iterations", i1["iterations"], i0["iterations"], flush=True)
        assert i1["iterations"] == i0["iterations"]
        assert np.array_equal(a1, a0)
    finally:
        S.close()


def test_default_mode_matches_eager(lib):
    """Without the reproducible mode the point pass sums with atomics, so
    the two agree to rounding: solved to a relative residual of 1e-12,
    iteration counts within 2 % and fitted values within 1e-9."""
    w = CASES["c2s"]()
    S = _smoother(w)
    try:
        a1, i1 = _solve(S, True, tol=1e-12, vcycle_graph=1, max_iter=20000)
        a0, i0 = _solve(S, True, tol=1e-12, vcycle_graph=0, max_iter=20000)
        f1, f0 = S.evaluate(a1, w["x"]).cpu().numpy(), S.evaluate(a0, w["x"]).cpu().numpy()
        print("iterations", i1["iterations"], i0["iterations"], "fitted %.2e" % gc.rel(f1, f0), flush=True)
        assert abs(i1["iterations"] - i0["iterations"]) <= max(1, i0["iterations"] // 50)
        assert gc.rel(f1, f0) <= 1e-9
    finally:
        S.close()


def test_vcycle_graph_checked(lib):
    w = CASES["d2"]()
    S = _smoother(w)
    try:
        with pytest.raises(tsmg.TsmgError) as ei:
            S.set_options(vcycle_graph=2)
        assert ei.value.status == tsmg.TS_EINVAL
    finally:
        S.close()
