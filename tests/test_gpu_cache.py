"""Problems built from the library's device-memory cache: a problem set up
after others were destroyed draws their released blocks, stale contents
included, and must solve as a problem built on fresh memory does (up to the
summation order of the atomics): nothing may rely on memory being zero, and
every counter and accumulator must be cleared where it is used. Solutions
are compared through their fitted values Phi alpha, which the tolerance
fixes whatever kappa(A) is."""
import numpy as np
import pytest

import gpu_cases as gc
from oracle import mg, system
from paper_1901_00654_amd import tsmg

pytestmark = pytest.mark.gpu


def _solve(w, precision):
    S = tsmg.Smoother(w["x"], w["y"], w["N"], w["lam"], lo=w["lo"], hi=w["hi"], tol=1e-10, max_iter=20000,
                      precision=precision)
    try:
        a, status, info = S.solve()
        assert status == tsmg.TS_OK, info
        return a.cpu().numpy().copy(), info
    finally:
        S.close()


@pytest.mark.parametrize("precision", [tsmg.TS_FP64, tsmg.TS_MIXED_FP32_VCYCLE])
def test_rebuilt_problem_matches_first_build(lib, precision):
    w = gc.case("c2", 20011, 16)
    first, i1 = _solve(w, precision)
    # other problems take the cached blocks and leave their data in them
    _solve(gc.uniform_case(3, 5003, 8, 1e-2, 3), precision)
    _solve(gc.uniform_case(3, 40009, 32, 1e-3, 4), precision)
    _solve(gc.case("c3", 8009, 4), precision)
    again, i2 = _solve(w, precision)
    print("iterations", i1["iterations"], i2["iterations"], flush=True)
    # kappa(A) is about 1e11 here: the global atomics' summation order alone
    # moves the iteration count by a few, more so with the FP32 V-cycle
    # (421 against 426 seen); the fitted values below are the real check
    assert abs(i1["iterations"] - i2["iterations"]) <= max(3, 0.03 * i1["iterations"])
    A, b, Phi, _ = system.system(w["x"], w["y"], w["lo"], w["hi"], w["N"], w["lam"])
    ref = mg.solve_direct(A, b)
    fit = np.linalg.norm(Phi @ ref)
    assert np.linalg.norm(Phi @ (again - first)) <= 1e-8 * fit
    assert np.linalg.norm(Phi @ (again - ref)) <= 1e-8 * fit
