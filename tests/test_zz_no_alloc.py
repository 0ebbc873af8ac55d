"""ts_solve_noalloc (the solve that allocates no device memory, in the
library's static scratch) against the existing entry points ts_create +
ts_solve on the same inputs: two calls in a row, the second smaller, each to
the FP64 bar (energy norm and fitted values within 1e-10 of the allocating
solve), and a problem larger than the scratch refused before any work."""
import numpy as np
import pytest
import torch

import gpu_cases as gc
from oracle import system
from paper_1901_00654_amd import tsmg

pytestmark = pytest.mark.gpu


def _noalloc(w, tol):
    d, n = w["d"], len(w["y"])
    o = tsmg.ts_default_options()
    o.tol = tol
    o.max_iter = 5000
    x = torch.as_tensor(w["x"]).cuda().contiguous()
    y = torch.as_tensor(w["y"]).cuda().contiguous()
    alpha = torch.full(((w["N"] + 3) ** d,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    status, info = tsmg.ts_solve_noalloc(d, 3, [w["N"]] * d, w["lo"], w["hi"], n, x, y, w["lam"], alpha, o)
    torch.cuda.synchronize()
    return alpha.cpu().numpy(), status, info.as_dict()


def _allocating(w, tol):
    S = tsmg.Smoother(w["x"], w["y"], w["N"], w["lam"], lo=w["lo"], hi=w["hi"], tol=tol, max_iter=5000)
    try:
        a, status, info = S.solve()
        return a.cpu().numpy(), status, info
    finally:
        S.close()


def test_noalloc_matches_allocating_solve_twice(lib):
    cases = [gc.uniform_case(3, 60013, 16, 1e-1, 32), gc.uniform_case(2, 3001, 16, 1e-3, 12)]
    for w in cases:
        print("no-alloc case d", w["d"], "N", w["N"], "n", len(w["y"]), flush=True)
        a0, s0, i0 = _noalloc(w, 1e-12)
        a1, s1, i1 = _allocating(w, 1e-12)
        assert s0 == tsmg.TS_OK and s1 == tsmg.TS_OK, (i0, i1)
        assert np.all(np.isfinite(a0))
        A, b, Phi, _ = system.system(w["x"], w["y"], w["lo"], w["hi"], w["N"], w["lam"])
        e = a0 - a1
        energy = np.sqrt(abs(e @ (A @ e)) / (a1 @ (A @ a1)))
        fitted = np.linalg.norm(Phi @ e) / np.linalg.norm(Phi @ a1)
        print("iterations %d vs %d, energy %.2e, fitted %.2e, history %d"
              % (i0["iterations"], i1["iterations"], energy, fitted, len(i0["residual_history"])), flush=True)
        assert energy <= 1e-10 and fitted <= 1e-10
        assert abs(i0["iterations"] - i1["iterations"]) <= 1
        assert len(i0["residual_history"]) == i0["iterations"] + 1 + i0["refinements"]


def test_noalloc_refuses_a_problem_beyond_the_scratch(lib):
    n, d, N = 200_000, 3, 64
    x = torch.rand((n, d), dtype=torch.float64, device="cuda")
    y = torch.rand(n, dtype=torch.float64, device="cuda")
    alpha = torch.empty((N + 3) ** d, dtype=torch.float64, device="cuda")
    with pytest.raises(tsmg.TsmgError) as ei:
        tsmg.ts_solve_noalloc(d, 3, [N] * d, [0.0] * d, [1.0] * d, n, x, y, 1e-3, alpha)
    assert ei.value.status == tsmg.TS_EINVAL
    assert "scratch" in str(ei.value)
