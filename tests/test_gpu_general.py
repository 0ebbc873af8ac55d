"""GPU parity of the general form against the oracle: B-spline degree q_p
and knot intervals N_p per dimension (Sec. 2.1), anisotropic and
non-power-of-two grids, the hierarchy halving every dimension while all N_p
are even (Sec. 3.2.1). Every piece of the path on every level - A_g c in FP64
and FP32, Phi'y, diag(A_g), the subdivision transfers of degree q_p
(eq. 2.5), the coarse solve, the V-cycle and the solves, and the fit - is
compared with the oracle's assembled matrices."""
import numpy as np
import pytest

import gpu_cases as gc
from oracle import mg, system
from paper_1901_00654_amd import tsmg

pytestmark = pytest.mark.gpu

# name: (d, N per dimension, q per dimension, n, lambda, seed)
CASES = {
    "q5_d1": (1, [20], [5], 400, 1e-3, 61),
    "aniso_d2": (2, [24, 12], [3, 2], 4001, 1e-3, 62),
    "mixed_d3": (3, [8, 4, 12], [2, 3, 4], 6001, 1e-2, 63),
    "cubic_aniso_d2": (2, [32, 8], [3, 3], 4001, 1e-3, 64),
    "q2_d3": (3, [16, 16, 16], [2, 2, 2], 20011, 1e-2, 65),
    "q4_d2_n6": (2, [6, 6], [4, 4], 3001, 1e-2, 66),
}


def _case(name):
    d, N, q, n, lam, seed = CASES[name]
    rng = np.random.default_rng(seed)
    lo = list(np.round(rng.uniform(-1.0, 0.0, d), 3))
    hi = list(np.round(rng.uniform(1.0, 2.0, d), 3))
    x = np.stack([rng.uniform(lo[p], hi[p], n) for p in range(d)], axis=1)
    x[0] = lo
    x[1] = hi
    y = np.sin(2 * np.pi * x.sum(axis=1)) + 0.1 * rng.standard_normal(n)
    return {"d": d, "N": N, "q": q, "x": x, "y": y, "lo": lo, "hi": hi, "lam": lam}


@pytest.fixture(scope="module", params=list(CASES))
def gen(request, lib):
    w = _case(request.param)
    print("general case", request.param, "N", w["N"], "q", w["q"], "n", len(w["y"]), flush=True)
    S = tsmg.Smoother(w["x"], w["y"], w["N"], w["lam"], lo=w["lo"], hi=w["hi"], degrees=w["q"])
    lev = system.hierarchy(w["x"], w["y"], w["lo"], w["hi"], w["N"], w["lam"], w["q"])
    assert S.G == max(lev)
    yield w, S, lev
    S.close()


def _energy(A, e, ref):
    return float(np.sqrt(abs(e @ (A @ e)) / (ref @ (A @ ref))))


def test_apply_rhs_diag_every_level(gen):
    w, S, lev = gen
    rng = np.random.default_rng(130)
    for g in range(1, S.G + 1):
        A = lev[g]["A"]
        assert S.K(g) == A.shape[0]
        c = rng.standard_normal(S.K(g))
        assert gc.rel(S.apply(g, c).cpu().numpy(), A @ c) < 1e-12, g
        c32 = c.astype(np.float32)
        assert gc.rel(S.apply(g, c32, fp32=True).cpu().numpy(), A @ c32.astype(np.float64)) < 3e-5, g
        assert gc.rel(S.diag(g).cpu().numpy(), A.diagonal()) < 1e-12, g
    assert gc.rel(S.rhs().cpu().numpy(), lev[S.G]["b"]) < 1e-12


def test_transfers_every_level(gen):
    w, S, lev = gen
    rng = np.random.default_rng(131)
    for g in range(2, S.G + 1):
        P = lev[g]["P"]
        e = rng.standard_normal(P.shape[1])
        r = rng.standard_normal(P.shape[0])
        assert gc.rel(S.prolong(g, e).cpu().numpy(), P @ e) < 1e-14, g
        assert gc.rel(S.restrict(g, r).cpu().numpy(), P.T @ r) < 1e-14, g


def test_coarse_solve_backward_error(gen):
    w, S, lev = gen
    A1 = lev[1]["A"].toarray()
    b = np.random.default_rng(132).standard_normal(A1.shape[0])
    x = S.coarse_solve(b).cpu().numpy()
    back = np.linalg.norm(A1 @ x - b) / (np.linalg.norm(A1, 2) * np.linalg.norm(x) + np.linalg.norm(b))
    assert back <= 1e-14


def test_vcycle_and_solves(gen):
    w, S, lev = gen
    M = mg.MG(w["x"], w["y"], w["lo"], w["hi"], w["N"], w["lam"], q=w["q"], levels=lev)
    A, b = lev[S.G]["A"], lev[S.G]["b"]
    r = np.random.default_rng(133).standard_normal(S.K())
    z, zr = S.vcycle(r).cpu().numpy(), M.vcycle(r)
    err = _energy(A, z - zr, zr)
    ref = mg.solve_direct(A, b)
    S.set_options(tol=1e-13, max_iter=5000)
    a, st, info = S.solve()
    a = a.cpu().numpy()
    Phi = lev[S.G]["Phi"]
    e64 = (_energy(A, a - ref, ref), np.linalg.norm(Phi @ (a - ref)) / np.linalg.norm(Phi @ ref))
    S.set_options(tol=1e-11, precision=tsmg.TS_MIXED_FP32_VCYCLE)
    a32, st32, info32 = S.solve()
    a32 = a32.cpu().numpy()
    e32 = (_energy(A, a32 - ref, ref), np.linalg.norm(Phi @ (a32 - ref)) / np.linalg.norm(Phi @ ref))
    _, it_o, _ = mg.pcg(A, b, M.vcycle, tol=1e-8, maxiter=5000)
    S.set_options(tol=1e-8, precision=tsmg.TS_FP64)
    _, st8, info8 = S.solve()
    print("V-cycle energy %.2e; fp64 energy/fitted %.2e %.2e; vcycle32 %.2e %.2e; iterations %d (oracle %d)"
          % (err, *e64, *e32, info8["iterations"], it_o), flush=True)
    assert err <= 1e-9
    assert st == tsmg.TS_OK and max(e64) <= 1e-10
    assert st32 == tsmg.TS_OK and max(e32) <= 1e-6
    assert st8 == tsmg.TS_OK and abs(info8["iterations"] - it_o) <= max(2, 0.03 * it_o)


def test_evaluate(gen):
    w, S, lev = gen
    rng = np.random.default_rng(134)
    alpha = rng.standard_normal(S.K())
    d = w["d"]
    xq = np.stack([rng.uniform(w["lo"][p], w["hi"][p], 501) for p in range(d)], axis=1)
    xq[0], xq[1] = w["lo"], w["hi"]
    yq = S.evaluate(S._dev(alpha, S.torch.float64), xq).cpu().numpy()
    ref = system.evaluate(alpha, xq, w["lo"], w["hi"], w["N"], w["q"])
    assert gc.rel(yq, ref) < 1e-13


def test_general_arguments_are_checked(lib):
    w = _case("aniso_d2")
    with pytest.raises(tsmg.TsmgError) as ei:
        tsmg.Smoother(w["x"], w["y"], w["N"], w["lam"], lo=w["lo"], hi=w["hi"], degrees=[3, 6])
    assert ei.value.status == tsmg.TS_EINVAL
    with pytest.raises(tsmg.TsmgError):
        tsmg.Smoother(w["x"], w["y"], [24, 0], w["lam"], lo=w["lo"], hi=w["hi"])
