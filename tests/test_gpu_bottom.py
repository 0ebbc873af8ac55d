"""The V-cycle below the finest level as one dense operator (ts_options
bottom_max_k): B_g, the map b -> alpha of Alg. 7 from level g down from a zero
start, is assembled at setup by dense products on the matrix cores and then
applied by one matrix-vector product. Checked against the same V-cycle run
level by level (bottom_max_k = -1) on the same data: the two are one linear
map computed in two orders, so they agree to rounding, in the energy norm
of A (applied by the GPU operator, which both problems share). The oracle
comparison of the default path, which takes the dense operator, is in
test_gpu_solve.py. Every size below is ragged against the 64 x 64 tiles of
the products (K_g = 121, 343, 1331, 2401, 67)."""
import numpy as np
import pytest

import gpu_cases as gc
from paper_1901_00654_amd import tsmg

pytestmark = pytest.mark.gpu

# (case, level expected to carry the operator with every coarse level held
# as a stencil)
CASES = {
    "d1": (lambda: gc.uniform_case(1, 701, 64, 1e-3, 1), 5),       # K_5 = 35
    "d2": (lambda: gc.uniform_case(2, 3001, 16, 1e-3, 12), 3),     # K_3 = 121
    "c2s": (lambda: gc.case("c2", 20011, 8), 2),                    # K_2 = 343
    "d3g4": (lambda: gc.uniform_case(3, 60013, 16, 1.0, 32), 3),   # K_3 = 1331
    "d4g3": (lambda: gc.uniform_case(4, 40009, 8, 1.0, 41), 2),    # K_2 = 2401
}


def _smoother(w, **opts):
    return tsmg.Smoother(w["x"], w["y"], w["N"], w["lam"], lo=w["lo"], hi=w["hi"],
                         stencil_mode=tsmg.TS_STENCIL_ALL, **opts)


def _energy_rel(S, e, ref):
    Ae = S.apply(S.G, e).cpu().numpy()
    Ar = S.apply(S.G, ref).cpu().numpy()
    return float(np.sqrt(abs(e @ Ae) / (ref @ Ar)))


@pytest.fixture(scope="module", params=list(CASES))
def pair(request, lib):
    make, gb = CASES[request.param]
    w = make()
    print("case", request.param, "d", w["d"], "N", w["N"], "n", len(w["y"]), flush=True)
    on, off = _smoother(w), _smoother(w, bottom_max_k=-1)
    yield request.param, w, on, off, gb
    on.close()
    off.close()


def test_level_chosen(pair):
    name, w, on, off, gb = pair
    assert on.bottom_level() == gb
    assert off.bottom_level() == 0


@pytest.mark.parametrize("fp32", [False, True])
def test_vcycle_matches_level_by_level(pair, fp32):
    name, w, on, off, gb = pair
    r = np.random.default_rng(120).standard_normal(on.K())
    if fp32:
        r = r.astype(np.float32)
    z1 = on.vcycle(r, fp32=fp32).cpu().numpy().astype(np.float64)
    z0 = off.vcycle(r, fp32=fp32).cpu().numpy().astype(np.float64)
    err = _energy_rel(off, z1 - z0, z0)
    print(name, "fp32" if fp32 else "fp64", "energy-norm difference %.2e, max-norm %.2e" % (err, gc.rel(z1, z0)),
          flush=True)
    # FP64: the bound of the oracle comparison of the V-cycle (the coarse
    # solve's rounding, here in two orders, enters through the coarse space)
    assert err <= (2e-5 if fp32 else 1e-9)


def test_solve_matches_level_by_level(pair):
    """Both solves to a relative residual of 1e-12: the same iteration count
    within 2 % (c2s, with clustered points and lambda = 1e-5, needs several
    hundred, where rounding moves the count) and solutions within 1e-9 in
    the energy norm."""
    name, w, on, off, gb = pair
    res = []
    for S in (on, off):
        S.set_options(tol=1e-12, max_iter=20000)
        a, status, info = S.solve()
        assert status == tsmg.TS_OK, info
        res.append((a.cpu().numpy(), info["iterations"]))
    (a1, i1), (a0, i0) = res
    err = _energy_rel(off, a1 - a0, a0)
    print(name, "iterations", i1, i0, "energy-norm difference %.2e" % err, flush=True)
    assert abs(i1 - i0) <= max(1, i0 // 50)
    assert err <= 1e-9


@pytest.mark.parametrize("nu", [(2, 2), (2, 1), (0, 1), (1, 0), (3, 3)])
def test_other_smoothing_counts(lib, nu):
    """The operator assembled for the nu1, nu2 given to ts_create (nu1 = 0:
    no pre-smoothing; nu1 != nu2: a non-symmetric B_g)."""
    w = CASES["d3g4"][0]()
    on = _smoother(w, nu1=nu[0], nu2=nu[1])
    off = _smoother(w, nu1=nu[0], nu2=nu[1], bottom_max_k=-1)
    try:
        assert on.bottom_level() == 3
        r = np.random.default_rng(121).standard_normal(on.K())
        z1, z0 = on.vcycle(r).cpu().numpy(), off.vcycle(r).cpu().numpy()
        err = _energy_rel(off, z1 - z0, z0)
        print("nu", nu, "energy-norm difference %.2e" % err, flush=True)
        assert err <= 1e-9
    finally:
        on.close()
        off.close()


def test_cap_and_coarsest_level(lib):
    w = CASES["d3g4"][0]()
    S = _smoother(w, bottom_max_k=343)
    try:
        assert S.bottom_level() == 2
    finally:
        S.close()
    on = _smoother(w, coarsest_level=2)
    off = _smoother(w, coarsest_level=2, bottom_max_k=-1)
    try:
        assert on.bottom_level() == 3
        r = np.random.default_rng(122).standard_normal(on.K())
        z1, z0 = on.vcycle(r).cpu().numpy(), off.vcycle(r).cpu().numpy()
        assert _energy_rel(off, z1 - z0, z0) <= 1e-9
    finally:
        on.close()
        off.close()


def test_falls_back_when_the_options_change(lib):
    """Smoothing counts or a smoother other than those the operator was
    assembled for: every level runs its own steps again."""
    w = CASES["d3g4"][0]()
    on, off = _smoother(w), _smoother(w, bottom_max_k=-1)
    try:
        r = np.random.default_rng(123).standard_normal(on.K())
        for kw in (dict(nu1=2, nu2=2), dict(nu1=1, nu2=1, smoother=tsmg.TS_SMOOTH_SSOR)):
            on.set_options(**kw)
            off.set_options(**kw)
            assert on.bottom_level() == 0
            z1, z0 = on.vcycle(r).cpu().numpy(), off.vcycle(r).cpu().numpy()
            assert _energy_rel(off, z1 - z0, z0) <= 1e-11
        on.set_options(nu1=1, nu2=1, smoother=tsmg.TS_SMOOTH_JACOBI)
        assert on.bottom_level() == 3
    finally:
        on.close()
        off.close()


def test_not_built_where_it_cannot_apply(lib):
    w = CASES["d3g4"][0]()
    for kw in (dict(stencil_mode=tsmg.TS_STENCIL_NONE), dict(coarse_solver=tsmg.TS_COARSE_CG),
               dict(smoother=tsmg.TS_SMOOTH_SSOR)):
        opts = dict(stencil_mode=tsmg.TS_STENCIL_ALL)
        opts.update(kw)
        S = tsmg.Smoother(w["x"], w["y"], w["N"], w["lam"], lo=w["lo"], hi=w["hi"], **opts)
        try:
            assert S.bottom_level() == 0, kw
        finally:
            S.close()


GENERAL = {
    # (d, intervals, degrees, n, lambda, seed), level expected to carry the operator
    "gen_d2": ((2, [40, 24], [2, 4], 20011, 1e-3, 71), 3),    # (20, 12) at level 3: K = 22 x 16 = 352
    "gen_d3": ((3, [24, 24, 24], [2, 2, 2], 60013, 1e-2, 72), 3),   # N = 12: K = 14^3 = 2744
    "gen_mixed_d3": ((3, [8, 4, 12], [2, 3, 4], 6001, 1e-2, 73), 2),  # (4, 2, 6): K = 6 x 5 x 10 = 300
}


def _general(name):
    (d, N, q, n, lam, seed), gb = GENERAL[name]
    w = gc.uniform_case(d, n, N[0], lam, seed)
    w["N"] = N
    w["q"] = q
    return w, gb


@pytest.mark.parametrize("name", list(GENERAL))
def test_general_form(lib, name):
    """The general form (degree and intervals per dimension): A_g assembled
    densely from the points, I_g from the subdivision passes run over a
    batch of coarse unit vectors."""
    w, gb = _general(name)
    make = lambda **kw: tsmg.Smoother(w["x"], w["y"], w["N"], w["lam"], lo=w["lo"], hi=w["hi"], degrees=w["q"], **kw)
    on, off = make(), make(bottom_max_k=-1)
    try:
        assert on.bottom_level() == gb and off.bottom_level() == 0
        r = np.random.default_rng(124).standard_normal(on.K())
        z1, z0 = on.vcycle(r).cpu().numpy(), off.vcycle(r).cpu().numpy()
        err = _energy_rel(off, z1 - z0, z0)
        res = []
        for S in (on, off):
            S.set_options(tol=1e-12, max_iter=20000)
            a, status, info = S.solve()
            assert status == tsmg.TS_OK, info
            res.append((a.cpu().numpy(), info["iterations"]))
        (a1, i1), (a0, i0) = res
        serr = _energy_rel(off, a1 - a0, a0)
        print(name, "V-cycle energy-norm difference %.2e" % err, "iterations", i1, i0,
              "solution difference %.2e" % serr, flush=True)
        assert err <= 1e-9
        assert abs(i1 - i0) <= max(1, i0 // 50)
        assert serr <= 1e-9
    finally:
        on.close()
        off.close()
