#!/usr/bin/env python3
"""Benchmark of the matrix-free multigrid-preconditioned spline smoother.

One step = the whole hot path on the d=3 clustered workload (64^3 knot
intervals, 300,763 coefficients, 2,000,000 points from a Gaussian mixture,
lambda = 1e-5) with the points already resident on the GPU: problem setup
(binning and sort, Jacobi diagonals, Lanczos damping, coarse assembly and
inversion), MGCG to a relative FP64 residual of 1e-8, and evaluation of the
fit at every data point.

Prints one JSON line: solves/s (value), the roofline of the dominant kernel
(the point pass of the finest-level operator apply, timed with HIP events on
its stream inside the library), the operator-apply rate for d = 2..5 at the
full workload sizes, the other precision mode for comparison, and the CPU
oracle timed on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64|mixed]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "PCG time-to-1e-8 residual + operator-apply GB/s (d=2–5); served solves/s, p99"
PEAK_FP64_VALU_TFLOPS = 78.6     # 256 CUs x 2.4 GHz x 64 lanes x 2 (FMA)
PEAK_HBM_GBPS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_data_c2.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1901_00654_amd", "csrc", "kernels.hip")


SERVE_PRECISION = {"mixed": lambda t: t.TS_MIXED_FP32, "vcycle32": lambda t: t.TS_MIXED_FP32_VCYCLE}
PRECISIONS_BY_CODE = {0: "fp64", 1: "mixed (FP32 CG, reliable FP64 updates)",
                      3: "vcycle32 (FP64 CG, FP32 V-cycle)"}


def algorithmic(d, n, K, fp32, q=3):
    """FLOP and bytes one point pass must spend: per point the d*4 cubic values
    (15 d FLOP), the tensor product (4^d), gather (2 * 4^d) and scatter
    (2 * 4^d) - with (q+1)^d in place of 4^d for degree q; per point its d
    cell coordinates and cell index; per coefficient one read of c and one
    write of the output."""
    s = 4 if fp32 else 8
    flops = n * (5 * (q + 1) ** d + 15 * d)
    nbytes = n * (d * s + 4) + 2 * K * s
    return flops, nbytes


def source_hash():
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_bytes():
    """HBM bytes per launch of the point pass from the committed rocprofv3
    counter summary, or None if absent or taken on another kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    try:
        t = json.load(open(TRAFFIC_FILE))
    except ValueError:
        return None
    if t.get("kernel_source_sha256_16") != source_hash():
        return None
    return t.get("hbm_bytes_per_launch")


SMOOTHER = {}   # nu, omega_scale overrides from the command line


def set_smoother(opt):
    if "ppb" in SMOOTHER:
        opt.points_per_block = SMOOTHER["ppb"]
    if "nu" in SMOOTHER:
        opt.nu1 = opt.nu2 = SMOOTHER["nu"]
    if "omega_scale" in SMOOTHER:
        opt.omega_scale = SMOOTHER["omega_scale"]
    return opt


def make_problem(tsmg, w, xd, yd, stream, precision, tol=1e-8):
    opt = tsmg.ts_default_options()
    opt.stream = stream.cuda_stream
    opt.tol = tol
    opt.precision = precision
    opt.max_iter = 100000
    set_smoother(opt)
    d = w["d"]
    return tsmg.ts_create(d, SMOOTHER.get("degree", 3), [w["N"]] * d, w["lo"], w["hi"], len(w["y"]), xd, yd,
                          w["lam"], opt)


def run_steps(tsmg, torch, w, xd, yd, stream, precision, steps, warmup):
    K = (w["N"] + 3) ** w["d"]
    n = len(w["y"])
    alpha = torch.empty(K, dtype=torch.float64, device="cuda")
    yq = torch.empty(n, dtype=torch.float64, device="cuda")
    infos = []

    def step():
        h = make_problem(tsmg, w, xd, yd, stream, precision)
        try:
            status, info = tsmg.ts_solve(h, alpha)
            if status != tsmg.TS_OK:
                raise RuntimeError("solve did not converge: %s" % info.as_dict())
            tsmg.ts_evaluate(h, alpha, n, xd, yq)
        finally:
            tsmg.ts_destroy(h)
        return info.as_dict()

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        infos.append(step())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0) / steps, infos, alpha


def apply_rate(tsmg, torch, w, stream, reps):
    """Operator-apply rate at one workload: HIP-event times of the Lambda
    passes and the point pass, FP64 and FP32, as algorithmic GB/s and FLOP/s."""
    xd = torch.from_numpy(w["x"]).cuda()
    yd = torch.from_numpy(w["y"]).cuda()
    torch.cuda.synchronize()
    h = make_problem(tsmg, w, xd, yd, stream, tsmg.TS_FP64)
    q = SMOOTHER.get("degree", 3)
    out = {"workload": w["name"], "d": w["d"], "N": w["N"], "n": len(w["y"]), "degree": q}
    try:
        G = tsmg.ts_num_levels(h)
        K = tsmg.ts_num_coeffs(h, G)
        for fp32 in (False, True):
            tsmg.ts_profile_apply(h, G, fp32, 2)
            ms_l, ms_d = tsmg.ts_profile_apply(h, G, fp32, reps)
            fl, by = algorithmic(w["d"], len(w["y"]), K, fp32, q)
            s = 4 if fp32 else 8
            by_total = by + 2 * K * s * w["d"]      # Lambda passes stream the tensors too
            t = (ms_l + ms_d) * 1e-3
            tag = "fp32" if fp32 else "fp64"
            out[tag] = {"ms_apply": ms_l + ms_d, "ms_point_pass": ms_d, "ms_lambda": ms_l,
                        "apply_GBps": by_total / t / 1e9,
                        "point_pass_TFLOPs": fl / (ms_d * 1e-3) / 1e12,
                        "point_pass_frac_fp64_valu": fl / (ms_d * 1e-3) / 1e12 / PEAK_FP64_VALU_TFLOPS}
    finally:
        tsmg.ts_destroy(h)
        del xd, yd
    return out


def serving(tsmg, workloads, R, slots, served_precision):
    """The serving trace (first R requests): plain FP64 one request at a time,
    then a mixed-precision mode through the serving loop with Poisson arrivals
    at twice the measured FP64 capacity. Both to a relative FP64 true residual
    of 1e-8; the served solutions are compared with the sequential FP64 ones
    on their coefficients and on their fitted values at the data points."""
    reqs = [workloads.serving_request(i) for i in range(R)]
    seq, _ = serve_run(tsmg, reqs, tsmg.TS_FP64, 1, None, label="fp64 sequential")
    s_seq = serve_summary(seq)
    out = {"requests": R, "sample": "requests 0..%d of the serving trace (d in 2..4, N in 16..64, "
                                    "n log-uniform 1e4..1e6, lambda log-uniform 1e-6..1e-2)" % (R - 1),
           "fp64_sequential": s_seq}
    rate = 2.0 * s_seq["solves_per_s"]
    mixed, st = serve_run(tsmg, reqs, served_precision, slots, rate, label="mixed served")
    m = serve_summary(mixed, st)
    m.update({"precision": PRECISIONS_BY_CODE[served_precision], "slots": slots, "arrival_rate_per_s": rate})
    out["mixed_served"] = m
    out.update(served_differences(reqs, seq, mixed))
    out["iterations_fp64"] = [res["info"]["iterations"] for _, res in seq]
    out["iterations_mixed"] = [res["info"]["iterations"] for _, res in mixed]
    return out


def fitted_values(alpha, x, N):
    """s(x_i) = sum_k alpha_k phi_k(x_i) at the points of a serving request
    (unit box, cubic B-splines on N uniform intervals per dimension, C-order
    coefficients), with torch on the GPU: used only to compare two solutions
    of the same request."""
    import itertools
    import torch
    xt = torch.as_tensor(x, dtype=torch.float64, device="cuda")
    a = torch.as_tensor(alpha, dtype=torch.float64, device="cuda")
    n, d = xt.shape
    u = xt * N
    cell = torch.clamp(torch.floor(u), 0, N - 1)
    t = u - cell
    s = 1.0 - t
    B = torch.stack([s ** 3 / 6, 2.0 / 3 - t ** 2 + t ** 3 / 2, 2.0 / 3 - s ** 2 + s ** 3 / 2, t ** 3 / 6], dim=-1)
    cell = cell.long()
    J = N + 3
    out = torch.zeros(n, dtype=torch.float64, device="cuda")
    for combo in itertools.product(range(4), repeat=d):
        idx = torch.zeros(n, dtype=torch.long, device="cuda")
        wgt = torch.ones(n, dtype=torch.float64, device="cuda")
        for p in range(d):
            idx = idx * J + cell[:, p] + combo[p]
            wgt = wgt * B[:, p, combo[p]]
        out += wgt * a[idx]
    return out


def served_differences(reqs, base, results):
    """Largest relative difference between two solutions of the same requests:
    of the coefficients, and of the fitted values at the request's points."""
    import numpy as np
    import torch
    dc, df = [], []
    for r, (a1, _), (a2, _) in zip(reqs, base, results):
        if a1 is None or a2 is None:
            continue
        dc.append(float(np.linalg.norm(a2 - a1) / np.linalg.norm(a1)))
        f1 = fitted_values(a1, r["x"], r["N"])
        f2 = fitted_values(a2, r["x"], r["N"])
        df.append(float(torch.linalg.norm(f2 - f1) / torch.linalg.norm(f1)))
    return {"max_rel_diff_alpha_vs_fp64_sequential": max(dc) if dc else None,
            "max_rel_diff_fitted_vs_fp64_sequential": max(df) if df else None}


def serve_run(tsmg, reqs, precision, slots, rate, policy=None, label=""):
    """Requests of the serving trace submitted at Poisson arrival times of the
    given rate (None: one at a time, each after the previous finished) to a
    server with `slots` concurrent solves; returns (solutions, results)."""
    import numpy as np
    from paper_1901_00654_amd import workloads

    def opts():
        o = tsmg.ts_default_options()
        o.precision = precision
        o.tol = 1e-8
        o.max_iter = 200000
        set_smoother(o)
        return o

    S = tsmg.Server(slots=slots, policy=policy)
    out = []
    try:
        if rate is None:
            for i, r in enumerate(reqs):
                t = S.submit(r["x"], r["y"], r["N"], r["lam"], options=opts())
                out.append(S.wait(t))
                print(json.dumps({"serve": label, "done": i + 1, "of": len(reqs)}), file=sys.stderr, flush=True)
        else:
            arrivals = workloads.poisson_arrivals(len(reqs), rate)
            t0 = time.perf_counter()
            tickets = []
            for i, r in enumerate(reqs):
                delay = t0 + arrivals[i] - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
                tickets.append(S.submit(r["x"], r["y"], r["N"], r["lam"], options=opts()))
                if i % 10 == 9:
                    print(json.dumps({"serve": label, "submitted": i + 1, "of": len(reqs)}), file=sys.stderr,
                          flush=True)
            for i, t in enumerate(tickets):
                out.append(S.wait(t))
                if i % 10 == 9:
                    print(json.dumps({"serve": label, "waited": i + 1, "of": len(reqs)}), file=sys.stderr,
                          flush=True)
        st = S.stats()
    finally:
        S.close()
    return out, st


def serve_summary(results, st=None):
    import numpy as np
    lat = np.array([res["t_done"] - res["t_submit"] for _, res in results])
    span = max(res["t_done"] for _, res in results) - min(res["t_submit"] for _, res in results)
    out = {"requests": len(results), "solves_per_s": len(results) / span, "span_s": span,
           "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
           "max_rel_residual": max(res["info"]["rel_residual"] for _, res in results),
           "failed": sum(res["status"] != 0 for _, res in results)}   # 0 = TS_OK
    if st:
        out["max_active"] = st["max_active"]
        out["max_in_use_bytes"] = st["max_in_use"]
    return out


def serve_study(tsmg, workloads, R, slots, served_precision, R_seq=None, legs=None, c64=None, c_mixed=None):
    """The serving trace (first R requests): plain FP64 one request at a time
    (capacity C64 from its first R_seq requests; always run, as the
    comparison), then the mixed mode served with `slots` concurrent solves at
    Poisson rates 2 C64 (throughput) and 0.7 x the mixed capacity measured
    there (latency), and plain FP64 served the same way at 2 C64 (control).
    Each served result is compared with the FP64 sequential solution of the
    same request (coefficients and fitted values). `legs` selects the served
    legs ("mixed2x", "fp64_2x", "mixed07"); a capacity given as c64 /
    c_mixed (from an earlier run) replaces the one measured here."""
    reqs = [workloads.serving_request(i) for i in range(R)]
    R_seq = R_seq or R
    legs = legs or ["seq", "mixed2x", "fp64_2x", "mixed07"]
    out = {"requests": R, "slots": slots,
           "sample": "requests 0..%d of the serving trace (d in 2..4, N in 16..64, n log-uniform "
                     "1e4..1e6, lambda log-uniform 1e-6..1e-2), each to a relative FP64 residual "
                     "of 1e-8" % (R - 1)}
    # the sequential FP64 solutions are the comparison for every leg
    seq, _ = serve_run(tsmg, reqs[:R_seq], tsmg.TS_FP64, 1, None, label="fp64 sequential")
    s_seq = serve_summary(seq)
    out["fp64_sequential"] = dict(s_seq, requests_timed=R_seq)
    if c64 is None:
        c64 = s_seq["solves_per_s"]
    out["fp64_capacity_per_s"] = c64
    for leg, prec, key in (("mixed2x", served_precision, "mixed_served_throughput"),
                           ("fp64_2x", tsmg.TS_FP64, "fp64_served_throughput")):
        if leg in legs:
            rate = 2.0 * c64
            res, st = serve_run(tsmg, reqs, prec, slots, rate, label=key)
            out[key] = dict(serve_summary(res, st), arrival_rate_per_s=rate, slots=slots,
                            precision=PRECISIONS_BY_CODE[prec], **served_differences(reqs, seq, res))
            print(json.dumps({"leg": key, **out[key]}), file=sys.stderr, flush=True)
            if leg == "mixed2x" and c_mixed is None:
                c_mixed = out[key]["solves_per_s"]
    if "mixed07" in legs:
        rate = 0.7 * c_mixed
        res, st = serve_run(tsmg, reqs, served_precision, slots, rate, label="mixed latency")
        out["mixed_served_latency"] = dict(serve_summary(res, st), arrival_rate_per_s=rate, slots=slots,
                                           mixed_capacity_per_s=c_mixed,
                                           precision=PRECISIONS_BY_CODE[served_precision],
                                           **served_differences(reqs, seq, res))
        print(json.dumps({"leg": "mixed_served_latency", **out["mixed_served_latency"]}), file=sys.stderr, flush=True)
    return out


def paper_experiments(tsmg, torch, workloads):
    """The paper's Sec. 4 test (sigmoid data, n = 100,000, lambda = 0.2):
    MGCG iterations and solve times for P = 2 under refinement G = 4..7
    (Fig. 2) and for P = 1..4 at G = 5 (Table 2), and the condition number of
    the V-cycle-preconditioned matrix B A at P = 2, G = 5 (Table 3), from the
    V-cycle and the operator applied to the unit vectors."""
    import numpy as np
    out = {"lambda": 0.2, "tol": 1e-8, "refinement_P2": [], "dimensions_G5": []}

    def run(P, N):
        w = workloads.paper_sigmoid(P, N=N)
        res = {"P": P, "G": int(np.log2(N))}
        for name, prec in (("fp64", tsmg.TS_FP64), ("vcycle32", tsmg.TS_MIXED_FP32_VCYCLE)):
            S = tsmg.Smoother(w["x"], w["y"], N, w["lam"], precision=prec, tol=1e-8, max_iter=20000)
            try:
                S.solve()
                t0 = time.perf_counter()
                _, status, info = S.solve()
                res[name] = {"iterations": info["iterations"], "solve_s": time.perf_counter() - t0,
                             "setup_s": info["setup_s"], "status": status}
            finally:
                S.close()
        return res, w

    for G in (4, 5, 6, 7):
        out["refinement_P2"].append(run(2, 2 ** G)[0])
    for P in (1, 2, 3, 4):
        out["dimensions_G5"].append(run(P, 32)[0])
    w = workloads.paper_sigmoid(2, N=32)
    S = tsmg.Smoother(w["x"], w["y"], 32, w["lam"])
    try:
        K = S.K()
        E = torch.eye(K, dtype=torch.float64)
        A = np.column_stack([S.apply(S.G, E[:, k]).cpu().numpy() for k in range(K)])
        B = np.column_stack([S.vcycle(E[:, k]).cpu().numpy() for k in range(K)])
    finally:
        S.close()
    ev_a = np.linalg.eigvalsh(0.5 * (A + A.T))
    ev_ba = np.sort(np.real(np.linalg.eigvals(B @ A)))
    out["kappa_A_P2G5"] = float(ev_a[-1] / ev_a[0])
    out["kappa_BA_P2G5"] = float(ev_ba[-1] / ev_ba[0])
    return out


def solve_all(tsmg, torch, workloads, stream, only=None, modes_only=None, ref_tol=1e-12):
    """Whole solves of every workload (c4 at 8^5 and 16^5 intervals) in the
    three precision modes, to a relative FP64 true residual of 1e-8: time,
    iterations, and each solution's distance to an FP64 solve of the same
    problem driven to 1e-12 (solve_study)."""
    os.environ.setdefault("TSMG_PROGRESS", "250")   # long solves print their progress
    cases = [("c1", {}), ("c2", {}), ("c3", {}), ("c4", {"N": 8}), ("c4", {"N": 16})]
    if only:
        cases = [c for c in cases if "%s/%d" % (c[0], c[1].get("N", 0)) in only or c[0] in only]
    modes = [("fp64", tsmg.TS_FP64), ("mixed", tsmg.TS_MIXED_FP32), ("vcycle32", tsmg.TS_MIXED_FP32_VCYCLE)]
    if modes_only:
        modes = [m for m in modes if m[0] in modes_only]
    out = []
    for name, kw in cases:
        w = workloads.CONFIGS[name](**kw)
        out.append(solve_study(tsmg, torch, w, stream, modes, ref_tol=ref_tol,
                               progress=lambda r: print(json.dumps({"progress": name, "N": w["N"], **r}),
                                                        file=sys.stderr, flush=True)))
    return out


def copy_calibration(torch):
    """A plain streaming kernel of known size (1 GiB read, 1 GiB written, as
    an elementwise multiply by one, which runs as a kernel where a same-type
    copy may go to a DMA engine), for scaling HBM byte counters."""
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    return src.numel() * 8


def accuracy(tsmg, torch, h, w, xd, alpha, ref):
    """Distance of a solution to a reference solution of the same problem:
    relative differences of the coefficients, of the fitted values at the data
    points (ts_evaluate) and in the energy norm (ts_apply)."""
    n = len(w["y"])
    G = tsmg.ts_num_levels(h)
    K = tsmg.ts_num_coeffs(h, G)
    e = (alpha - ref).contiguous()
    fe = torch.empty(n, dtype=torch.float64, device="cuda")
    fr = torch.empty(n, dtype=torch.float64, device="cuda")
    tsmg.ts_evaluate(h, e, n, xd, fe)
    tsmg.ts_evaluate(h, ref, n, xd, fr)
    Ae = torch.empty(K, dtype=torch.float64, device="cuda")
    Ar = torch.empty(K, dtype=torch.float64, device="cuda")
    tsmg.ts_apply(h, G, e, Ae)
    tsmg.ts_apply(h, G, ref, Ar)
    torch.cuda.synchronize()
    return {"coef": float(torch.linalg.norm(e) / torch.linalg.norm(ref)),
            "fitted": float(torch.linalg.norm(fe) / torch.linalg.norm(fr)),
            "energy": float(torch.sqrt(torch.abs(e @ Ae) / (ref @ Ar)))}


def solve_study(tsmg, torch, w, stream, modes, ref_tol=1e-12, progress=None):
    """Whole solves of one workload to a relative FP64 residual of 1e-8 in the
    given modes, each with its time, iterations and its distance to an FP64
    solve of the same problem driven to ref_tol (None: no reference)."""
    xd = torch.from_numpy(w["x"]).cuda()
    yd = torch.from_numpy(w["y"]).cuda()
    torch.cuda.synchronize()
    K = (w["N"] + 3) ** w["d"]
    out = {"workload": w["name"], "d": w["d"], "N": w["N"], "n": len(w["y"]), "lambda": w["lam"]}
    h = make_problem(tsmg, w, xd, yd, stream, tsmg.TS_FP64, tol=ref_tol or 1e-8)
    try:
        ref = None
        if ref_tol:
            ref = torch.empty(K, dtype=torch.float64, device="cuda")
            t0 = time.perf_counter()
            st, info = tsmg.ts_solve(h, ref)
            out["reference"] = {"tol": ref_tol, "status": st, "iterations": info.iterations,
                                "rel_residual": info.rel_residual, "solve_s": time.perf_counter() - t0}
            if progress:
                progress({"reference": out["reference"]})
        for name, prec in modes:
            o = tsmg.ts_default_options()
            o.precision = prec
            o.tol = 1e-8
            o.max_iter = 100000
            set_smoother(o)
            tsmg.ts_set_options(h, o)
            a = torch.empty(K, dtype=torch.float64, device="cuda")
            t0 = time.perf_counter()
            st, info = tsmg.ts_solve(h, a)
            dt = time.perf_counter() - t0
            out[name] = {"status": st, "iterations": info.iterations, "refinements": info.refinements,
                         "rel_residual": info.rel_residual, "solve_s": dt, "setup_s": info.setup_s}
            if ref is not None:
                out[name]["vs_fp64_ref"] = accuracy(tsmg, torch, h, w, xd, a, ref)
            if progress:
                progress({name: out[name]})
    finally:
        tsmg.ts_destroy(h)
        del xd, yd
        torch.cuda.empty_cache()
    return out


def per_iteration(tsmg, torch, w, stream, iters, precision):
    """Time of a fixed number of MGCG iterations on one workload (the solve
    stopped by max_iter): ms per iteration, setup excluded."""
    xd = torch.from_numpy(w["x"]).cuda()
    yd = torch.from_numpy(w["y"]).cuda()
    torch.cuda.synchronize()
    K = (w["N"] + 3) ** w["d"]
    h = make_problem(tsmg, w, xd, yd, stream, precision)
    try:
        o = tsmg.ts_default_options()
        o.precision = precision
        o.tol = 1e-30
        o.max_iter = iters
        o.max_refine = 1000
        set_smoother(o)
        tsmg.ts_set_options(h, o)
        a = torch.empty(K, dtype=torch.float64, device="cuda")
        t0 = time.perf_counter()
        st, info = tsmg.ts_solve(h, a)
        dt = time.perf_counter() - t0
        return {"iterations_timed": info.iterations, "solve_s": dt, "ms_per_iteration": dt / info.iterations * 1e3,
                "setup_s": info.setup_s}
    finally:
        tsmg.ts_destroy(h)
        del xd, yd
        torch.cuda.empty_cache()


def cpu_baseline(tsmg, torch, workloads, stream, w_full, budget_apply_s=8.0):
    """The oracle as it stands, timed on this host on a bounded sample of the
    c2 workload: its whole MGCG solve (assembled hierarchy, Lanczos damping,
    Alg. 8 to a relative residual of 1e-8) on the c2 recipe at 1/64 of the
    size (N = 16, n = 31,250: the same points per cell), next to the GPU's
    solve of the same sample; and its matrix-free FP64 apply on the full c2
    points next to the GPU's."""
    import numpy as np
    from oracle import matfree, mg, system
    ws = workloads.c2(n=31250, N=16)
    t0 = time.perf_counter()
    levels = system.hierarchy(ws["x"], ws["y"], ws["lo"], ws["hi"], ws["N"], ws["lam"])
    M = mg.MG(ws["x"], ws["y"], ws["lo"], ws["hi"], ws["N"], ws["lam"], levels=levels)
    top = levels[M.G]
    _, its_cpu, _ = mg.pcg(top["A"], top["b"], M.vcycle, tol=1e-8, maxiter=20000)
    t_cpu = time.perf_counter() - t0
    # the GPU on the same sample (setup + solve)
    xd = torch.from_numpy(ws["x"]).cuda()
    yd = torch.from_numpy(ws["y"]).cuda()
    torch.cuda.synchronize()
    K = (ws["N"] + 3) ** 3
    a = torch.empty(K, dtype=torch.float64, device="cuda")
    times = []
    for _ in range(4):
        t0 = time.perf_counter()
        h = make_problem(tsmg, ws, xd, yd, stream, tsmg.TS_FP64)
        try:
            st, info = tsmg.ts_solve(h, a)
        finally:
            tsmg.ts_destroy(h)
        times.append(time.perf_counter() - t0)
    t_gpu = float(np.median(times[1:]))
    # the matrix-free apply at full size
    c = np.random.default_rng(0).standard_normal((w_full["N"] + 3) ** w_full["d"])
    ta = []
    t_start = time.perf_counter()
    while not ta or (time.perf_counter() - t_start < budget_apply_s and len(ta) < 3):
        t0 = time.perf_counter()
        matfree.apply(w_full["x"], c, w_full["lo"], w_full["hi"], w_full["N"], w_full["lam"])
        ta.append(time.perf_counter() - t0)
    return {"value": 1.0 / t_cpu, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": ("c2 recipe at 1/64 size (d=3, N=16, n=31,250, same points per cell): the oracle's "
                       "whole MGCG solve (assembly, Lanczos, Alg. 8 to 1e-8) took %.1f s in %d "
                       "iterations (single-threaded SciPy sparse); the GPU solves the same sample "
                       "(setup + solve) in %.2f ms in %d iterations" % (t_cpu, its_cpu, t_gpu * 1e3,
                                                                         info.iterations)),
            "gpu_same_sample_solves_per_s": 1.0 / t_gpu,
            "per_apply_full_c2": {"oracle_s": float(np.median(ta)), "applies_timed": len(ta),
                                  "label": "per apply, not per solve: the oracle's matrix-free FP64 "
                                           "A c on the full c2 points"},
            "host_cpus": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--reps", type=int, default=20, help="timed launches per apply measurement")
    ap.add_argument("--no-sweep", action="store_true", help="skip the d=2..5 apply sweep")
    ap.add_argument("--no-compare", action="store_true", help="skip the other precision")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--serve-requests", type=int, default=32,
                    help="requests of the serving trace to run (0: skip the serving leg)")
    ap.add_argument("--serve-slots", type=int, default=4, help="concurrent solves in the serving loop")
    ap.add_argument("--serve-precision", choices=["mixed", "vcycle32"], default="vcycle32",
                    help="mode of the served requests: FP32 CG with reliable updates, or FP64 CG "
                         "with an FP32 V-cycle")
    ap.add_argument("--only-serve", action="store_true", help="run only the serving leg")
    ap.add_argument("--serve-study", action="store_true",
                    help="only the serving study: FP64 sequential, mixed and FP64 served at 2x the FP64 "
                         "capacity, mixed served at 0.7x its capacity; prints one JSON line")
    ap.add_argument("--serve-seq", type=int, default=None,
                    help="with --serve-study: requests timed one at a time for the FP64 capacity")
    ap.add_argument("--serve-legs", default=None,
                    help="with --serve-study: comma-separated legs (seq, mixed2x, fp64_2x, mixed07)")
    ap.add_argument("--serve-c64", type=float, default=None,
                    help="with --serve-study: FP64 capacity (solves/s) measured in an earlier run")
    ap.add_argument("--serve-cmixed", type=float, default=None,
                    help="with --serve-study: mixed served capacity (solves/s) measured in an earlier run")
    ap.add_argument("--solve-all", action="store_true",
                    help="only whole solves of c1..c4 in every precision mode; prints one JSON line")
    ap.add_argument("--cases", default=None,
                    help="with --solve-all: comma-separated workloads, e.g. c3 or c4/16")
    ap.add_argument("--modes", default=None, help="with --solve-all: comma-separated modes (fp64,mixed,vcycle32)")
    ap.add_argument("--ref-tol", type=float, default=1e-12,
                    help="with --solve-all: tolerance of the FP64 reference solve (default 1e-12)")
    ap.add_argument("--no-reference", action="store_true",
                    help="with --solve-all: skip the tight FP64 reference solve and the distances to it")
    ap.add_argument("--paper", action="store_true",
                    help="only the paper's own test problem (Sec. 4): iterations under refinement and "
                         "across dimensions, kappa(A) and kappa(BA); prints one JSON line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration under rocprofv3)")
    ap.add_argument("--nu", type=int, default=None, help="smoothing steps nu1 = nu2 (default: the library's)")
    ap.add_argument("--omega-scale", type=float, default=None, help="Jacobi damping scale (default: the library's)")
    ap.add_argument("--ppb", type=int, default=None, help="points per workgroup of the point pass (default: auto)")
    ap.add_argument("--no-c3", action="store_true", help="skip the whole c3 solves")
    ap.add_argument("--no-c4", action="store_true", help="skip the c4 per-iteration timing")
    ap.add_argument("--intervals", type=int, default=None,
                    help="with --only-apply: knot intervals per dimension instead of the workload's (any N >= 1; "
                         "other than a power of two it runs the general form)")
    ap.add_argument("--degree", type=int, default=None,
                    help="with --only-apply: B-spline degree 1..5 (other than 3 it runs the general form)")
    ap.add_argument("--only-apply", default=None, metavar="WORKLOAD",
                    help="only time the finest-level operator apply of one workload (c1..c4), "
                         "for profiling runs; prints one JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1901_00654_amd import tsmg, workloads

    tsmg.load_library()
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    if args.nu is not None:
        SMOOTHER["nu"] = args.nu
    if args.omega_scale is not None:
        SMOOTHER["omega_scale"] = args.omega_scale
    if args.ppb is not None:
        SMOOTHER["ppb"] = args.ppb
    if args.solve_all:
        print(json.dumps(solve_all(tsmg, torch, workloads, stream, args.cases.split(",") if args.cases else None,
                                   args.modes.split(",") if args.modes else None,
                                   None if args.no_reference else args.ref_tol)), flush=True)
        return
    if args.paper:
        print(json.dumps(paper_experiments(tsmg, torch, workloads)), flush=True)
        return
    if args.serve_study:
        print(json.dumps(serve_study(tsmg, workloads, args.serve_requests, args.serve_slots,
                                     SERVE_PRECISION[args.serve_precision](tsmg), args.serve_seq,
                                     args.serve_legs.split(",") if args.serve_legs else None,
                                     args.serve_c64, args.serve_cmixed)), flush=True)
        return
    if args.only_serve:
        print(json.dumps(serving(tsmg, workloads, args.serve_requests, args.serve_slots,
                                 SERVE_PRECISION[args.serve_precision](tsmg))), flush=True)
        return
    if args.degree is not None:
        SMOOTHER["degree"] = args.degree
    if args.only_apply:
        wk = workloads.CONFIGS[args.only_apply](**({"N": args.intervals} if args.intervals else {}))
        res = apply_rate(tsmg, torch, wk, stream, args.reps)
        if args.copy_calibration:
            res["copy_calibration_bytes"] = copy_calibration(torch)
        print(json.dumps(res), flush=True)
        return
    w = workloads.c2()
    xd = torch.from_numpy(w["x"]).cuda()
    yd = torch.from_numpy(w["y"]).cuda()
    torch.cuda.synchronize()
    prec = tsmg.TS_FP64 if args.precision == "fp64" else tsmg.TS_MIXED_FP32
    sec, infos, alpha = run_steps(tsmg, torch, w, xd, yd, stream, prec, args.steps, args.warmup)
    info = infos[-1]

    # roofline of the dominant kernel: the finest-level point pass, FP64
    h = make_problem(tsmg, w, xd, yd, stream, tsmg.TS_FP64)
    try:
        G = tsmg.ts_num_levels(h)
        K = tsmg.ts_num_coeffs(h, G)
        fp32 = prec != tsmg.TS_FP64 and False
        tsmg.ts_profile_apply(h, G, fp32, 2)
        ms_lam, ms_data = tsmg.ts_profile_apply(h, G, fp32, args.reps)
    finally:
        tsmg.ts_destroy(h)
    flops, nbytes = algorithmic(w["d"], len(w["y"]), K, False)
    t_data = ms_data * 1e-3
    achieved = flops / t_data / 1e12
    tr = traffic_bytes()
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VALU_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_VALU_TFLOPS, "traffic": tr,
                "kernel": "k_data<3,double,apply> (point pass, finest level)",
                "ms_per_launch": ms_data, "algorithmic_flop": flops, "algorithmic_bytes": nbytes,
                "algorithmic_GBps": nbytes / t_data / 1e9,
                # the same launch against the other roof: algorithmic and
                # counted HBM bytes over the 8 TB/s peak
                "hbm_frac_algorithmic": nbytes / t_data / 1e9 / PEAK_HBM_GBPS,
                "hbm_frac_measured": (tr / t_data / 1e9 / PEAK_HBM_GBPS) if tr else None}

    result = {
        "metric": METRIC, "value": 1.0 / sec, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": sec * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if prec == tsmg.TS_FP64 else "f32+f64",
        "data": "synthetic (seeded Gaussian mixture, see workloads.c2)",
        "config": {"workload": "c2: d=3 cubic, 64^3 intervals (K=300763), n=2,000,000 clustered points, "
                               "lambda=1e-5, MGCG to rel. FP64 residual 1e-8",
                   "precision": args.precision, "levels": G,
                   "nu": SMOOTHER.get("nu", tsmg.ts_default_options().nu1),
                   "omega_scale": SMOOTHER.get("omega_scale", tsmg.ts_default_options().omega_scale)},
        "time_to_tol_s": info["solve_s"], "setup_s": info["setup_s"], "iterations": info["iterations"],
        "refinements": info["refinements"], "rel_residual": info["rel_residual"],
        "applies_per_solve": info["applies"], "roofline": roofline,
        "lambda_passes_ms": ms_lam,
    }

    def progress(tag):
        return lambda r: print(json.dumps({"progress": tag, **r}), file=sys.stderr, flush=True)

    del xd, yd
    torch.cuda.empty_cache()
    modes = [("fp64", tsmg.TS_FP64), ("mixed", tsmg.TS_MIXED_FP32), ("vcycle32", tsmg.TS_MIXED_FP32_VCYCLE)]
    if not args.no_compare:
        # every precision mode on the headline workload, with its distance to
        # an FP64 solve driven to 1e-12
        result["precision_modes_c2"] = solve_study(tsmg, torch, w, stream, modes, progress=progress("c2"))
    if not args.no_c3:
        # the d = 4 workload (10^7 points, 35^4 coefficients) solved whole,
        # FP64 and with the FP32 V-cycle
        result["solve_c3"] = solve_study(tsmg, torch, workloads.c3(), stream, [modes[0], modes[2]],
                                         progress=progress("c3"))
    if not args.no_c4:
        # d = 5 (2e7 points, 19^5 coefficients): MGCG iterations timed for a
        # fixed count; the iteration count to 1e-8 comes from whole solves
        # (bench.py --solve-all --cases c4/16), so the time to tolerance here is
        # ms per iteration x that count, labelled as such
        w4 = workloads.c4()
        rec = {"workload": "c4", "d": 5, "N": 16, "n": len(w4["y"])}
        for name, pm in (modes[0], modes[2]):
            rec[name] = per_iteration(tsmg, torch, w4, stream, 20, pm)
            progress("c4")({name: rec[name]})
        result["per_iteration_c4"] = rec
        del w4

    if not args.no_sweep:
        sweep = []
        for name in ("c1", "c2", "c3", "c4"):
            wk = w if name == "c2" else workloads.CONFIGS[name]()
            sweep.append(apply_rate(tsmg, torch, wk, stream, args.reps))
            torch.cuda.empty_cache()
        result["apply_sweep"] = sweep

    if args.serve_requests > 0:
        result["serving"] = serving(tsmg, workloads, args.serve_requests, args.serve_slots,
                                    SERVE_PRECISION[args.serve_precision](tsmg))

    if args.copy_calibration:
        result["copy_calibration_bytes"] = copy_calibration(torch)

    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(tsmg, torch, workloads, stream, w)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
