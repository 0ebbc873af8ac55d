"""ctypes binding of the tsmg C ABI (include/tsmg.h).

The functions ``ts_*`` below carry the header's names and arguments one for
one; vector arguments are device addresses given as ints or as torch tensors
(their ``data_ptr()``; shape, dtype and device are checked here). Nothing in
this module computes: every step runs in the HIP kernels of libtsmg.so, and
loading fails loudly if that library is not built.

``Smoother`` is a thin convenience wrapper that allocates outputs as torch
tensors on the GPU, runs everything on its own torch stream and synchronises
before returning.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtsmg.so")

TS_OK, TS_ENOTCONV, TS_EINVAL, TS_ENOMEM, TS_EDEVICE, TS_ESINGULAR, TS_EBREAKDOWN = 0, 1, -1, -2, -3, -4, -5
TS_FP64, TS_MIXED_FP32, TS_MIXED_BF16, TS_MIXED_FP32_VCYCLE = 0, 1, 2, 3
TS_STENCIL_AUTO, TS_STENCIL_NONE, TS_STENCIL_ALL = 0, 1, 2
TS_PC_MG, TS_PC_NONE, TS_PC_JACOBI = 0, 1, 2
TS_SMOOTH_JACOBI, TS_SMOOTH_SSOR = 0, 1
TS_COARSE_DIRECT, TS_COARSE_CG = 0, 1
TS_ADMIT_SHORTEST, TS_ADMIT_FIFO = 0, 1
_STATUS = {0: "TS_OK", 1: "TS_ENOTCONV", -1: "TS_EINVAL", -2: "TS_ENOMEM", -3: "TS_EDEVICE",
           -4: "TS_ESINGULAR", -5: "TS_EBREAKDOWN"}


class ts_options(ctypes.Structure):
    _fields_ = [("nu1", ctypes.c_int), ("nu2", ctypes.c_int),
                ("omega_scale", ctypes.c_double), ("lanczos_steps", ctypes.c_int),
                ("omega_fixed", ctypes.c_double), ("precision", ctypes.c_int),
                ("max_iter", ctypes.c_int), ("tol", ctypes.c_double),
                ("inner_tol", ctypes.c_double), ("max_refine", ctypes.c_int),
                ("points_per_block", ctypes.c_int), ("stencil_mode", ctypes.c_int),
                ("stream", ctypes.c_void_p),
                ("preconditioner", ctypes.c_int), ("smoother", ctypes.c_int),
                ("ssor_omega", ctypes.c_double), ("coarse_solver", ctypes.c_int),
                ("coarse_tol", ctypes.c_double), ("coarse_max_iter", ctypes.c_int),
                ("coarsest_level", ctypes.c_int), ("degrees", ctypes.POINTER(ctypes.c_int32)),
                ("deterministic", ctypes.c_int), ("bottom_max_k", ctypes.c_int),
                ("vcycle_graph", ctypes.c_int)]


class ts_solve_info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("refinements", ctypes.c_int),
                ("converged", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("setup_s", ctypes.c_double), ("solve_s", ctypes.c_double),
                ("applies", ctypes.c_int64),
                ("residual_history", ctypes.POINTER(ctypes.c_double)), ("history_len", ctypes.c_int)]

    def as_dict(self):
        out = {k: getattr(self, k) for k, _ in self._fields_ if k != "residual_history"}
        n = self.history_len
        out["residual_history"] = ([self.residual_history[i] for i in range(n)]
                                   if n > 0 and self.residual_history else [])
        return out


class ts_server_options(ctypes.Structure):
    _fields_ = [("memory_budget", ctypes.c_size_t), ("slots", ctypes.c_int), ("policy", ctypes.c_int),
                ("max_wait_s", ctypes.c_double)]


class ts_request(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("q", ctypes.c_int),
                ("intervals", ctypes.POINTER(ctypes.c_int32)),
                ("lo", ctypes.POINTER(ctypes.c_double)), ("hi", ctypes.POINTER(ctypes.c_double)),
                ("n", ctypes.c_int64),
                ("x", ctypes.POINTER(ctypes.c_double)), ("y", ctypes.POINTER(ctypes.c_double)),
                ("lam", ctypes.c_double), ("opt", ctypes.POINTER(ts_options))]


class ts_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("info", ts_solve_info), ("K", ctypes.c_int64),
                ("footprint", ctypes.c_size_t), ("peak_bytes", ctypes.c_size_t),
                ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double), ("t_done", ctypes.c_double),
                ("error", ctypes.c_char * 256)]

    def as_dict(self):
        out = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("info", "error")}
        out["info"] = self.info.as_dict()
        out["error"] = self.error.decode(errors="replace")
        return out


class ts_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("active", ctypes.c_int), ("max_active", ctypes.c_int),
                ("in_use", ctypes.c_size_t), ("max_in_use", ctypes.c_size_t),
                ("memory_budget", ctypes.c_size_t)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TsmgError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s (%d): %s" % (_STATUS.get(status, "?"), status, message))
        self.status = status


_lib = None
_P = ctypes.c_void_p
_D = ctypes.c_double
_I = ctypes.c_int
_I64 = ctypes.c_int64

_SIGNATURES = {
    "ts_default_options": (None, [ctypes.POINTER(ts_options)]),
    "ts_version": (ctypes.c_char_p, []),
    "ts_last_error": (ctypes.c_char_p, []),
    "ts_create": (_I, [_I, _I, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_D), ctypes.POINTER(_D),
                       _I64, _P, _P, _D, ctypes.POINTER(ts_options), ctypes.POINTER(_P)]),
    "ts_destroy": (None, [_P]),
    "ts_set_options": (_I, [_P, ctypes.POINTER(ts_options)]),
    "ts_num_levels": (_I, [_P, ctypes.POINTER(_I)]),
    "ts_num_coeffs": (_I, [_P, _I, ctypes.POINTER(_I64)]),
    "ts_get_omega": (_I, [_P, _I, ctypes.POINTER(_D)]),
    "ts_bottom_level": (_I, [_P, ctypes.POINTER(_I)]),
    "ts_rhs": (_I, [_P, _P]),
    "ts_apply": (_I, [_P, _I, _P, _P]),
    "ts_apply_f32": (_I, [_P, _I, _P, _P]),
    "ts_diag": (_I, [_P, _I, _P]),
    "ts_prolong": (_I, [_P, _I, _P, _P]),
    "ts_restrict": (_I, [_P, _I, _P, _P]),
    "ts_coarse_solve": (_I, [_P, _P, _P]),
    "ts_vcycle": (_I, [_P, _P, _P]),
    "ts_vcycle_f32": (_I, [_P, _P, _P]),
    "ts_solve": (_I, [_P, _P, _I, ctypes.POINTER(ts_solve_info)]),
    "ts_evaluate": (_I, [_P, _P, _I64, _P, _P]),
    "ts_profile_apply": (_I, [_P, _I, _I, _I, ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "ts_memory": (_I, [_P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
    "ts_footprint": (_I, [_I, _I, ctypes.POINTER(ctypes.c_int32), _I64, ctypes.POINTER(ts_options),
                          ctypes.POINTER(ctypes.c_size_t)]),
    "ts_solve_noalloc": (_I, [_I, _I, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_D), ctypes.POINTER(_D),
                              _I64, _P, _P, _D, ctypes.POINTER(ts_options), _P, ctypes.POINTER(ts_solve_info)]),
    "ts_server_default_options": (None, [ctypes.POINTER(ts_server_options)]),
    "ts_server_create": (_I, [ctypes.POINTER(ts_server_options), ctypes.POINTER(_P)]),
    "ts_server_submit": (_I, [_P, ctypes.POINTER(ts_request), ctypes.POINTER(ctypes.c_uint64)]),
    "ts_server_poll": (_I, [_P, ctypes.c_uint64, ctypes.POINTER(_I)]),
    "ts_server_wait": (_I, [_P, ctypes.c_uint64, _P, _I64, ctypes.POINTER(ts_result)]),
    "ts_server_get_stats": (_I, [_P, ctypes.POINTER(ts_server_stats)]),
    "ts_server_destroy": (None, [_P]),
}


def load_library(path=None):
    """Loads libtsmg.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError("libtsmg.so not found at %s; build it with "
                           "`python -m paper_1901_00654_amd.build`" % path)
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    """Names of the C entry points this binding declares."""
    return list(_SIGNATURES)


def _check(status):
    if status < 0:
        raise TsmgError(status, load_library().ts_last_error().decode())
    return status


def _ptr(t, dtype=None, numel=None):
    """Device address of a torch tensor (checked) or an int address."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    import torch
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError("tensor dtype %s, expected %s" % (t.dtype, dtype))
    if numel is not None and t.numel() < numel:
        raise ValueError("tensor has %d elements, needs %d" % (t.numel(), numel))
    return t.data_ptr()


# --- the C ABI, one function per entry point -------------------------------

def ts_default_options():
    o = ts_options()
    load_library().ts_default_options(ctypes.byref(o))
    return o


def ts_version():
    return load_library().ts_version().decode()


def ts_last_error():
    return load_library().ts_last_error().decode()


def ts_create(d, q, intervals, lo, hi, n, x, y, lam, opt=None):
    lib = load_library()
    iv = (ctypes.c_int32 * d)(*[int(v) for v in intervals])
    lo_ = (ctypes.c_double * d)(*[float(v) for v in lo])
    hi_ = (ctypes.c_double * d)(*[float(v) for v in hi])
    h = _P()
    _check(lib.ts_create(int(d), int(q), iv, lo_, hi_, int(n), _ptr(x), _ptr(y), float(lam),
                         ctypes.byref(opt) if opt is not None else None, ctypes.byref(h)))
    return h.value


def ts_destroy(h):
    load_library().ts_destroy(h)


def ts_set_options(h, opt):
    return _check(load_library().ts_set_options(h, ctypes.byref(opt)))


def ts_num_levels(h):
    G = _I()
    _check(load_library().ts_num_levels(h, ctypes.byref(G)))
    return G.value


def ts_num_coeffs(h, level):
    K = _I64()
    _check(load_library().ts_num_coeffs(h, int(level), ctypes.byref(K)))
    return K.value


def ts_bottom_level(h):
    g = _I()
    _check(load_library().ts_bottom_level(h, ctypes.byref(g)))
    return g.value


def ts_get_omega(h, level):
    w = _D()
    _check(load_library().ts_get_omega(h, int(level), ctypes.byref(w)))
    return w.value


def ts_rhs(h, b):
    return _check(load_library().ts_rhs(h, _ptr(b)))


def ts_apply(h, level, c, out):
    return _check(load_library().ts_apply(h, int(level), _ptr(c), _ptr(out)))


def ts_apply_f32(h, level, c, out):
    return _check(load_library().ts_apply_f32(h, int(level), _ptr(c), _ptr(out)))


def ts_diag(h, level, D):
    return _check(load_library().ts_diag(h, int(level), _ptr(D)))


def ts_prolong(h, level, e, out):
    return _check(load_library().ts_prolong(h, int(level), _ptr(e), _ptr(out)))


def ts_restrict(h, level, r, out):
    return _check(load_library().ts_restrict(h, int(level), _ptr(r), _ptr(out)))


def ts_coarse_solve(h, b, x):
    return _check(load_library().ts_coarse_solve(h, _ptr(b), _ptr(x)))


def ts_vcycle(h, r, z):
    return _check(load_library().ts_vcycle(h, _ptr(r), _ptr(z)))


def ts_vcycle_f32(h, r, z):
    return _check(load_library().ts_vcycle_f32(h, _ptr(r), _ptr(z)))


def ts_solve(h, alpha, use_start=False):
    info = ts_solve_info()
    status = _check(load_library().ts_solve(h, _ptr(alpha), int(bool(use_start)), ctypes.byref(info)))
    return status, info


def ts_evaluate(h, alpha, m, xq, yq):
    return _check(load_library().ts_evaluate(h, _ptr(alpha), int(m), _ptr(xq), _ptr(yq)))


def ts_profile_apply(h, level, fp32, reps):
    """Average ms per launch of (lambda passes, point pass) of A_level."""
    a, b = _D(), _D()
    _check(load_library().ts_profile_apply(h, int(level), int(bool(fp32)), int(reps), ctypes.byref(a),
                                           ctypes.byref(b)))
    return a.value, b.value


def ts_memory(h):
    """(resident, peak) device bytes of a problem."""
    r, p = ctypes.c_size_t(), ctypes.c_size_t()
    _check(load_library().ts_memory(h, ctypes.byref(r), ctypes.byref(p)))
    return r.value, p.value


def ts_footprint(d, q, intervals, n, opt=None):
    iv = (ctypes.c_int32 * d)(*[int(v) for v in intervals])
    b = ctypes.c_size_t()
    _check(load_library().ts_footprint(int(d), int(q), iv, int(n), ctypes.byref(opt) if opt is not None else None,
                                       ctypes.byref(b)))
    return b.value


TS_NOALLOC_SCRATCH_BYTES = 64 << 20


def ts_solve_noalloc(d, q, intervals, lo, hi, n, x, y, lam, alpha, opt=None):
    """ts_create + ts_solve + ts_destroy in the library's static device
    scratch (no device allocation); returns (status, info)."""
    lib = load_library()
    iv = (ctypes.c_int32 * d)(*[int(v) for v in intervals])
    lo_ = (ctypes.c_double * d)(*[float(v) for v in lo])
    hi_ = (ctypes.c_double * d)(*[float(v) for v in hi])
    info = ts_solve_info()
    status = _check(lib.ts_solve_noalloc(int(d), int(q), iv, lo_, hi_, int(n), _ptr(x), _ptr(y), float(lam),
                                         ctypes.byref(opt) if opt is not None else None, _ptr(alpha),
                                         ctypes.byref(info)))
    return status, info


def ts_server_default_options():
    o = ts_server_options()
    load_library().ts_server_default_options(ctypes.byref(o))
    return o


def ts_server_create(opt=None):
    h = _P()
    _check(load_library().ts_server_create(ctypes.byref(opt) if opt is not None else None, ctypes.byref(h)))
    return h.value


def ts_server_submit(s, req):
    t = ctypes.c_uint64()
    _check(load_library().ts_server_submit(s, ctypes.byref(req), ctypes.byref(t)))
    return t.value


def ts_server_poll(s, ticket):
    done = _I()
    _check(load_library().ts_server_poll(s, ctypes.c_uint64(ticket), ctypes.byref(done)))
    return bool(done.value)


def ts_server_wait(s, ticket, alpha, capacity):
    """alpha: host buffer address (int) or None; returns the ts_result."""
    res = ts_result()
    _check(load_library().ts_server_wait(s, ctypes.c_uint64(ticket), alpha, int(capacity), ctypes.byref(res)))
    return res


def ts_server_get_stats(s):
    st = ts_server_stats()
    _check(load_library().ts_server_get_stats(s, ctypes.byref(st)))
    return st


def ts_server_destroy(s):
    load_library().ts_server_destroy(s)


# --- convenience wrappers --------------------------------------------------

class Server:
    """Serving loop on the current GPU: submit numpy requests, wait for numpy
    solutions. Requests are copied at submit; solutions come back as float64
    arrays of K = (N + 3)^d coefficients (C order)."""

    def __init__(self, memory_budget=0, slots=4, policy=None, max_wait_s=None):
        o = ts_server_default_options()
        o.memory_budget = int(memory_budget)
        o.slots = int(slots)
        if policy is not None:
            o.policy = int(policy)
        if max_wait_s is not None:
            o.max_wait_s = float(max_wait_s)
        self.handle = ts_server_create(o)
        self._K = {}

    def submit(self, x, y, N, lam, lo=None, hi=None, options=None, **opts):
        import numpy as np
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        n, d = x.shape
        if y.shape != (n,):
            raise ValueError("y must have shape (n,)")
        lo = [0.0] * d if lo is None else lo
        hi = [1.0] * d if hi is None else hi
        opt = options if options is not None else ts_default_options()
        for k, v in opts.items():
            setattr(opt, k, v)
        iv = (ctypes.c_int32 * d)(*([int(N)] * d))
        lo_ = (ctypes.c_double * d)(*[float(v) for v in lo])
        hi_ = (ctypes.c_double * d)(*[float(v) for v in hi])
        req = ts_request(d=d, q=3, intervals=iv, lo=lo_, hi=hi_, n=n,
                         x=x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                         y=y.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                         lam=float(lam), opt=ctypes.pointer(opt))
        t = ts_server_submit(self.handle, req)
        self._K[t] = (int(N) + 3) ** d
        return t

    def poll(self, ticket):
        return ts_server_poll(self.handle, ticket)

    def wait(self, ticket):
        """(alpha or None if the request failed, result dict)."""
        import numpy as np
        K = self._K.get(ticket)
        if K is None:     # unknown here: let the library report it
            ts_server_wait(self.handle, ticket, None, 0)
        alpha = np.empty(K, dtype=np.float64)
        res = ts_server_wait(self.handle, ticket, alpha.ctypes.data, K)
        del self._K[ticket]
        return (alpha if res.status >= 0 else None), res.as_dict()

    def stats(self):
        return ts_server_get_stats(self.handle).as_dict()

    def close(self):
        if self.handle is not None:
            ts_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Smoother:
    """One smoothing problem on the current GPU, outputs as torch tensors.

    x: (n, d) float64, y: (n,) float64 (numpy arrays or torch tensors; copied
    to the GPU if needed). All work runs on a private torch stream; every
    method synchronises it before returning.
    """

    def __init__(self, x, y, N, lam, lo=None, hi=None, options=None, stream=None, q=3, degrees=None, **opts):
        """N: knot intervals, one int for every dimension or one per
        dimension; q: the B-spline degree, or degrees: one per dimension."""
        import torch
        self.torch = torch
        self.stream = stream if stream is not None else torch.cuda.Stream()
        x = torch.as_tensor(x, dtype=torch.float64)
        y = torch.as_tensor(y, dtype=torch.float64)
        n, d = x.shape
        self.d, self.n, self.lam = int(d), int(n), float(lam)
        self.intervals = [int(v) for v in N] if hasattr(N, "__len__") else [int(N)] * self.d
        self.N = self.intervals[0]
        self.lo = [0.0] * d if lo is None else [float(v) for v in lo]
        self.hi = [1.0] * d if hi is None else [float(v) for v in hi]
        opt = options if options is not None else ts_default_options()
        for k, v in opts.items():
            setattr(opt, k, v)
        opt.stream = self.stream.cuda_stream
        self._degrees = None
        if degrees is not None:
            self._degrees = (ctypes.c_int32 * d)(*[int(v) for v in degrees])
            opt.degrees = ctypes.cast(self._degrees, ctypes.POINTER(ctypes.c_int32))
        self.options = opt
        self.handle = None
        with torch.cuda.stream(self.stream):
            xd = x.to("cuda").contiguous()
            yd = y.to("cuda").contiguous()
            self.stream.synchronize()
            self.handle = ts_create(d, int(q), self.intervals, self.lo, self.hi, n, xd, yd, lam, opt)
        self.G = ts_num_levels(self.handle)

    def close(self):
        if self.handle is not None:
            ts_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_options(self, **kw):
        """Changes solve-time options (tol, precision, max_iter, nu1, nu2, ...)."""
        for k, v in kw.items():
            setattr(self.options, k, v)
        ts_set_options(self.handle, self.options)

    def K(self, level=None):
        return ts_num_coeffs(self.handle, self.G if level is None else level)

    def _new(self, n, dtype=None):
        torch = self.torch
        return torch.empty(n, dtype=dtype or torch.float64, device="cuda")

    def _run(self, fn):
        torch = self.torch
        with torch.cuda.stream(self.stream):
            out = fn()
        self.stream.synchronize()
        return out

    def _dev(self, v, dtype):
        torch = self.torch
        return torch.as_tensor(v, dtype=dtype).to("cuda").contiguous()

    def rhs(self):
        def f():
            b = self._new(self.K())
            ts_rhs(self.handle, b)
            return b
        return self._run(f)

    def apply(self, level, c, fp32=False):
        torch = self.torch
        dt = torch.float32 if fp32 else torch.float64
        K = self.K(level)

        def f():
            cd = self._dev(c, dt)
            out = self._new(K, dt)
            (ts_apply_f32 if fp32 else ts_apply)(self.handle, level, _ptr(cd, dt, K), out)
            return out
        return self._run(f)

    def diag(self, level):
        def f():
            D = self._new(self.K(level))
            ts_diag(self.handle, level, D)
            return D
        return self._run(f)

    def omega(self, level):
        return ts_get_omega(self.handle, level)

    def bottom_level(self):
        """Level whose V-cycle runs as one dense operator (0: none)."""
        return ts_bottom_level(self.handle)

    def prolong(self, level, e):
        def f():
            ed = self._dev(e, self.torch.float64)
            out = self._new(self.K(level))
            ts_prolong(self.handle, level, _ptr(ed, numel=self.K(level - 1)), out)
            return out
        return self._run(f)

    def restrict(self, level, r):
        def f():
            rd = self._dev(r, self.torch.float64)
            out = self._new(self.K(level - 1))
            ts_restrict(self.handle, level, _ptr(rd, numel=self.K(level)), out)
            return out
        return self._run(f)

    def coarse_solve(self, b):
        def f():
            bd = self._dev(b, self.torch.float64)
            x = self._new(self.K(1))
            ts_coarse_solve(self.handle, _ptr(bd, numel=self.K(1)), x)
            return x
        return self._run(f)

    def vcycle(self, r, fp32=False):
        torch = self.torch
        dt = torch.float32 if fp32 else torch.float64

        def f():
            rd = self._dev(r, dt)
            z = self._new(self.K(), dt)
            (ts_vcycle_f32 if fp32 else ts_vcycle)(self.handle, _ptr(rd, dt, self.K()), z)
            return z
        return self._run(f)

    def solve(self, start=None):
        def f():
            if start is not None:
                alpha = self._dev(start, self.torch.float64).clone()
            else:
                alpha = self._new(self.K())
            status, info = ts_solve(self.handle, alpha, start is not None)
            return alpha, status, info.as_dict()
        return self._run(f)

    def evaluate(self, alpha, xq):
        def f():
            xd = self._dev(xq, self.torch.float64)
            m = xd.shape[0]
            yq = self._new(m)
            ts_evaluate(self.handle, _ptr(alpha, self.torch.float64, self.K()), m, xd, yq)
            return yq
        return self._run(f)
