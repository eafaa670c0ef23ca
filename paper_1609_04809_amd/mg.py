"""ctypes binding of libmg.so (the C ABI in include/mg.h).

Argument marshalling only: every step of the solver runs in the HIP
library.  PyTorch supplies device memory (CUDA/HIP tensors) and the current
stream.  The library must have been built (``python -m
paper_1609_04809_amd.build``); importing this module without it raises.
"""

import ctypes
import os

import numpy as np
import torch  # loaded before libmg.so so that both share one HIP runtime

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "lib", "libmg.so")

MG_OK, MG_E_ARG, MG_E_NOMEM, MG_E_HIP, MG_E_NOT_SPD = 0, 1, 2, 3, 4
MG_E_MAXIT, MG_E_DIVERGED, MG_E_NONFINITE, MG_E_STATE = 5, 6, 7, 8
STATUS_NAMES = {0: "ok", 1: "arg", 2: "nomem", 3: "hip", 4: "not_spd",
                5: "maxit", 6: "diverged", 7: "nonfinite", 8: "state"}

OP = {"stencil": 0, "csr": 1}
SMOOTHER = {"jacobi": 0, "rbgs": 1, "gs": 2}
PREC = {"fp64": 0, "fp32_ir": 1}
CYCLE = {"V": 0, "W": 1, "F": 2}
FLAG_NO_GRAPH = 1
FLAG_NO_TAIL = 2
FLAG_NO_FUSE = 4
FLAG_PCG = 8
FLAG_PAIR = 16
FLAG_WARM = 32
FLAG_NO_SPLIT = 64

# mg_apply_smooth steps
STEP_JACOBI, STEP_RB0, STEP_RB1, STEP_RB_PRE, STEP_RB_POST = 0, 1, 2, 3, 4
STEP_GS0 = 5          # STEP_GS0 + c: multicolour Gauss-Seidel update of colour c
# mg_profile_enable kernel ids
(PROF_SMOOTH, PROF_RESID, PROF_RESTRICT, PROF_PROLONG, PROF_PAIR, PROF_SMOOTH_PRO,
 PROF_SMOOTH_IR, PROF_RESID_RESTRICT, PROF_SMOOTH_ZERO) = 0, 1, 2, 3, 4, 5, 6, 7, 8


class MgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int), ("levels", ctypes.c_int),
                ("op", ctypes.c_int), ("smoother", ctypes.c_int),
                ("nu_pre", ctypes.c_int), ("nu_post", ctypes.c_int),
                ("omega", ctypes.c_double), ("precision", ctypes.c_int),
                ("max_iter", ctypes.c_int), ("flags", ctypes.c_int), ("cycle", ctypes.c_int),
                ("sigma", ctypes.c_double)]


_VP = ctypes.c_void_p
_I = ctypes.c_int

# name -> (restype, argtypes); every exported symbol of include/mg.h
SIGNATURES = {
    "mg_options_default": (None, [ctypes.POINTER(Options)]),
    "mg_footprint_bytes": (ctypes.c_size_t, [ctypes.POINTER(Options)]),
    "mg_setup": (_I, [ctypes.POINTER(Options), _VP, _VP, ctypes.POINTER(_VP)]),
    "mg_solve": (_I, [_VP, _VP, _VP, ctypes.c_double, ctypes.POINTER(_I),
                      ctypes.POINTER(ctypes.c_double), _VP]),
    "mg_destroy": (None, [_VP]),
    "mg_last_error": (ctypes.c_char_p, []),
    "mg_level_info": (_I, [_VP, _I, ctypes.POINTER(_I), ctypes.POINTER(ctypes.c_size_t)]),
    "mg_apply_residual": (_I, [_VP, _I, _I, _VP, _VP, _VP, _VP]),
    "mg_apply_smooth": (_I, [_VP, _I, _I, _I, _VP, _VP, _VP, _VP]),
    "mg_apply_restrict": (_I, [_VP, _I, _I, _VP, _VP, _VP]),
    "mg_apply_residual_restrict": (_I, [_VP, _I, _I, _VP, _VP, _VP, _VP]),
    "mg_apply_prolong_add": (_I, [_VP, _I, _I, _VP, _VP, _VP]),
    "mg_apply_coarse_solve": (_I, [_VP, _I, _VP, _VP, _VP]),
    "mg_vcycle": (_I, [_VP, _I, _VP, _VP, _VP]),
    "mg_norm2": (_I, [_VP, _I, _I, _VP, ctypes.POINTER(ctypes.c_double), _VP]),
    "mg_cn_rhs": (_I, [_VP, _VP, _VP, _VP, ctypes.c_double, _VP, ctypes.c_double, _VP,
                       ctypes.c_double, _VP, _VP]),
    "mg_apply_mass": (_I, [_VP, _VP, _VP, _VP]),
    "mg_solve_noalloc": (_I, [ctypes.POINTER(Options), _VP, _VP, _VP, ctypes.c_double,
                              ctypes.POINTER(_I), ctypes.POINTER(ctypes.c_double), _VP]),
    "mg_profile_enable": (_I, [_VP, _I, _I]),
    "mg_profile_read": (_I, [_VP, ctypes.POINTER(ctypes.c_long),
                             ctypes.POINTER(ctypes.c_double)]),
}


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("admitted", ctypes.c_uint64),
                ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("launches", ctypes.c_uint64), ("fused_ops", ctypes.c_uint64),
                ("steps", ctypes.c_uint64), ("busy_s", ctypes.c_double),
                ("hbm_in_use", ctypes.c_size_t), ("hbm_peak", ctypes.c_size_t),
                ("in_flight", ctypes.c_int), ("queued", ctypes.c_int)]


_DP = ctypes.POINTER(ctypes.c_double)
SERVER_SIGNATURES = {
    "mg_server_create": (_I, [ctypes.c_size_t, _I, ctypes.POINTER(_VP)]),
    "mg_server_submit": (_I, [_VP, ctypes.POINTER(Options), _DP, _DP, _DP, ctypes.c_double,
                              ctypes.POINTER(ctypes.c_uint64)]),
    "mg_server_poll": (_I, [_VP, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(_I),
                            ctypes.POINTER(_I), _DP, _DP, _I, ctypes.POINTER(_I)]),
    "mg_server_drain": (_I, [_VP, ctypes.c_double]),
    "mg_server_get_stats": (_I, [_VP, ctypes.POINTER(ServerStats)]),
    "mg_server_destroy": (None, [_VP]),
}


def load_library(path=LIB_PATH):
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with `python -m paper_1609_04809_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in {**SIGNATURES, **SERVER_SIGNATURES}.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


def _check(st):
    if st != MG_OK:
        raise MgError(st, lib().mg_last_error().decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return ctypes.c_void_p(t.data_ptr())


def make_options(dim, n, levels, op="stencil", smoother="rbgs", nu_pre=2, nu_post=2,
                 omega=2.0 / 3.0, precision="fp64", max_iter=100, flags=0, cycle="V",
                 sigma=0.0):
    o = Options()
    lib().mg_options_default(ctypes.byref(o))
    o.dim, o.n, o.levels = dim, n, levels
    o.op, o.smoother = OP[op], SMOOTHER[smoother]
    o.nu_pre, o.nu_post, o.omega = nu_pre, nu_post, omega
    o.precision, o.max_iter, o.flags = PREC[precision], max_iter, flags
    o.cycle = CYCLE[cycle] if isinstance(cycle, str) else cycle
    o.sigma = sigma
    return o


def footprint_bytes(**kw):
    return lib().mg_footprint_bytes(ctypes.byref(make_options(**kw)))


class Solver:
    """One context: a level hierarchy resident on the current device."""

    def __init__(self, dim, n, levels, kappa=None, **kw):
        self.dim, self.n, self.levels = dim, n, levels
        self.opts = make_options(dim, n, levels, **kw)
        self.precision = kw.get("precision", "fp64")
        self.max_iter = self.opts.max_iter
        kdev = None
        if kappa is not None:
            kdev = torch.as_tensor(np.asarray(kappa, dtype=np.float64)
                                   if not torch.is_tensor(kappa) else kappa,
                                   dtype=torch.float64, device="cuda").contiguous()
        ctx = ctypes.c_void_p()
        st = lib().mg_setup(ctypes.byref(self.opts), _ptr(kdev), _stream(), ctypes.byref(ctx))
        _check(st)
        self._ctx = ctx

    # -- lifecycle
    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            torch.cuda.synchronize()
            lib().mg_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- info
    def level_n(self, level):
        n = ctypes.c_int()
        nodes = ctypes.c_size_t()
        _check(lib().mg_level_info(self._ctx, level, ctypes.byref(n), ctypes.byref(nodes)))
        return n.value

    def nodes(self, level=0):
        n = self.level_n(level)
        return (n + 1) ** self.dim

    # -- solve
    def solve(self, b, tol, u=None, raise_on_error=False):
        """Solve with b a device float64 tensor of (n+1)^dim nodes (u: the
        output, and with FLAG_WARM the initial iterate).
        Returns (u, iters, hist, status_name)."""
        if u is None:
            if self.opts.flags & FLAG_WARM:
                raise ValueError("a warm-started solve needs u")
            u = torch.empty_like(b)
        iters = ctypes.c_int()
        hist = (ctypes.c_double * (self.max_iter + 1))()
        st = lib().mg_solve(self._ctx, _ptr(b), _ptr(u), float(tol), ctypes.byref(iters),
                            hist, _stream())
        if st not in (MG_OK, MG_E_MAXIT, MG_E_DIVERGED) or (raise_on_error and st != MG_OK):
            _check(st)
        k = iters.value
        return u, k, list(hist[: k + 1]), STATUS_NAMES[st]

    def cn_rhs(self, u, g0=None, c0=0.0, g1=None, c1=0.0, F=None, cf=0.0, b=None, guess=None):
        """Crank-Nicolson right-hand side b = (sigma M - K) x0 - (sigma M +
        K) x1 + cf F (x0 = u inside, c0 g0 on the boundary; x1 = c1 g1 on
        the boundary; F a load vector); with `guess` (the solution one step
        back) also guess <- 2 u - guess.  Device float64 node tensors, None
        for absent data."""
        if b is None:
            b = torch.empty_like(u)
        _check(lib().mg_cn_rhs(self._ctx, _ptr(u), _ptr(guess), _ptr(g0), float(c0), _ptr(g1),
                               float(c1), _ptr(F), float(cf), _ptr(b), _stream()))
        return b

    def mass(self, f, F=None):
        """Load vector F = M f of nodal values f (device float64 node tensor)."""
        if F is None:
            F = torch.empty_like(f)
        _check(lib().mg_apply_mass(self._ctx, _ptr(f), _ptr(F), _stream()))
        return F

    # -- single steps
    def _prec(self, t):
        return PREC["fp64"] if t.dtype == torch.float64 else PREC["fp32_ir"]

    def residual(self, level, x, b, r):
        _check(lib().mg_apply_residual(self._ctx, level, self._prec(x), _ptr(x), _ptr(b),
                                       _ptr(r), _stream()))
        return r

    def smooth(self, level, step, x_in, b, x_out):
        _check(lib().mg_apply_smooth(self._ctx, level, self._prec(b), step, _ptr(x_in),
                                     _ptr(b), _ptr(x_out), _stream()))
        return x_out

    def restrict(self, level, r, bc):
        _check(lib().mg_apply_restrict(self._ctx, level, self._prec(r), _ptr(r), _ptr(bc),
                                       _stream()))
        return bc

    def residual_restrict(self, level, x, b, bc):
        _check(lib().mg_apply_residual_restrict(self._ctx, level, self._prec(x), _ptr(x),
                                                _ptr(b), _ptr(bc), _stream()))
        return bc

    def prolong_add(self, level, e, x):
        _check(lib().mg_apply_prolong_add(self._ctx, level, self._prec(x), _ptr(e), _ptr(x),
                                          _stream()))
        return x

    def coarse_solve(self, bc, xc):
        _check(lib().mg_apply_coarse_solve(self._ctx, self._prec(bc), _ptr(bc), _ptr(xc),
                                           _stream()))
        return xc

    def vcycle(self, x, b):
        _check(lib().mg_vcycle(self._ctx, self._prec(x), _ptr(x), _ptr(b), _stream()))
        return x

    def norm2(self, level, v):
        out = ctypes.c_double()
        _check(lib().mg_norm2(self._ctx, level, self._prec(v), _ptr(v), ctypes.byref(out),
                              _stream()))
        return out.value

    # -- kernel timing
    def profile(self, kernel_id, enable=True):
        _check(lib().mg_profile_enable(self._ctx, kernel_id, 1 if enable else 0))

    def profile_read(self):
        n = ctypes.c_long()
        ms = ctypes.c_double()
        _check(lib().mg_profile_read(self._ctx, ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value


def solve_noalloc(dim, n, levels, b, tol, u=None, kappa=None, **kw):
    """mg_solve_noalloc: one solve of a small hierarchy without a context or
    any device allocation by the library (b, u, kappa: device float64
    tensors).  Returns (u, iters, hist, status_name) like Solver.solve."""
    o = make_options(dim, n, levels, **kw)
    if u is None:
        u = torch.empty_like(b)
    iters = ctypes.c_int()
    hist = (ctypes.c_double * (o.max_iter + 1))()
    st = lib().mg_solve_noalloc(ctypes.byref(o), _ptr(kappa), _ptr(b), _ptr(u), float(tol),
                                ctypes.byref(iters), hist, _stream())
    if st not in (MG_OK, MG_E_MAXIT, MG_E_DIVERGED):
        _check(st)
    k = iters.value
    return u, k, list(hist[: k + 1]), STATUS_NAMES[st]


class Server:
    """Continuous-batching solve server (mg_server_* in the C ABI).

    Requests are host arrays; results land in host arrays owned by this
    object until they are collected with :meth:`poll`."""

    def __init__(self, hbm_budget_bytes, max_slots=64):
        srv = ctypes.c_void_p()
        _check(lib().mg_server_create(int(hbm_budget_bytes), int(max_slots), ctypes.byref(srv)))
        self._srv = srv
        self._pending = {}   # id -> (u_host, b_host, kappa_host) kept alive until done

    def submit(self, dim, n, levels, b_full, tol, kappa=None, **kw):
        """b_full: float64 host array of (n+1)^dim nodes.  Returns the id."""
        o = make_options(dim, n, levels, **kw)
        b = np.ascontiguousarray(b_full, dtype=np.float64)
        if b.size != (n + 1) ** dim:
            raise ValueError("b has the wrong size")
        k = None if kappa is None else np.ascontiguousarray(kappa, dtype=np.float64)
        u = np.empty_like(b)
        rid = ctypes.c_uint64()
        _check(lib().mg_server_submit(
            self._srv, ctypes.byref(o), b.ctypes.data_as(_DP),
            None if k is None else k.ctypes.data_as(_DP), u.ctypes.data_as(_DP),
            float(tol), ctypes.byref(rid)))
        self._pending[rid.value] = u
        return rid.value

    def poll(self, max_items=4096):
        """Finished requests: list of dicts (id, u, iters, status, rel_residual,
        latency_us)."""
        ids = (ctypes.c_uint64 * max_items)()
        iters = (ctypes.c_int * max_items)()
        st = (ctypes.c_int * max_items)()
        rho = (ctypes.c_double * max_items)()
        lat = (ctypes.c_double * max_items)()
        n = ctypes.c_int()
        _check(lib().mg_server_poll(self._srv, ids, iters, st, rho, lat, max_items,
                                    ctypes.byref(n)))
        out = []
        for q in range(n.value):
            out.append(dict(id=ids[q], u=self._pending.pop(ids[q]), iters=iters[q],
                            status=STATUS_NAMES.get(st[q], st[q]), rel_residual=rho[q],
                            latency_us=lat[q]))
        return out

    def drain(self, timeout_s=600.0):
        _check(lib().mg_server_drain(self._srv, float(timeout_s)))

    def stats(self):
        s = ServerStats()
        _check(lib().mg_server_get_stats(self._srv, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_srv", None) is not None and self._srv.value:
            lib().mg_server_destroy(self._srv)
            self._srv = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
