"""Python binding of libamg.so (include/amg.h): argument marshalling only.

Every function has the C ABI's name.  Device vectors are passed as torch
tensors on the GPU (or raw device addresses as int); streams as
``torch.cuda.Stream`` or raw ``hipStream_t`` ints (None = the current torch
stream).  All computation happens in the HIP library; if ``libamg.so`` is
missing, importing this module raises instead of falling back to anything.
"""
from __future__ import annotations

import ctypes
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
# AMG_LIBRARY names another build of the same library (the host-sanitizer
# build of build.py); the default is the in-tree libamg.so
LIB_PATH = os.environ.get("AMG_LIBRARY") or os.path.join(_HERE, "libamg.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "amg.h")

AMG_OK, AMG_NOT_CONVERGED, AMG_DIVERGED = 0, 1, 2
AMG_EINVAL, AMG_ENOMEM, AMG_EHIP, AMG_ENOTSUP = -1, -2, -3, -4
AMG_K_CONST, AMG_K_WEIGHTED, AMG_K_FRACTIONAL, AMG_K_GENERATORS = 0, 1, 2, 3
AMG_K_WEAKLY_SINGULAR = 4
AMG_K_FRACTIONAL_NEAR = 5
AMG_FP64, AMG_MIXED = 0, 1
AMG_FLAG_HOST_ONLY = 1
AMG_FLAG_PROFILE = 2
AMG_FLAG_EAGER = 4
AMG_FLAG_ACCURATE_RESIDUAL = 8
AMG_FLAG_DEEP_FOLD = 16
AMG_INNER_VCYCLE, AMG_INNER_PCG, AMG_INNER_GMRES = 0, 1, 2
AMG_SCHEME_SHIFTED, AMG_SCHEME_STANDARD = 0, 1


class AmgError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {strerror(status)} (status {status})")
        self.status = status


class amg_kernel_t(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("alpha", ctypes.c_double), ("wl", ctypes.c_double),
                ("wr", ctypes.c_double), ("gen", ctypes.POINTER(ctypes.c_double)),
                ("scheme", ctypes.c_int), ("gamma", ctypes.c_double)]


class amg_opts_t(ctypes.Structure):
    _fields_ = [("m1", ctypes.c_int), ("m2", ctypes.c_int), ("omega_pre", ctypes.c_double),
                ("omega_post", ctypes.c_double), ("coarsest_log2", ctypes.c_int),
                ("precision", ctypes.c_int), ("max_iter", ctypes.c_int), ("flags", ctypes.c_int),
                ("inner", ctypes.c_int), ("shift", ctypes.c_double), ("scale", ctypes.c_double),
                ("restart", ctypes.c_int), ("cycle", ctypes.c_int)]


class amg_server_result_t(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("status", ctypes.c_int), ("iters", ctypes.c_int),
                ("relres", ctypes.c_double), ("cached", ctypes.c_int)]


class amg_server_stats_t(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in
                ("submitted", "finished", "rounds", "cache_hits", "cache_misses", "evictions",
                 "reserved_bytes", "peak_reserved_bytes", "cached_hierarchies",
                 "start_us", "rebuild_us", "rounds_us", "setup_us", "rebuilds")]


class amg_stat_t(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2202_11288_amd.build`")
    # One HIP runtime per process: torch ships its own libamdhip64, and a
    # library loaded before torch would bind a second copy from the ROCm
    # install, which then finds no device once torch's copy holds it.
    # Importing torch first lets libamg.so resolve to the copy torch loaded.
    try:
        import torch  # noqa: F401
    except ImportError:  # pragma: no cover - torch is a dependency of the binding
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P, D, I, I64 = ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_int64
    DP = ctypes.POINTER(ctypes.c_double)
    IP = ctypes.POINTER(ctypes.c_int)
    sig = {
        "amg_default_opts": (None, [ctypes.POINTER(amg_opts_t)]),
        "amg_setup": (I, [ctypes.POINTER(amg_kernel_t), D, I64, ctypes.POINTER(amg_opts_t), P,
                          ctypes.POINTER(P)]),
        "amg_matvec": (I, [P, P, P, P]),
        "amg_matvec_noalloc": (I, [P, P, P, P]),
        "amg_residual": (I, [P, P, P, P, P]),
        "amg_level_matvec": (I, [P, I, P, P, P]),
        "amg_level_matvec_f32": (I, [P, I, P, P, P]),
        "amg_vcycle": (I, [P, P, P, P]),
        "amg_solve": (I, [P, P, P, D, P, IP, DP]),
        "amg_residual_history": (I, [P, DP, I]),
        "amg_bdf4_step": (I, [P, P, P, P, P, P, P, D, P, IP, DP]),
        "amg_solve_batch": (I, [I, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P),
                                DP, P, IP, DP]),
        "amg_profile_stats": (I, [P, ctypes.POINTER(amg_stat_t), I, I]),
        "amg_num_levels": (I, [P]),
        "amg_level_size": (I64, [P, I]),
        "amg_level_tpx": (I, [P, I, DP, DP, DP, DP, DP, DP, DP, DP, DP]),
        "amg_level_band": (I, [P, I, DP, DP, DP]),
        "amg_manufactured_rhs": (I, [ctypes.POINTER(amg_kernel_t), D, I64, DP]),
        "amg_volume_reach": (I64, [ctypes.POINTER(amg_kernel_t), D, I64]),
        "amg_volume_rhs": (I, [ctypes.POINTER(amg_kernel_t), D, I64, DP, DP, DP]),
        "amg_footprint_bytes": (I64, [ctypes.POINTER(amg_kernel_t), D, I64,
                                      ctypes.POINTER(amg_opts_t)]),
        "amg_destroy": (I, [P]),
        "amg_server_create": (I, [I64, I, P, ctypes.POINTER(P)]),
        "amg_server_submit": (I, [P, ctypes.POINTER(amg_kernel_t), D, I64,
                                  ctypes.POINTER(amg_opts_t), P, P, D,
                                  ctypes.POINTER(ctypes.c_int64)]),
        "amg_server_step": (I, [P, I, IP, IP]),
        "amg_server_poll": (I, [P, ctypes.POINTER(amg_server_result_t), I]),
        "amg_server_stats": (I, [P, ctypes.POINTER(amg_server_stats_t)]),
        "amg_server_destroy": (I, [P]),
        "amg_server_lanes": (I, [P, ctypes.c_int64, I]),
        "amg_autotune": (I, [I, I, P]),
        "amg_plan_get": (I, [I, IP, IP, ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(ctypes.c_double), IP, IP]),
        "amg_plan_set": (I, [I, I, I]),
        "amg_strerror": (ctypes.c_char_p, [I]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def declared_symbols(header: str = HEADER):
    """Function names declared in include/amg.h."""
    txt = open(header).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(amg_[a-z0-9_]+)\s*\(", txt)))


def strerror(status: int) -> str:
    return lib.amg_strerror(int(status)).decode()


def _check(status: int, what: str, ok=(AMG_OK,)):
    if status not in ok:
        raise AmgError(status, what)
    return status


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return ctypes.c_void_p(t)
    return ctypes.c_void_p(t.data_ptr())


_PRECISION = {}  # handle address -> amg_precision of its setup (for amg_vcycle's dtype)


def _vec(h, t, what: str, level: int = 0, f32: bool = False):
    """A device vector argument: a raw address (int, passed as is) or a CUDA
    tensor that must be contiguous, of the level's length 2n+1 and float64
    (float32 where `f32`), so that the library never reads past it."""
    if t is None or isinstance(t, int):
        return _ptr(t)
    import torch
    m = lib.amg_level_size(h, int(level))
    want = torch.float32 if f32 else torch.float64
    if m < 0:
        raise AmgError(int(m), what)
    if not (t.is_cuda and t.is_contiguous() and t.dtype == want and t.numel() == m):
        raise ValueError(f"{what}: need a contiguous {want} CUDA tensor of {m} values, got "
                         f"{t.dtype} {tuple(t.shape)} on {t.device}"
                         f"{'' if t.is_contiguous() else ' (not contiguous)'}")
    return _ptr(t)


def _hkey(h):
    return h.value if isinstance(h, ctypes.c_void_p) else h


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def kernel(kind: int, alpha: float = 0.0, wl: float = 1.0, wr: float = 1.0, gen=None,
           scheme: int = AMG_SCHEME_SHIFTED, gamma: float = 0.0):
    """amg_kernel_t; for AMG_K_GENERATORS `gen` is a float64 numpy array that
    must stay alive until amg_setup returns."""
    k = amg_kernel_t(kind, alpha, wl, wr, None, scheme, gamma)
    if gen is not None:
        k.gen = gen.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return k


def amg_default_opts(**over) -> amg_opts_t:
    o = amg_opts_t()
    lib.amg_default_opts(ctypes.byref(o))
    fields = {name for name, _ in amg_opts_t._fields_}
    for k, v in over.items():
        if k not in fields:
            raise TypeError(f"amg_opts_t has no field {k!r}")
        setattr(o, k, v)
    return o


def amg_setup(kern: amg_kernel_t, delta: float, N: int, opts: amg_opts_t | None = None,
              stream=None):
    h = ctypes.c_void_p()
    host_only = opts is not None and (opts.flags & AMG_FLAG_HOST_ONLY)
    st = lib.amg_setup(ctypes.byref(kern), float(delta), int(N),
                       ctypes.byref(opts) if opts is not None else None,
                       None if host_only else _stream(stream), ctypes.byref(h))
    _check(st, "amg_setup")
    _PRECISION[h.value] = opts.precision if opts is not None else AMG_FP64
    return h


def amg_destroy(h):
    _PRECISION.pop(_hkey(h), None)
    return _check(lib.amg_destroy(h), "amg_destroy")


def amg_matvec(h, x, y, stream=None):
    return _check(lib.amg_matvec(h, _vec(h, x, "amg_matvec x"), _vec(h, y, "amg_matvec y"),
                                 _stream(stream)), "amg_matvec")


def amg_residual(h, b, x, r, stream=None):
    """r = b - A x, evaluated as the solve's outer residual."""
    return _check(lib.amg_residual(h, _vec(h, b, "amg_residual b"), _vec(h, x, "amg_residual x"),
                                   _vec(h, r, "amg_residual r"), _stream(stream)), "amg_residual")


def amg_matvec_noalloc(h, x, y, stream=None):
    """amg_matvec with the library's static work memory (N <= 2^18)."""
    return _check(lib.amg_matvec_noalloc(h, _vec(h, x, "amg_matvec_noalloc x"),
                                         _vec(h, y, "amg_matvec_noalloc y"), _stream(stream)),
                  "amg_matvec_noalloc")


def amg_level_matvec(h, level: int, x, y, stream=None):
    return _check(lib.amg_level_matvec(h, int(level), _vec(h, x, "amg_level_matvec x", level),
                                       _vec(h, y, "amg_level_matvec y", level), _stream(stream)),
                  "amg_level_matvec")


def amg_level_matvec_f32(h, level: int, x, y, stream=None):
    """FP32 level matvec of an AMG_MIXED handle; x, y float32."""
    return _check(lib.amg_level_matvec_f32(
        h, int(level), _vec(h, x, "amg_level_matvec_f32 x", level, f32=True),
        _vec(h, y, "amg_level_matvec_f32 y", level, f32=True), _stream(stream)),
        "amg_level_matvec_f32")


def amg_vcycle(h, r, e, stream=None):
    """r, e in the handle's V-cycle precision (float32 for AMG_MIXED)."""
    f32 = _PRECISION.get(_hkey(h), AMG_FP64) == AMG_MIXED
    return _check(lib.amg_vcycle(h, _vec(h, r, "amg_vcycle r", f32=f32),
                                 _vec(h, e, "amg_vcycle e", f32=f32), _stream(stream)), "amg_vcycle")


def amg_solve(h, b, x, tol: float, stream=None, allow=(AMG_OK,)):
    """Returns (status, iters, relres); raises unless status is in `allow`."""
    it = ctypes.c_int()
    rr = ctypes.c_double()
    st = lib.amg_solve(h, _vec(h, b, "amg_solve b"), _vec(h, x, "amg_solve x"), float(tol),
                       _stream(stream), ctypes.byref(it), ctypes.byref(rr))
    _check(st, "amg_solve", ok=allow)
    return st, it.value, rr.value


def amg_bdf4_step(h, hist, src, x, tol: float, stream=None, allow=(AMG_OK,)):
    """hist = (U^{k-1}, U^{k-2}, U^{k-3}, U^{k-4}); src = tau (F^k - E g^k) or
    None.  Returns (status, iters, relres)."""
    if len(hist) != 4:
        raise ValueError("BDF4 needs four previous time levels")
    it = ctypes.c_int()
    rr = ctypes.c_double()
    st = lib.amg_bdf4_step(h, *[_vec(h, u, "amg_bdf4_step history") for u in hist],
                           _vec(h, src, "amg_bdf4_step src"), _vec(h, x, "amg_bdf4_step x"),
                           float(tol), _stream(stream), ctypes.byref(it), ctypes.byref(rr))
    _check(st, "amg_bdf4_step", ok=allow)
    return st, it.value, rr.value


def amg_solve_batch(hs, bs, xs, tols, stream=None, allow=(AMG_OK,)):
    """Solve independent instances; returns (status, iters list, relres list)."""
    k = len(hs)
    H = (ctypes.c_void_p * k)(*[h.value if isinstance(h, ctypes.c_void_p) else h for h in hs])
    if not (len(bs) == k and len(xs) == k and len(tols) == k):
        raise ValueError("amg_solve_batch: one b, x and tol per handle")
    def addr(h, t, what):
        v = _vec(h, t, what)
        return None if v is None else v.value
    Bp = (ctypes.c_void_p * k)(*[addr(h, b, "amg_solve_batch b") for h, b in zip(hs, bs)])
    Xp = (ctypes.c_void_p * k)(*[addr(h, x, "amg_solve_batch x") for h, x in zip(hs, xs)])
    T = (ctypes.c_double * k)(*[float(t) for t in tols])
    it = (ctypes.c_int * k)()
    rr = (ctypes.c_double * k)()
    st = lib.amg_solve_batch(k, H, Bp, Xp, T, _stream(stream), it, rr)
    _check(st, "amg_solve_batch", ok=allow)
    return st, list(it), list(rr)


def amg_residual_history(h, cap: int = 100001):
    import numpy as np
    buf = np.zeros(cap)
    k = lib.amg_residual_history(h, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), cap)
    if k < 0:
        raise AmgError(k, "amg_residual_history")
    return buf[:k].copy()


def amg_profile_stats(h, reset: bool = False):
    """{name: (launches, total_ms)} recorded under AMG_FLAG_PROFILE."""
    arr = (amg_stat_t * 16)()
    k = lib.amg_profile_stats(h, arr, 16, int(bool(reset)))
    if k < 0:
        raise AmgError(k, "amg_profile_stats")
    return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms) for i in range(k)}


def amg_num_levels(h) -> int:
    return lib.amg_num_levels(h)


def amg_level_size(h, level: int) -> int:
    return lib.amg_level_size(h, int(level))


def amg_level_band(h, level: int):
    """(sub, main, sup) of the level's tridiagonal band, or None."""
    import numpy as np
    m = amg_level_size(h, level)
    if m < 0:
        raise AmgError(int(m), "amg_level_band")
    out = [np.zeros(m) for _ in range(3)]
    DP = ctypes.POINTER(ctypes.c_double)
    st = lib.amg_level_band(h, int(level), *[a.ctypes.data_as(DP) for a in out])
    if st < 0:
        raise AmgError(st, "amg_level_band")
    return tuple(out) if st == 1 else None


def amg_level_tpx(h, level: int):
    """dict with the level's generators a, b, c, d, Cross vectors p, q, xi,
    zeta and o (host copies)."""
    import numpy as np
    m = amg_level_size(h, level)
    if m < 0:
        raise AmgError(int(m), "amg_level_tpx")
    n = (m - 1) // 2
    arr = {k: np.zeros(2 * n - 1) for k in "abcd"}
    arr.update({k: np.zeros(n) for k in ("p", "q", "xi", "zeta")})
    o = ctypes.c_double()
    DP = ctypes.POINTER(ctypes.c_double)
    args = [arr[k].ctypes.data_as(DP) for k in ("a", "b", "c", "d", "p", "q", "xi", "zeta")]
    _check(lib.amg_level_tpx(h, int(level), *args, ctypes.byref(o)), "amg_level_tpx")
    arr["o"] = o.value
    arr["n"] = n
    return arr


def amg_manufactured_rhs(kern: amg_kernel_t, delta: float, N: int):
    import numpy as np
    b = np.zeros(2 * N - 1)
    _check(lib.amg_manufactured_rhs(ctypes.byref(kern), float(delta), int(N),
                                    b.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
           "amg_manufactured_rhs")
    return b


def amg_volume_reach(kern: amg_kernel_t, delta: float, N: int) -> int:
    S = lib.amg_volume_reach(ctypes.byref(kern), float(delta), int(N))
    if S < 0:
        raise AmgError(int(S), "amg_volume_reach")
    return int(S)


def amg_volume_rhs(kern: amg_kernel_t, delta: float, N: int, g_left, g_right, b):
    """b -= E g in place; g_left, g_right, b are contiguous float64 numpy
    arrays (S + 1, S + 1 and 2N - 1 values)."""
    import numpy as np
    S = amg_volume_reach(kern, delta, N)
    DP = ctypes.POINTER(ctypes.c_double)
    for name, a, m in (("g_left", g_left, S + 1), ("g_right", g_right, S + 1), ("b", b, 2 * N - 1)):
        if not (isinstance(a, np.ndarray) and a.dtype == np.float64 and a.flags.c_contiguous
                and a.shape == (m,)):
            raise ValueError(f"{name} must be a contiguous float64 array of {m} values")
    _check(lib.amg_volume_rhs(ctypes.byref(kern), float(delta), int(N), g_left.ctypes.data_as(DP),
                              g_right.ctypes.data_as(DP), b.ctypes.data_as(DP)), "amg_volume_rhs")
    return b


def amg_footprint_bytes(kern: amg_kernel_t, delta: float, N: int, opts: amg_opts_t | None = None):
    return lib.amg_footprint_bytes(ctypes.byref(kern), float(delta), int(N),
                                   ctypes.byref(opts) if opts is not None else None)


# ---- serving ---------------------------------------------------------------

def amg_server_create(mem_budget_bytes: int, workers: int = 4, stream=None):
    sv = ctypes.c_void_p()
    _check(lib.amg_server_create(int(mem_budget_bytes), int(workers), _stream(stream),
                                 ctypes.byref(sv)), "amg_server_create")
    return sv


def amg_server_submit(sv, kern: amg_kernel_t, delta: float, N: int, b, x, tol: float,
                      opts: amg_opts_t | None = None) -> int:
    """Queue a request; b, x are contiguous float64 CUDA tensors of 2N - 1
    values that must stay alive until the request is polled."""
    import torch
    m = 2 * int(N) - 1
    for name, t in (("b", b), ("x", x)):
        if not (t.is_cuda and t.is_contiguous() and t.dtype == torch.float64 and t.numel() == m):
            raise ValueError(f"amg_server_submit {name}: need a contiguous float64 CUDA tensor "
                             f"of {m} values")
    rid = ctypes.c_int64()
    _check(lib.amg_server_submit(sv, ctypes.byref(kern), float(delta), int(N),
                                 ctypes.byref(opts) if opts is not None else None, _ptr(b), _ptr(x),
                                 float(tol), ctypes.byref(rid)), "amg_server_submit")
    return rid.value


def amg_server_step(sv, rounds: int = 1):
    """Returns (in_flight, waiting)."""
    a, w = ctypes.c_int(), ctypes.c_int()
    _check(lib.amg_server_step(sv, int(rounds), ctypes.byref(a), ctypes.byref(w)),
           "amg_server_step")
    return a.value, w.value


def amg_server_poll(sv, cap: int = 4096):
    """[(id, status, iters, relres, cached)] of the requests finished since the
    last poll."""
    arr = (amg_server_result_t * cap)()
    k = lib.amg_server_poll(sv, arr, cap)
    if k < 0:
        raise AmgError(k, "amg_server_poll")
    return [(arr[i].id, arr[i].status, arr[i].iters, arr[i].relres, arr[i].cached)
            for i in range(k)]


def amg_server_stats(sv) -> dict:
    st = amg_server_stats_t()
    _check(lib.amg_server_stats(sv, ctypes.byref(st)), "amg_server_stats")
    return {name: getattr(st, name) for name, _ in amg_server_stats_t._fields_}


def amg_server_destroy(sv):
    return _check(lib.amg_server_destroy(sv), "amg_server_destroy")


def amg_autotune(logL_min: int = 13, logL_max: int = 23, stream=None):
    """Time every candidate geometry of the level matvec for the sizes
    2^logL_min .. 2^logL_max and select the fastest (process-wide)."""
    _check(lib.amg_autotune(int(logL_min), int(logL_max), _stream(stream)), "amg_autotune")


def amg_plan_get(logL: int):
    """The geometry in use for size 2^logL and the tuner's record of it."""
    l1, tc, cand, rej = (ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int())
    ud, ub = ctypes.c_double(), ctypes.c_double()
    _check(lib.amg_plan_get(int(logL), ctypes.byref(l1), ctypes.byref(tc), ctypes.byref(ud),
                            ctypes.byref(ub), ctypes.byref(cand), ctypes.byref(rej)),
           "amg_plan_get")
    return {"logL": int(logL), "logL1": l1.value, "tcols": tc.value, "us_default": ud.value,
            "us_best": ub.value, "candidates": cand.value, "rejected": rej.value}


def amg_plan_set(logL: int, logL1: int = 0, tcols: int = 0):
    """Select a candidate geometry for size 2^logL (logL1 = 0: the default)."""
    _check(lib.amg_plan_set(int(logL), int(logL1), int(tcols)), "amg_plan_set")


def amg_server_lanes(sv, small_max_N: int, small_rounds: int = 3):
    """Requests with N <= small_max_N get their own lane (stream) and
    small_rounds rounds per round of the others; 0 = one lane."""
    _check(lib.amg_server_lanes(sv, int(small_max_N), int(small_rounds)), "amg_server_lanes")
