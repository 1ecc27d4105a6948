"""Thin ctypes binding of libpmf (include/pmf.h): same names, argument marshalling
only.  Every step of the filter runs in the HIP library; nothing here computes.

Models and priors are taken from any object with the fields of ``pmf_model`` /
``pmf_prior`` (``nx, A, Q, N, grid, ...``; ``w, mean, cov``).  Streams are HIP
stream handles: a ``torch.cuda.Stream``, its integer ``cuda_stream``, or None.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpmf.so")

PMF_OK, PMF_E_INVALID, PMF_E_NOMEM, PMF_E_DEVICE, PMF_E_DEGENERATE, PMF_E_BUSY = 0, 1, 2, 3, 4, 5
PMF_W_BOUNDARY = 64
PMF_FP64, PMF_FP32 = 0, 1
PMF_STATE_MAGIC = 0x504D4631


PMF_MAX_NX, PMF_MAX_TERRAIN = 4, 8
PMF_H_TERRAIN = 3


class pmf_model(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("A", C.c_double * 16), ("Q", C.c_double * 16), ("grid", C.c_int),
        ("N", C.c_int * 4), ("span_sigmas", C.c_double), ("t_nominal", C.c_double),
        ("integrator", C.c_int), ("substeps", C.c_int), ("precision", C.c_int), ("interp", C.c_int),
        ("meas_kind", C.c_int), ("nz", C.c_int), ("H", C.c_double * 12), ("hparam", C.c_double * 4),
        ("nterrain", C.c_int), ("terrain", C.c_double * (PMF_MAX_TERRAIN * 6)),
        ("noise_ncomp", C.c_int), ("noise_w", C.c_double * 4), ("noise_mean", C.c_double * 12),
        ("noise_cov", C.c_double * 36),
    ]


class pmf_prior(C.Structure):
    _fields_ = [("ncomp", C.c_int), ("w", C.c_double * 4), ("mean", C.c_double * 16),
                ("cov", C.c_double * 64)]


class pmf_state_header(C.Structure):
    _fields_ = [("magic", C.c_uint), ("version", C.c_int), ("nx", C.c_int), ("grid", C.c_int),
                ("precision", C.c_int), ("status", C.c_int), ("N", C.c_int * 4),
                ("c", C.c_double * 4), ("M", C.c_double * 16), ("t", C.c_double)]


PMF_OP_PREDICT, PMF_OP_UPDATE = 0, 1


class pmf_completion(C.Structure):
    _fields_ = [("tag", C.c_longlong), ("track", C.c_int), ("op", C.c_int), ("status", C.c_int),
                ("fused", C.c_int), ("loglik", C.c_double), ("latency_us", C.c_double)]


class pmf_server_stats(C.Structure):
    _fields_ = [("budget_bytes", C.c_size_t), ("used_bytes", C.c_size_t), ("tracks", C.c_int),
                ("waiting_tracks", C.c_int), ("submitted", C.c_longlong), ("completed", C.c_longlong),
                ("rounds", C.c_longlong), ("fused_ops", C.c_longlong), ("single_ops", C.c_longlong),
                ("admitted_late", C.c_longlong)]


class PmfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"pmf status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libpmf.so; fails loudly when the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2412_07240_amd.build` (hipcc, gfx950)")
        # torch's wheel carries its own HIP runtime under the system runtime's
        # soname.  Loaded first, it is the one copy libpmf.so binds to; loaded
        # after libpmf.so, it would be a second runtime in the process, and the
        # second of two runtimes to initialise finds no GPU.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, ip, dp = C.c_void_p, C.c_int, C.POINTER(C.c_double)
        sig = {
            "pmf_model_check": (ip, [C.POINTER(pmf_model), C.POINTER(C.c_int), C.c_char_p, C.c_size_t]),
            "pmf_ctx_create": (ip, [ip, C.POINTER(pmf_allocator), C.POINTER(vp)]),
            "pmf_ctx_destroy": (None, [vp]),
            "pmf_create": (ip, [vp, C.POINTER(pmf_model), C.POINTER(pmf_prior), C.POINTER(vp)]),
            "pmf_destroy": (None, [vp]),
            "pmf_predict": (ip, [vp, C.c_double, vp]),
            "pmf_update": (ip, [vp, dp, dp, vp]),
            "pmf_moments": (ip, [vp, dp, dp, vp]),
            "pmf_sync_status": (ip, [vp, vp]),
            "pmf_last_substeps": (ip, [vp, C.POINTER(C.c_int)]),
            "pmf_get_state": (ip, [vp, vp, C.POINTER(C.c_size_t)]),
            "pmf_set_state": (ip, [vp, vp, C.c_size_t]),
            "pmf_batch_step": (ip, [vp, C.POINTER(vp), ip, C.c_double, dp, dp, vp]),
            "pmf_batch_step_noalloc": (ip, [vp, C.POINTER(vp), ip, C.c_double, dp, dp, vp]),
            "pmf_batch_run": (ip, [vp, C.POINTER(vp), ip, C.c_double, ip, dp, dp, vp]),
            "pmf_density_ptr": (vp, [vp]),
            "pmf_stream_sync": (ip, [vp]),
            "pmf_batch_profile": (ip, [vp, ip]),
            "pmf_batch_kernel_time": (ip, [vp, dp, C.POINTER(C.c_int)]),
            "pmf_autotune": (ip, [vp, C.POINTER(C.c_int), ip, C.c_char_p, C.c_char_p, C.c_size_t]),
            "pmf_get_schedule": (ip, [vp, ip, ip, C.POINTER(C.c_int)]),
            "pmf_set_schedule": (ip, [vp, ip, ip, ip]),
            "pmf_last_error": (C.c_char_p, []),
            "pmf_server_create": (ip, [vp, C.c_size_t, ip, C.POINTER(vp)]),
            "pmf_server_destroy": (None, [vp]),
            "pmf_server_add_track": (ip, [vp, C.POINTER(pmf_model), C.POINTER(pmf_prior), C.POINTER(C.c_int)]),
            "pmf_server_remove_track": (ip, [vp, ip]),
            "pmf_server_submit": (ip, [vp, ip, ip, C.c_double, dp, C.c_longlong]),
            "pmf_server_submit_cycle": (ip, [vp, ip, C.c_double, dp, C.c_longlong]),
            "pmf_server_poll": (ip, [vp, C.POINTER(pmf_completion), ip, C.POINTER(C.c_int)]),
            "pmf_server_drain": (ip, [vp]),
            "pmf_server_stats_get": (ip, [vp, C.POINTER(pmf_server_stats)]),
            "pmf_server_filter": (vp, [vp, ip]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


EXPORTED = ("pmf_model_check", "pmf_ctx_create", "pmf_ctx_destroy", "pmf_create", "pmf_destroy", "pmf_predict",
            "pmf_update", "pmf_moments", "pmf_sync_status", "pmf_last_substeps", "pmf_get_state",
            "pmf_set_state", "pmf_batch_step", "pmf_batch_step_noalloc", "pmf_batch_run", "pmf_density_ptr", "pmf_stream_sync", "pmf_batch_profile",
            "pmf_batch_kernel_time", "pmf_autotune", "pmf_get_schedule", "pmf_set_schedule", "pmf_last_error", "pmf_server_create", "pmf_server_destroy",
            "pmf_server_add_track", "pmf_server_remove_track", "pmf_server_submit", "pmf_server_submit_cycle", "pmf_server_poll",
            "pmf_server_drain", "pmf_server_stats_get", "pmf_server_filter")


def pmf_last_error() -> str:
    return lib().pmf_last_error().decode()


def _check(status: int, ok=(PMF_OK,)):
    if status not in ok:
        raise PmfError(status, pmf_last_error())
    return status


def _stream(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _fill(arr, values):
    flat = np.asarray(values, dtype=float).ravel()
    for i, v in enumerate(flat):
        arr[i] = float(v)


def make_model(spec) -> pmf_model:
    m = pmf_model()
    nx = int(spec.nx)
    m.nx = nx
    _fill(m.A, np.asarray(spec.A, float).reshape(nx, nx))
    _fill(m.Q, np.asarray(spec.Q, float).reshape(nx, nx))
    m.grid = int(spec.grid)
    _fill_int = list(spec.N)[:nx] + [1] * (4 - nx)
    for i in range(4):
        m.N[i] = int(_fill_int[i])
    m.span_sigmas = float(spec.span_sigmas)
    m.t_nominal = float(spec.t_nominal)
    m.integrator = int(spec.integrator)
    m.substeps = int(spec.substeps)
    m.precision = int(spec.precision)
    m.interp = int(spec.interp)
    m.meas_kind = int(spec.meas_kind)
    m.nz = int(spec.nz)
    if int(spec.meas_kind) == 0:
        _fill(m.H, np.asarray(spec.H, float).reshape(m.nz, nx))
    _fill(m.hparam, np.asarray(spec.hparam, float).ravel()[:4])
    terr = getattr(spec, "terrain", None)
    if int(spec.meas_kind) == PMF_H_TERRAIN and terr is not None:
        terr = np.asarray(terr, float).reshape(-1, 2 + nx)
        m.nterrain = len(terr)
        for c, row in enumerate(terr):
            for i, v in enumerate(row):
                m.terrain[6 * c + i] = float(v)
    w = np.asarray(spec.noise_w, float).ravel()
    m.noise_ncomp = len(w)
    _fill(m.noise_w, w)
    means = np.asarray(spec.noise_mean, float).reshape(len(w), -1)
    covs = np.asarray(spec.noise_cov, float).reshape(len(w), m.nz, m.nz)
    for g in range(len(w)):
        for i in range(m.nz):
            m.noise_mean[3 * g + i] = means[g, i]
            for j in range(m.nz):
                m.noise_cov[9 * g + i * m.nz + j] = covs[g, i, j]
    return m


def make_prior(spec, nx: int) -> pmf_prior:
    p = pmf_prior()
    w = np.asarray(spec.w, float).ravel()
    p.ncomp = len(w)
    _fill(p.w, w)
    means = np.asarray(spec.mean, float).reshape(len(w), nx)
    covs = np.asarray(spec.cov, float).reshape(len(w), nx, nx)
    for g in range(len(w)):
        for i in range(nx):
            p.mean[4 * g + i] = means[g, i]
            for j in range(nx):
                p.cov[16 * g + i * nx + j] = covs[g, i, j]
    return p


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class pmf_allocator(C.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", C.c_void_p)]


_ctx_allocators = {}   # context -> (allocator struct, callbacks): kept alive with the context


def torch_allocator(device: int = 0, counter: dict | None = None):
    """A pmf_allocator whose calls go to PyTorch's caching allocator on `device`
    (torch.cuda.caching_allocator_alloc / caching_allocator_delete).  counter, if
    given, counts the calls ("alloc", "free", "bytes")."""
    import torch

    def _alloc(nbytes, user, stream):
        try:
            p = torch.cuda.caching_allocator_alloc(int(nbytes), device=device)
        except RuntimeError:
            return None
        if counter is not None:
            counter["alloc"] = counter.get("alloc", 0) + 1
            counter["bytes"] = counter.get("bytes", 0) + int(nbytes)
        return p

    def _free(ptr, user, stream):
        if ptr:
            torch.cuda.caching_allocator_delete(int(ptr))
            if counter is not None:
                counter["free"] = counter.get("free", 0) + 1

    fa, ff = _ALLOC_FN(_alloc), _FREE_FN(_free)
    return pmf_allocator(fa, ff, None), (fa, ff)


def pmf_ctx_create(device: int = 0, allocator=None):
    """allocator: None (hipMalloc / hipFree), "torch" (PyTorch's caching allocator)
    or a (pmf_allocator, callbacks) pair as torch_allocator returns."""
    out = C.c_void_p()
    if allocator is None:
        _check(lib().pmf_ctx_create(device, None, C.byref(out)))
        return out
    if allocator == "torch":
        allocator = torch_allocator(device)
    a, keep = allocator
    _check(lib().pmf_ctx_create(device, C.byref(a), C.byref(out)))
    _ctx_allocators[out.value] = (a, keep)
    return out


def pmf_ctx_destroy(ctx) -> None:
    lib().pmf_ctx_destroy(ctx)
    _ctx_allocators.pop(getattr(ctx, "value", ctx), None)


def pmf_model_check(model):
    """(fusable, reason) for a valid model (reason "" when fusable); raises
    PmfError for a model pmf_create would refuse.  Host only: no device is used."""
    m = make_model(model)
    fus = C.c_int(0)
    buf = C.create_string_buffer(512)
    _check(lib().pmf_model_check(C.byref(m), C.byref(fus), buf, len(buf)))
    return bool(fus.value), buf.value.decode()


def pmf_create(ctx, model, prior):
    out = C.c_void_p()
    m = make_model(model)
    p = make_prior(prior, int(model.nx))
    _check(lib().pmf_create(ctx, C.byref(m), C.byref(p), C.byref(out)))
    return out


def pmf_destroy(f) -> None:
    lib().pmf_destroy(f)


def pmf_predict(f, T: float, stream=None) -> None:
    _check(lib().pmf_predict(f, float(T), _stream(stream)))


def pmf_update(f, z, stream=None, want_loglik: bool = False):
    """Enqueue the update; with want_loglik the stream is synchronised and
    log p(z | past) is returned."""
    zz = np.ascontiguousarray(np.atleast_1d(np.asarray(z, float)))
    zp = zz.ctypes.data_as(C.POINTER(C.c_double))
    if not want_loglik:
        _check(lib().pmf_update(f, zp, None, _stream(stream)))
        return None
    ll = C.c_double(float("nan"))
    _check(lib().pmf_update(f, zp, C.byref(ll), _stream(stream)))
    _check(lib().pmf_stream_sync(_stream(stream)))
    return ll.value


def pmf_moments(f, nx: int, stream=None):
    """(mean, cov, status) of the current density; status carries the warning bits."""
    mean = np.zeros(nx)
    cov = np.zeros((nx, nx))
    st = lib().pmf_moments(f, mean.ctypes.data_as(C.POINTER(C.c_double)),
                           cov.ctypes.data_as(C.POINTER(C.c_double)), _stream(stream))
    if st & ~(PMF_W_BOUNDARY | PMF_E_DEGENERATE):
        raise PmfError(st, pmf_last_error())
    return mean, cov, st


def pmf_sync_status(f, stream=None) -> int:
    st = lib().pmf_sync_status(f, _stream(stream))
    if st & ~(PMF_W_BOUNDARY | PMF_E_DEGENERATE):
        raise PmfError(st, pmf_last_error())
    return st


def pmf_last_substeps(f) -> int:
    l = C.c_int()
    _check(lib().pmf_last_substeps(f, C.byref(l)))
    return l.value


def pmf_get_state(f):
    """(header, c, M, t, density ndarray) of the current state."""
    nbytes = C.c_size_t(0)
    _check(lib().pmf_get_state(f, None, C.byref(nbytes)))
    buf = (C.c_ubyte * nbytes.value)()
    _check(lib().pmf_get_state(f, buf, C.byref(nbytes)))
    h = pmf_state_header.from_buffer_copy(buf)
    nx = h.nx
    shape = tuple(h.N[i] for i in range(nx))
    dt = np.float64 if h.precision == PMF_FP64 else np.float32
    off = C.sizeof(pmf_state_header)
    P = np.frombuffer(bytes(buf)[off:], dtype=dt, count=int(np.prod(shape))).reshape(shape).copy()
    c = np.array(h.c[:nx])
    M = np.array(h.M[:]).reshape(4, 4)[:nx, :nx].copy()
    return h, c, M, h.t, P


def pmf_set_state(f, c, M, t, P, grid: int, precision: int) -> None:
    """Replace grid (c, M, t) and density P of a filter of the same kind."""
    P = np.ascontiguousarray(P, dtype=np.float64 if precision == PMF_FP64 else np.float32)
    nx = P.ndim
    h = pmf_state_header()
    h.magic = PMF_STATE_MAGIC
    h.version = 2
    h.nx = nx
    h.grid = int(grid)
    h.precision = int(precision)
    for i in range(4):
        h.N[i] = P.shape[i] if i < nx else 1
    Mm = np.asarray(M, float).reshape(nx, nx)
    for i in range(nx):
        h.c[i] = float(c[i])
        for j in range(nx):
            h.M[4 * i + j] = float(Mm[i, j])
    h.t = float(t)
    blob = bytes(h) + P.tobytes()
    buf = (C.c_ubyte * len(blob)).from_buffer_copy(blob)
    _check(lib().pmf_set_state(f, buf, len(blob)))


class FilterArray:
    """A list of filter handles marshalled once for repeated pmf_batch_step calls."""

    def __init__(self, filters):
        self.n = len(filters)
        self.arr = (C.c_void_p * self.n)(*[f.value for f in filters])


def pmf_batch_step(ctx, filters, T: float, z, stream=None, want_loglik: bool = False):
    """filters: a list of handles or a FilterArray (cheaper when called every step)."""
    fa = filters if isinstance(filters, FilterArray) else FilterArray(filters)
    n = fa.n
    zz = np.ascontiguousarray(np.asarray(z, float).reshape(n, -1))
    ll = np.full(n, np.nan) if want_loglik else None
    _check(lib().pmf_batch_step(ctx, fa.arr, n, float(T), zz.ctypes.data_as(C.POINTER(C.c_double)),
                                ll.ctypes.data_as(C.POINTER(C.c_double)) if want_loglik else None,
                                _stream(stream)))
    if want_loglik:
        _check(lib().pmf_stream_sync(_stream(stream)))
    return ll


def pmf_batch_run(ctx, filters, T: float, z, stream=None):
    """K cycles at once from z of shape (K, n, nz_max), or (K, n) when every nz is 1
    (one captured graph, synchronous); returns the (K, n) log-likelihoods."""
    fa = filters if isinstance(filters, FilterArray) else FilterArray(filters)
    n = fa.n
    zz = np.asarray(z, float)
    if zz.ndim == 2:
        zz = zz[:, :, None]
    if zz.ndim != 3 or zz.shape[1] != n:
        raise ValueError(f"z must have shape (K, {n}, nz_max) or (K, {n}), not {np.shape(z)}")
    zz = np.ascontiguousarray(zz)
    K = zz.shape[0]
    ll = np.full((K, n), np.nan)
    _check(lib().pmf_batch_run(ctx, fa.arr, n, float(T), K, zz.ctypes.data_as(C.POINTER(C.c_double)),
                               ll.ctypes.data_as(C.POINTER(C.c_double)), _stream(stream)))
    return ll


def pmf_batch_step_noalloc(ctx, filters, T: float, z, stream=None):
    """The allocation-free batched step (synchronous); returns the log-likelihoods."""
    fa = filters if isinstance(filters, FilterArray) else FilterArray(filters)
    n = fa.n
    zz = np.ascontiguousarray(np.asarray(z, float).reshape(n, -1))
    ll = np.full(n, np.nan)
    _check(lib().pmf_batch_step_noalloc(ctx, fa.arr, n, float(T), zz.ctypes.data_as(C.POINTER(C.c_double)),
                                        ll.ctypes.data_as(C.POINTER(C.c_double)), _stream(stream)))
    return ll


def pmf_density_ptr(f) -> int:
    return lib().pmf_density_ptr(f)


def pmf_stream_sync(stream=None) -> None:
    _check(lib().pmf_stream_sync(_stream(stream)))


def pmf_batch_profile(ctx, enable: bool) -> None:
    _check(lib().pmf_batch_profile(ctx, 1 if enable else 0))


def pmf_batch_kernel_time(ctx):
    """(summed event time in ms, launches) of batched steps since the last call."""
    ms = C.c_double(0.0)
    n = C.c_int(0)
    _check(lib().pmf_batch_kernel_time(ctx, C.byref(ms), C.byref(n)))
    return ms.value, n.value


TUNE_SIZES = (32, 48, 64, 96, 128)


def pmf_autotune(ctx, counts=None, steps: int = 10, cache_path=None) -> str:
    """Tune the fused kernel's schedule variants for a mix of 2-D sizes: counts
    maps N (32, 48, 64, 96, 128) to the number of N x N filters in the caller's
    batches (None: 1024 each); or read the schedules from the JSON cache at
    cache_path.  Returns the library's text report."""
    arr = None
    if counts is not None:
        arr = (C.c_int * 5)(*[int(counts.get(N, 0)) for N in TUNE_SIZES])
    buf = C.create_string_buffer(4096)
    path = None if cache_path is None else os.fsencode(cache_path)
    _check(lib().pmf_autotune(ctx, arr, int(steps), path, buf, len(buf)))
    return buf.value.decode()


def pmf_get_schedule(ctx, nx: int, N: int) -> int:
    v = C.c_int(0)
    _check(lib().pmf_get_schedule(ctx, int(nx), int(N), C.byref(v)))
    return v.value


def pmf_set_schedule(ctx, nx: int, N: int, variant: int) -> None:
    _check(lib().pmf_set_schedule(ctx, int(nx), int(N), int(variant)))


# ------------------------------------------------------------------ serving

def pmf_server_create(ctx, budget_bytes: int, max_tracks: int):
    out = C.c_void_p()
    _check(lib().pmf_server_create(ctx, int(budget_bytes), int(max_tracks), C.byref(out)))
    return out


def pmf_server_destroy(s) -> None:
    lib().pmf_server_destroy(s)


def pmf_server_add_track(s, model, prior) -> int:
    m = make_model(model)
    p = make_prior(prior, model.nx)
    t = C.c_int(-1)
    _check(lib().pmf_server_add_track(s, C.byref(m), C.byref(p), C.byref(t)))
    return t.value


def pmf_server_remove_track(s, track: int) -> None:
    _check(lib().pmf_server_remove_track(s, int(track)))


def pmf_server_submit(s, track: int, op: int, T: float = 0.0, z=None, tag: int = 0) -> None:
    zp = None
    if z is not None:
        zz = np.ascontiguousarray(np.asarray(z, float).ravel())
        zp = zz.ctypes.data_as(C.POINTER(C.c_double))
    _check(lib().pmf_server_submit(s, int(track), int(op), float(T), zp, int(tag)))


def pmf_server_submit_cycle(s, track: int, T: float, z, tag: int = 0) -> None:
    zz = np.ascontiguousarray(np.asarray(z, float).ravel())
    _check(lib().pmf_server_submit_cycle(s, int(track), float(T), zz.ctypes.data_as(C.POINTER(C.c_double)),
                                         int(tag)))


def pmf_server_poll(s, cap: int = 4096):
    """Completions as a list of dicts (oldest first)."""
    buf = (pmf_completion * cap)()
    n = C.c_int(0)
    _check(lib().pmf_server_poll(s, buf, cap, C.byref(n)))
    return [{"tag": c.tag, "track": c.track, "op": c.op, "status": c.status, "fused": c.fused,
             "loglik": c.loglik, "latency_us": c.latency_us} for c in buf[:n.value]]


def pmf_server_drain(s) -> None:
    _check(lib().pmf_server_drain(s))


def pmf_server_stats_get(s) -> dict:
    st = pmf_server_stats()
    _check(lib().pmf_server_stats_get(s, C.byref(st)))
    return {k: getattr(st, k) for k, _ in pmf_server_stats._fields_}


def pmf_server_filter(s, track: int):
    p = lib().pmf_server_filter(s, int(track))
    return C.c_void_p(p) if p else None
