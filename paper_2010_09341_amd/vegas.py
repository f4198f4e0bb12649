"""Python binding of libvegas.so: the C interface of include/vegas.h, one
function per C entry point under the same name, marshalling arguments only.

PyTorch supplies the device memory (a workspace tensor bound to each handle)
and the HIP stream (a torch stream bound to each handle). Every step of the
computation runs in the library's HIP kernels; if the library is missing this
module raises instead of computing anything itself.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvegas.so")

VEGAS_OK, VEGAS_EINVAL, VEGAS_ENOMEM, VEGAS_EDEVICE = 0, -1, -2, -3
VEGAS_ESTATE, VEGAS_ENONFINITE, VEGAS_EBUSY, VEGAS_ECOMPILE = -4, -5, -6, -7
VEGAS_FP64, VEGAS_FP32_EVAL = 0, 1
(VEGAS_F_CONST, VEGAS_F_SUM, VEGAS_F_GAUSS, VEGAS_F_LO_TOY, VEGAS_F_RAMBO24,
 VEGAS_F_BW_FLAT) = range(6)
VEGAS_MAX_DIM, VEGAS_MAX_BINS, VEGAS_MAX_CELLS = 32, 512, 8192
VEGAS_MAX_PARAMS, VEGAS_MAX_RUN_ITER = 33, 1024
VEGAS_F_USER, VEGAS_MAX_USER, VEGAS_MAX_USER_PARAMS = 64, 64, 32


class VegasError(RuntimeError):
    def __init__(self, code: int, what: str, log: str = ""):
        self.code = code
        self.log = log
        msg = f"{what}: {strerror(code)} ({code})"
        super().__init__(msg + ("\n" + log if log else ""))


_lib = None
_lock = threading.Lock()

_c = ctypes
_vp = _c.c_void_p
_pd = _c.POINTER(_c.c_double)
_i64 = _c.c_int64
_u64 = _c.c_uint64

_SIGS = {
    "vegas_create": ([_c.c_int, _c.c_int, _c.POINTER(_vp)]),
    "vegas_destroy": ([_vp]),
    "vegas_reset": ([_vp]),
    "vegas_set_params": ([_vp, _c.c_int, _pd, _c.c_int]),
    "vegas_set_precision": ([_vp, _c.c_int]),
    "vegas_bind_stream": ([_vp, _vp]),
    "vegas_workspace_bytes": ([_c.c_int, _c.c_int, _c.POINTER(_c.c_size_t)]),
    "vegas_bind_workspace": ([_vp, _vp, _c.c_size_t]),
    "vegas_iterate": ([_vp, _c.c_int, _i64, _u64, _pd, _pd]),
    "vegas_refine": ([_vp, _c.c_double]),
    "vegas_run": ([_vp, _c.c_int, _i64, _u64, _c.c_int, _c.c_double, _pd, _pd]),
    "vegas_result": ([_vp, _pd, _pd, _pd]),
    "vegas_get_grid": ([_vp, _pd, _c.c_size_t]),
    "vegas_set_grid": ([_vp, _pd, _c.c_size_t]),
    "vegas_get_hist": ([_vp, _pd, _c.c_size_t]),
    "vegas_set_hist": ([_vp, _pd, _c.c_size_t]),
    "vegas_get_iteration": ([_vp, _c.POINTER(_c.c_uint32)]),
    "vegas_set_iteration": ([_vp, _c.c_uint32]),
    "vegas_nonfinite": ([_vp, _c.POINTER(_i64)]),
    "vegas_dump_weights": ([_vp, _c.c_int, _u64, _u64, _i64, _pd]),
    "vegas_set_launch": ([_vp, _c.c_int, _c.c_int]),
    "vegas_timing": ([_vp, _c.c_int, _c.c_int, _pd, _c.POINTER(_i64)]),
    "vegas_set_graph": ([_vp, _c.c_int]),
    "vegas_set_events_limit": ([_vp, _i64]),
    "vegas_state_bytes": ([_vp, _c.POINTER(_c.c_size_t)]),
    "vegas_save": ([_vp, _vp, _c.c_size_t]),
    "vegas_load": ([_vp, _vp, _c.c_size_t]),
    "vegas_integrand_compile": ([_c.c_char_p, _c.c_int, _c.POINTER(_c.c_int), _c.c_char_p,
                                 _c.c_size_t]),
    "vegas_server_create": ([_c.c_size_t, _c.c_int, _i64, _c.POINTER(_vp)]),
    "vegas_server_submit": ([_vp, _vp, _c.POINTER(_u64)]),
    "vegas_server_wait": ([_vp, _u64, _c.c_double, _pd, _pd, _pd, _pd]),
    "vegas_server_iterations": ([_vp, _u64, _pd, _pd]),
    "vegas_server_release": ([_vp, _u64]),
    "vegas_server_stats": ([_vp, _c.POINTER(_i64), _c.POINTER(_i64), _c.POINTER(_i64),
                            _c.POINTER(_i64)]),
    "vegas_server_destroy": ([_vp]),
    "vegas_server_set_graph": ([_vp, _c.c_int]),
    "vegas_server_ticks": ([_vp, _c.POINTER(_i64), _c.POINTER(_i64)]),
    "vegas_iterate_noalloc": ([_c.c_int, _c.c_int, _c.c_int, _c.c_int, _pd, _c.c_int, _vp,
                               _i64, _u64, _c.c_uint32, _vp, _vp, _vp]),
    "vegas_server_set_chain": ([_vp, _c.c_int]),
    "vegas_server_chains": ([_vp, _c.POINTER(_i64)]),
    "vegas_server_set_lanes": ([_vp, _c.c_int]),
}


def lib():
    """Load libvegas.so (built by `python -m paper_2010_09341_amd.build`)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"{LIB_PATH} is missing: build it with "
                                  "`python -m paper_2010_09341_amd.build`")
            # torch ships its own HIP runtime under the same shared-object
            # name as the system one; loading torch first makes the library
            # bind to that runtime, so that both share one (loading the
            # library first has left torch without a usable GPU)
            import torch  # noqa: F401
            L = ctypes.CDLL(LIB_PATH)
            for name, args in _SIGS.items():
                try:
                    fn = getattr(L, name)
                except AttributeError:
                    continue  # reported by the export test; calling it raises
                fn.argtypes = args
                fn.restype = _c.c_int
            L.vegas_strerror.argtypes = [_c.c_int]
            L.vegas_strerror.restype = _c.c_char_p
            _lib = L
    return _lib


def strerror(code: int) -> str:
    try:
        return lib().vegas_strerror(code).decode()
    except ImportError:
        return str(code)


def _check(rc: int, what: str, ok=(VEGAS_OK,)):
    if rc not in ok:
        raise VegasError(rc, what)
    return rc


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_pd)


class Handle:
    """An opaque vegas_h plus the torch objects that back it."""

    def __init__(self, ptr, dim, n_bins, workspace=None, stream=None):
        self.ptr = ptr
        self.dim = dim
        self.n_bins = n_bins
        self.workspace = workspace
        self.stream = stream

    @property
    def _as_parameter_(self):
        return self.ptr

    def __del__(self):
        try:
            if self.ptr:
                vegas_destroy(self)
        except Exception:
            pass


def vegas_workspace_bytes(dim: int, n_bins: int) -> int:
    n = _c.c_size_t()
    _check(lib().vegas_workspace_bytes(dim, n_bins, _c.byref(n)), "vegas_workspace_bytes")
    return n.value


def vegas_create(dim: int, n_bins: int, torch_memory: bool = True) -> Handle:
    """Create a handle; by default its workspace is a torch tensor on the
    current device and its stream a torch stream."""
    out = _vp()
    _check(lib().vegas_create(dim, n_bins, _c.byref(out)), "vegas_create")
    h = Handle(out.value, dim, n_bins)
    if torch_memory:
        import torch
        nbytes = vegas_workspace_bytes(dim, n_bins)
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        base = ws.data_ptr()
        aligned = (base + 255) & ~255
        vegas_bind_workspace(h, aligned, nbytes)
        h.workspace = ws
        st = torch.cuda.Stream()
        vegas_bind_stream(h, st.cuda_stream)
        h.stream = st
    return h


def vegas_destroy(h: Handle):
    if h.ptr:
        rc = lib().vegas_destroy(h.ptr)
        h.ptr = None
        _check(rc, "vegas_destroy")


def vegas_reset(h: Handle):
    _check(lib().vegas_reset(h), "vegas_reset")


def vegas_set_params(h: Handle, integrand_id: int, params=None):
    p = np.ascontiguousarray(params if params is not None else [], dtype=np.float64)
    _check(lib().vegas_set_params(h, integrand_id, _dptr(p) if p.size else None, int(p.size)),
           "vegas_set_params")


def vegas_set_precision(h: Handle, prec: int):
    _check(lib().vegas_set_precision(h, prec), "vegas_set_precision")


def vegas_bind_stream(h: Handle, stream):
    ptr = stream if isinstance(stream, int) or stream is None else stream.cuda_stream
    _check(lib().vegas_bind_stream(h, ptr), "vegas_bind_stream")


def vegas_bind_workspace(h: Handle, dev_ptr: int, nbytes: int):
    _check(lib().vegas_bind_workspace(h, dev_ptr, nbytes), "vegas_bind_workspace")


def vegas_iterate(h: Handle, integrand_id: int, n_events: int, seed: int):
    """(I, sigma) of one iteration. Non-finite weights do not raise: see
    vegas_nonfinite."""
    I = _c.c_double()
    s = _c.c_double()
    _check(lib().vegas_iterate(h, integrand_id, n_events, seed, _c.byref(I), _c.byref(s)),
           "vegas_iterate", ok=(VEGAS_OK, VEGAS_ENONFINITE))
    return I.value, s.value


def vegas_refine(h: Handle, alpha: float):
    _check(lib().vegas_refine(h, alpha), "vegas_refine")


def vegas_run(h: Handle, integrand_id: int, n_events: int, seed: int, n_iter: int,
              alpha: float):
    """Per-iteration (I_t, sigma_t) arrays of a whole run."""
    I_t = np.zeros(n_iter)
    s_t = np.zeros(n_iter)
    _check(lib().vegas_run(h, integrand_id, n_events, seed, n_iter, alpha, _dptr(I_t),
                           _dptr(s_t)), "vegas_run", ok=(VEGAS_OK, VEGAS_ENONFINITE))
    return I_t, s_t


def vegas_result(h: Handle):
    I, s, c = _c.c_double(), _c.c_double(), _c.c_double()
    _check(lib().vegas_result(h, _c.byref(I), _c.byref(s), _c.byref(c)), "vegas_result")
    return I.value, s.value, c.value


def vegas_get_grid(h: Handle):
    e = np.zeros((h.dim, h.n_bins + 1))
    _check(lib().vegas_get_grid(h, _dptr(e), e.size), "vegas_get_grid")
    return e


def vegas_set_grid(h: Handle, edges):
    e = np.ascontiguousarray(edges, dtype=np.float64)
    _check(lib().vegas_set_grid(h, _dptr(e), e.size), "vegas_set_grid")


def vegas_get_hist(h: Handle):
    a = np.zeros((h.dim, h.n_bins))
    _check(lib().vegas_get_hist(h, _dptr(a), a.size), "vegas_get_hist")
    return a


def vegas_set_hist(h: Handle, hist):
    a = np.ascontiguousarray(hist, dtype=np.float64)
    _check(lib().vegas_set_hist(h, _dptr(a), a.size), "vegas_set_hist")


def vegas_get_iteration(h: Handle) -> int:
    t = _c.c_uint32()
    _check(lib().vegas_get_iteration(h, _c.byref(t)), "vegas_get_iteration")
    return t.value


def vegas_set_iteration(h: Handle, t: int):
    _check(lib().vegas_set_iteration(h, t), "vegas_set_iteration")


def vegas_nonfinite(h: Handle) -> int:
    n = _i64()
    _check(lib().vegas_nonfinite(h, _c.byref(n)), "vegas_nonfinite")
    return n.value


def vegas_dump_weights(h: Handle, integrand_id: int, seed: int, first: int, count: int):
    w = np.zeros(count)
    _check(lib().vegas_dump_weights(h, integrand_id, seed, first, count,
                                    _dptr(w) if count else None), "vegas_dump_weights")
    return w


def vegas_iterate_noalloc(dim: int, n_bins: int, prec: int, integrand_id: int, params,
                          edges_dev: int, n_events: int, seed: int, t: int, hist_dev: int,
                          result_dev: int, stream: int = 0):
    """One iteration that allocates nothing: device pointers (ints) for the
    edges, the histogram (0: none) and the 4 result values; `stream` a raw
    hipStream_t (torch.cuda.Stream.cuda_stream). Asynchronous."""
    p = np.ascontiguousarray(params if params is not None else [], dtype=np.float64)
    _check(lib().vegas_iterate_noalloc(dim, n_bins, prec, integrand_id,
                                       _dptr(p) if p.size else None, int(p.size),
                                       _vp(edges_dev), n_events, seed, t,
                                       _vp(hist_dev) if hist_dev else None, _vp(result_dev),
                                       _vp(stream) if stream else None),
           "vegas_iterate_noalloc")


def vegas_set_launch(h: Handle, max_blocks: int = 0, threads: int = 0):
    _check(lib().vegas_set_launch(h, max_blocks, threads), "vegas_set_launch")


def vegas_state_bytes(h: Handle) -> int:
    n = _c.c_size_t()
    _check(lib().vegas_state_bytes(h, _c.byref(n)), "vegas_state_bytes")
    return n.value


def vegas_save(h: Handle) -> bytes:
    n = vegas_state_bytes(h)
    buf = _c.create_string_buffer(n)
    _check(lib().vegas_save(h, buf, n), "vegas_save")
    return buf.raw


def vegas_load(h: Handle, state: bytes):
    buf = _c.create_string_buffer(bytes(state), len(state))
    _check(lib().vegas_load(h, buf, len(state)), "vegas_load")


def vegas_integrand_compile(source: str, dim: int = 0) -> int:
    """Compile HIP device source defining vegas_user_f64 / vegas_user_f32
    into a run-time integrand id; raises VegasError carrying the compiler log
    if it does not compile."""
    fid = _c.c_int(-1)
    log = _c.create_string_buffer(1 << 16)
    rc = lib().vegas_integrand_compile(source.encode(), dim, _c.byref(fid), log, len(log))
    if rc != VEGAS_OK:
        raise VegasError(rc, "vegas_integrand_compile", log.value.decode(errors="replace"))
    return fid.value


def vegas_set_events_limit(h: Handle, limit: int):
    _check(lib().vegas_set_events_limit(h, limit), "vegas_set_events_limit")


def vegas_set_graph(h: Handle, enable: bool):
    _check(lib().vegas_set_graph(h, int(enable)), "vegas_set_graph")


def vegas_timing(h: Handle, enable: bool, reset: bool = False):
    """(summed iteration-kernel milliseconds, launches) since the last reset."""
    ms = _c.c_double()
    n = _i64()
    _check(lib().vegas_timing(h, int(enable), int(reset), _c.byref(ms), _c.byref(n)),
           "vegas_timing")
    return ms.value, n.value


# ---- serving -----------------------------------------------------------------
class vegas_request(ctypes.Structure):
    _fields_ = [("dim", _c.c_int), ("n_bins", _c.c_int), ("integrand_id", _c.c_int),
                ("n_params", _c.c_int), ("params", _pd), ("n_events", _i64),
                ("n_iter", _c.c_int), ("alpha", _c.c_double), ("seed", _u64),
                ("prec", _c.c_int)]


class Server:
    """An opaque vegas_server."""

    def __init__(self, ptr):
        self.ptr = ptr

    @property
    def _as_parameter_(self):
        return self.ptr

    def __del__(self):
        try:
            if self.ptr:
                vegas_server_destroy(self)
        except Exception:
            pass


def vegas_server_create(mem_budget_bytes: int, max_slots: int, chunk_events: int = 0) -> Server:
    out = _vp()
    _check(lib().vegas_server_create(mem_budget_bytes, max_slots, chunk_events, _c.byref(out)),
           "vegas_server_create")
    return Server(out.value)


def vegas_server_submit(s: Server, dim: int, n_bins: int, integrand_id: int, params,
                        n_events: int, n_iter: int, alpha: float, seed: int,
                        prec: int = VEGAS_FP32_EVAL) -> int:
    p = np.ascontiguousarray(params if params is not None else [], dtype=np.float64)
    req = vegas_request(dim, n_bins, integrand_id, int(p.size), _dptr(p) if p.size else None,
                        n_events, n_iter, alpha, seed, prec)
    t = _u64()
    _check(lib().vegas_server_submit(s, _c.byref(req), _c.byref(t)), "vegas_server_submit")
    return t.value


def vegas_server_wait(s: Server, ticket: int, timeout_s: float = -1.0):
    """(I, sigma, chi2_dof, latency_s) of a finished request."""
    I, sg, c2, lat = _c.c_double(), _c.c_double(), _c.c_double(), _c.c_double()
    _check(lib().vegas_server_wait(s, ticket, timeout_s, _c.byref(I), _c.byref(sg), _c.byref(c2),
                                   _c.byref(lat)), "vegas_server_wait",
           ok=(VEGAS_OK, VEGAS_ENONFINITE))
    return I.value, sg.value, c2.value, lat.value


def vegas_server_iterations(s: Server, ticket: int, n_iter: int):
    I_t = np.zeros(n_iter)
    s_t = np.zeros(n_iter)
    _check(lib().vegas_server_iterations(s, ticket, _dptr(I_t), _dptr(s_t)),
           "vegas_server_iterations")
    return I_t, s_t


def vegas_server_release(s: Server, ticket: int):
    _check(lib().vegas_server_release(s, ticket), "vegas_server_release")


def vegas_server_stats(s: Server):
    """(completed, events, work_items, peak_active)."""
    v = [_i64() for _ in range(4)]
    _check(lib().vegas_server_stats(s, *[_c.byref(x) for x in v]), "vegas_server_stats")
    return tuple(x.value for x in v)


def vegas_server_set_graph(s: Server, enable: bool):
    _check(lib().vegas_server_set_graph(s, int(enable)), "vegas_server_set_graph")


def vegas_server_ticks(s: Server):
    """(ticks, graph_ticks)."""
    a, b = _i64(), _i64()
    _check(lib().vegas_server_ticks(s, _c.byref(a), _c.byref(b)), "vegas_server_ticks")
    return a.value, b.value


def vegas_server_set_chain(s: Server, max_ticks: int):
    _check(lib().vegas_server_set_chain(s, int(max_ticks)), "vegas_server_set_chain")


def vegas_server_set_lanes(s: Server, lanes: int):
    _check(lib().vegas_server_set_lanes(s, int(lanes)), "vegas_server_set_lanes")


def vegas_server_chains(s: Server) -> int:
    a = _i64()
    _check(lib().vegas_server_chains(s, _c.byref(a)), "vegas_server_chains")
    return a.value


def vegas_server_destroy(s: Server):
    if s.ptr:
        rc = lib().vegas_server_destroy(s.ptr)
        s.ptr = None
        _check(rc, "vegas_server_destroy")
