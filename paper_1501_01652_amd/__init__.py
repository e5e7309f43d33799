"""Python binding of libhank: fast order-0 Bessel sums on MI355X.

    f_k = sum_n c_n J_0(r_k w_n)

for Schlomilch expansions, Fourier-Bessel expansions and the order-0 discrete
Hankel transform (Townsend, "A fast analysis-based discrete Hankel transform
using asymptotic expansions").  Every function here only marshals arguments
into the C ABI of ``include/hank.h``; all arithmetic runs in the library's HIP
kernels.  Tensors are PyTorch tensors on the GPU (PyTorch supplies device
memory and streams, nothing else).  The library must be built first
(``paper_1501_01652_amd.build.build()``); without it every call raises.
"""
from __future__ import annotations

import ctypes
import os
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("HANK_LIB") or os.path.join(_HERE, "libhank.so")

TASKS = {"schlomilch": 0, "fourier_bessel": 1, "dht0": 2,
         "schlomilch_paper_grid": 3, "fourier_bessel_paper_grid": 4}

STATUS = {0: "HANK_OK", 1: "HANK_EINVAL", 2: "HANK_ENOMEM", 3: "HANK_EDEVICE", 4: "HANK_EUNSUPPORTED"}

EXPORTS = ["hank_schlomilch", "hank_fourier_bessel", "hank_dht0", "hank_transform", "hank_batch",
           "hank_last_error", "hank_cache_clear", "hank_cache_bytes", "hank_param_s", "hank_param_t",
           "hank_param_neumann", "hank_param_pK", "hank_param_qT", "hank_plan_info",
           "hank_plan_block", "hank_root_offsets", "hank_j0", "hank_profile", "hank_profile_report",
           "hank_server_create", "hank_server_warm", "hank_server_submit", "hank_server_start",
           "hank_server_drain", "hank_server_status", "hank_server_stats", "hank_server_destroy",
           "hank_batch_graph_create", "hank_batch_graph_launch", "hank_batch_graph_destroy",
           "hank_autotune", "hank_autotune_reset", "hank_dht0_inverse", "hank_dht0_weights",
           "hank_transform_noalloc", "hank_cache_limit", "hank_autotune_save", "hank_autotune_load"]


class HankError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS.get(status, str(status)), message))
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("plan_mode", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("direct", ctypes.c_int32), ("prefer_far", ctypes.c_int32), ("nrhs", ctypes.c_int32),
                ("M", ctypes.c_int32), ("nu", ctypes.c_int32), ("shift", ctypes.c_int32)]


class PlanSummary(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("K", ctypes.c_int32), ("T", ctypes.c_int32),
                ("P", ctypes.c_int32), ("nblocks", ctypes.c_int32), ("s", ctypes.c_double),
                ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("near_entries", ctypes.c_int64), ("far_transforms", ctypes.c_int64),
                ("fft_points", ctypes.c_int64), ("fft_bytes", ctypes.c_double),
                ("first_direct", ctypes.c_int32), ("bulk_fp32", ctypes.c_int32),
                ("fp32_transforms", ctypes.c_int32), ("model_s", ctypes.c_double)]


class BlockInfo(ctypes.Structure):
    _fields_ = [("row0", ctypes.c_int64), ("row1", ctypes.c_int64), ("col0", ctypes.c_int64),
                ("col1", ctypes.c_int64), ("fft_len", ctypes.c_int64), ("groups", ctypes.c_int32),
                ("terms", ctypes.c_int32), ("zmin", ctypes.c_double), ("fft_l1", ctypes.c_int32),
                ("fft_l2", ctypes.c_int32)]


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("bytes", ctypes.c_double), ("work", ctypes.c_double)]


class Request(ctypes.Structure):
    _fields_ = [("task", ctypes.c_int32), ("precision", ctypes.c_int32), ("N", ctypes.c_int64),
                ("nrhs", ctypes.c_int64), ("ldc", ctypes.c_int64), ("ldo", ctypes.c_int64),
                ("eps", ctypes.c_double), ("c", ctypes.c_void_p), ("out", ctypes.c_void_p),
                ("nu", ctypes.c_int32), ("shift", ctypes.c_int32)]


_lib = None
_lock = threading.Lock()


def lib():
    """The loaded C library (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError("libhank.so is missing: build it with "
                                   "paper_1501_01652_amd.build.build()")
            L = ctypes.CDLL(LIB_PATH)
            i32, i64, d, p = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
            for name in ("hank_schlomilch", "hank_fourier_bessel", "hank_dht0"):
                f = getattr(L, name)
                f.restype = i32
                f.argtypes = [p, i64, d, p, p]
            L.hank_transform.restype = i32
            L.hank_transform.argtypes = [i32, p, i64, i64, i64, d, p, i64, ctypes.POINTER(Options), p]
            L.hank_transform_noalloc.restype = i32
            L.hank_transform_noalloc.argtypes = [i32, p, i64, i64, i64, d, p, i64, ctypes.POINTER(Options), p]
            L.hank_batch.restype = i32
            L.hank_batch.argtypes = [ctypes.POINTER(Request), i64, p]
            L.hank_batch_graph_create.restype = i32
            L.hank_batch_graph_create.argtypes = [ctypes.POINTER(Request), i64, p, ctypes.POINTER(p)]
            L.hank_batch_graph_launch.restype = i32
            L.hank_batch_graph_launch.argtypes = [p, p]
            L.hank_batch_graph_destroy.restype = i32
            L.hank_batch_graph_destroy.argtypes = [p]
            L.hank_autotune.restype = i32
            L.hank_autotune.argtypes = [p, ctypes.POINTER(i32)]
            L.hank_autotune_reset.restype = i32
            L.hank_autotune_reset.argtypes = []
            for name in ("hank_autotune_save", "hank_autotune_load"):
                f = getattr(L, name)
                f.restype = i32
                f.argtypes = [ctypes.c_char_p]
            L.hank_last_error.restype = ctypes.c_char_p
            L.hank_last_error.argtypes = []
            L.hank_cache_clear.restype = i32
            L.hank_cache_bytes.restype = i64
            L.hank_cache_limit.restype = i32
            L.hank_cache_limit.argtypes = [i64]
            for name in ("hank_param_s", "hank_param_t"):
                f = getattr(L, name)
                f.restype = d
                f.argtypes = [i32, i32, d]
            for name in ("hank_param_neumann", "hank_param_pK", "hank_param_qT"):
                f = getattr(L, name)
                f.restype = d
                f.argtypes = [i32, d]
            L.hank_plan_info.restype = i32
            L.hank_plan_info.argtypes = [i32, i64, d, ctypes.POINTER(Options), ctypes.POINTER(PlanSummary)]
            L.hank_plan_block.restype = i32
            L.hank_plan_block.argtypes = [i32, i64, d, ctypes.POINTER(Options), i32,
                                          ctypes.POINTER(BlockInfo)]
            L.hank_root_offsets.restype = i32
            L.hank_root_offsets.argtypes = [i64, p, p]
            L.hank_dht0_inverse.restype = i32
            L.hank_dht0_inverse.argtypes = [p, i64, d, p, p]
            L.hank_dht0_weights.restype = i32
            L.hank_dht0_weights.argtypes = [i64, p, p]
            L.hank_j0.restype = i32
            L.hank_j0.argtypes = [p, i64, p, p]
            L.hank_profile.restype = i32
            L.hank_profile.argtypes = [i32]
            L.hank_profile_report.restype = i32
            L.hank_profile_report.argtypes = [ctypes.POINTER(KernelStat), i32, ctypes.POINTER(i32)]
            _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        raise HankError(status, lib().hank_last_error().decode(errors="replace"))


def last_error() -> str:
    return lib().hank_last_error().decode(errors="replace")


def _task(task) -> int:
    return TASKS[task] if isinstance(task, str) else int(task)


def _options(plan_mode=0, precision=0, direct=0, prefer_far=0, nrhs=0, M=0, nu=0, shift=0) -> Options:
    return Options(int(plan_mode), int(precision), int(direct), int(prefer_far), int(nrhs), int(M), int(nu),
                   int(shift))


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _dev_f64(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError("%s must be a float64 GPU tensor" % name)
    if not t.is_contiguous():
        raise TypeError("%s must be contiguous" % name)
    return t


def transform(task, c, eps: float, out=None, plan_mode: int = 0, precision: int = 0,
              direct: int = 0, prefer_far: int = 0, stream=None, M: int = 0, nu: int = 0, shift: int = 0):
    """f = J_0(r w^T) c for c of shape (N,) or (nrhs, N) (one right-hand side per row).
    plan_mode 0 tuned, 1 paper, 2 paper with one far block; M overrides the
    paper's number of asymptotic terms in modes 1 and 2.  Schlomilch tasks:
    order nu (J_nu) and w_n = (n + shift) pi."""
    import torch
    c = _dev_f64(c, "c")
    if out is None:
        out = torch.empty_like(c)
    out = _dev_f64(out, "out")
    if out.shape != c.shape:
        raise ValueError("out must have the shape of c")
    N = c.shape[-1]
    nrhs = 1 if c.dim() == 1 else c.shape[0]
    opts = _options(plan_mode, precision, direct, prefer_far, 0, M, nu, shift)
    _check(lib().hank_transform(_task(task), ctypes.c_void_p(c.data_ptr()), N, nrhs, N, float(eps),
                                ctypes.c_void_p(out.data_ptr()), N, ctypes.byref(opts), _stream(stream)))
    return out


def transform_noalloc(task, c, eps: float, out, plan_mode: int = 0, precision: int = 0, direct: int = 0,
                      prefer_far: int = 0, stream=None, M: int = 0, nu: int = 0, shift: int = 0):
    """transform() through hank_transform_noalloc: no device allocation in the
    library (workspace from its static scratch array); the plan must be cached
    by an earlier transform() with the same arguments, and `out` is required."""
    c = _dev_f64(c, "c")
    out = _dev_f64(out, "out")
    if out.shape != c.shape:
        raise ValueError("out must have the shape of c")
    N = c.shape[-1]
    nrhs = 1 if c.dim() == 1 else c.shape[0]
    opts = _options(plan_mode, precision, direct, prefer_far, 0, M, nu, shift)
    _check(lib().hank_transform_noalloc(_task(task), ctypes.c_void_p(c.data_ptr()), N, nrhs, N, float(eps),
                                        ctypes.c_void_p(out.data_ptr()), N, ctypes.byref(opts), _stream(stream)))
    return out


def schlomilch(c, eps: float, out=None, stream=None):
    """f_k = sum_n c_n J_0((k-1)/(N-1) * n pi)  (Sec. 4)."""
    import torch
    c = _dev_f64(c, "c")
    out = _dev_f64(torch.empty_like(c) if out is None else out, "out")
    _check(lib().hank_schlomilch(ctypes.c_void_p(c.data_ptr()), c.numel(), float(eps),
                                 ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def fourier_bessel(c, eps: float, out=None, stream=None):
    """f_k = sum_n c_n J_0((k-1)/(N-1) * j_{0,n})  (Sec. 5)."""
    import torch
    c = _dev_f64(c, "c")
    out = _dev_f64(torch.empty_like(c) if out is None else out, "out")
    _check(lib().hank_fourier_bessel(ctypes.c_void_p(c.data_ptr()), c.numel(), float(eps),
                                     ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def dht0(c, eps: float, out=None, stream=None):
    """f_k = sum_n c_n J_0(j_{0,k} j_{0,n} / j_{0,N+1})  (Sec. 6, eq. (DHT))."""
    import torch
    c = _dev_f64(c, "c")
    out = _dev_f64(torch.empty_like(c) if out is None else out, "out")
    _check(lib().hank_dht0(ctypes.c_void_p(c.data_ptr()), c.numel(), float(eps),
                           ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def dht0_inverse(f, eps: float, out=None, stream=None):
    """c = (1/j_{0,N+1}^2) D_v J D_v f with v_n = 2/J_1(j_{0,n})^2: the inverse
    of dht0 by the self-inverse relation of Sec. 6 (eq. (selfinverse))."""
    import torch
    f = _dev_f64(f, "f")
    out = _dev_f64(torch.empty_like(f) if out is None else out, "out")
    _check(lib().hank_dht0_inverse(ctypes.c_void_p(f.data_ptr()), f.numel(), float(eps),
                                   ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def dht0_weights(N: int, out=None, stream=None):
    """v_n = 2/J_1(j_{0,n})^2 for n = 1..N, computed on the GPU."""
    import torch
    if out is None:
        out = torch.empty(int(N), dtype=torch.float64, device="cuda")
    out = _dev_f64(out, "out")
    _check(lib().hank_dht0_weights(int(N), ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def _requests(requests):
    reqs = list(requests)
    arr = (Request * max(1, len(reqs)))()
    for i, r in enumerate(reqs):
        c = _dev_f64(r["c"], "c")
        o = _dev_f64(r["out"], "out")
        N = c.shape[-1]
        nrhs = 1 if c.dim() == 1 else c.shape[0]
        arr[i] = Request(_task(r["task"]), int(r.get("precision", 0)), N, nrhs, N, N, float(r["eps"]),
                         c.data_ptr(), o.data_ptr(), int(r.get("nu", 0)), int(r.get("shift", 0)))
    return arr, len(reqs)


def batch(requests, stream=None):
    """Submit many transforms at once.  requests: iterable of dicts with keys
    task, c, out, eps and optionally precision, nu, shift (c, out of shape (N,)
    or (nrhs, N))."""
    arr, n = _requests(requests)
    _check(lib().hank_batch(arr, n, _stream(stream)))


def autotune(stream=None) -> dict:
    """Time the far-field passes for each FFT length 2^10..2^23 and install the
    fastest split L = L1 x L2 for plans built afterwards; {log2 L: log2 L2}."""
    arr = (ctypes.c_int32 * 24)()
    _check(lib().hank_autotune(_stream(stream), arr))
    return {lg: arr[lg] for lg in range(10, 24)}


def autotune_reset():
    """Default FFT splits for plans built afterwards."""
    _check(lib().hank_autotune_reset())


def autotune_save(path: str):
    """Write the installed FFT splits to a text file (host only)."""
    _check(lib().hank_autotune_save(os.fsencode(path)))


def autotune_load(path: str):
    """Install the FFT splits of a file written by autotune_save (host only)."""
    _check(lib().hank_autotune_load(os.fsencode(path)))


class BatchGraph:
    """A batch captured once as a HIP graph (hank_batch_graph_*): launch()
    replays the same requests, reading and writing the same tensors, without
    host work.  Keep the tensors alive while the graph is used."""

    def __init__(self, requests, stream=None):
        self._reqs = list(requests)  # keeps the tensors referenced
        arr, n = _requests(self._reqs)
        h = ctypes.c_void_p()
        _check(lib().hank_batch_graph_create(arr, n, _stream(stream), ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _check(lib().hank_batch_graph_launch(self._h, _stream(stream)))

    def close(self):
        if self._h:
            import torch
            torch.cuda.synchronize()
            _check(lib().hank_batch_graph_destroy(self._h))
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def plan_info(task, N: int, eps: float, plan_mode: int = 0, precision: int = 0, direct: int = 0,
              prefer_far: int = 0, nrhs: int = 1, M: int = 0, nu: int = 0, shift: int = 0) -> dict:
    """Parameters and costs of the plan the library would use for nrhs
    right-hand sides (host only)."""
    s = PlanSummary()
    opts = _options(plan_mode, precision, direct, prefer_far, nrhs, M, nu, shift)
    _check(lib().hank_plan_info(_task(task), int(N), float(eps), ctypes.byref(opts), ctypes.byref(s)))
    return {name: getattr(s, name) for name, _ in PlanSummary._fields_}


def plan_block(task, N: int, eps: float, k: int, plan_mode: int = 0, precision: int = 0,
               prefer_far: int = 0, nrhs: int = 1, M: int = 0, nu: int = 0, shift: int = 0) -> dict:
    b = BlockInfo()
    opts = _options(plan_mode, precision, 0, prefer_far, nrhs, M, nu, shift)
    _check(lib().hank_plan_block(_task(task), int(N), float(eps), ctypes.byref(opts), int(k), ctypes.byref(b)))
    return {name: getattr(b, name) for name, _ in BlockInfo._fields_}


def plan_blocks(task, N: int, eps: float, plan_mode: int = 0, precision: int = 0,
                prefer_far: int = 0, nrhs: int = 1, M: int = 0, nu: int = 0, shift: int = 0) -> list:
    n = plan_info(task, N, eps, plan_mode, precision, prefer_far=prefer_far, nrhs=nrhs, M=M, nu=nu,
                  shift=shift)["nblocks"]
    return [plan_block(task, N, eps, k, plan_mode, precision, prefer_far, nrhs, M, nu, shift) for k in range(n)]


def param_s(nu: int, M: int, eps: float) -> float:
    return lib().hank_param_s(int(nu), int(M), float(eps))


def param_t(nu: int, T: int, eps: float) -> float:
    return lib().hank_param_t(int(nu), int(T), float(eps))


def param_neumann(K: int, eps: float) -> float:
    return lib().hank_param_neumann(int(K), float(eps))


def param_pK(K: int, eps: float) -> float:
    return lib().hank_param_pK(int(K), float(eps))


def param_qT(T: int, eps: float) -> float:
    return lib().hank_param_qT(int(T), float(eps))


def root_offsets(nmax: int, out=None, stream=None):
    """b_n = j_{0,n} - (n - 1/4) pi for n = 1..nmax, computed on the GPU."""
    import torch
    if out is None:
        out = torch.empty(int(nmax), dtype=torch.float64, device="cuda")
    out = _dev_f64(out, "out")
    _check(lib().hank_root_offsets(int(nmax), ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def j0(z, out=None, stream=None):
    """J_0 by the library's device evaluator."""
    import torch
    z = _dev_f64(z, "z")
    out = _dev_f64(torch.empty_like(z) if out is None else out, "out")
    _check(lib().hank_j0(ctypes.c_void_p(z.data_ptr()), z.numel(), ctypes.c_void_p(out.data_ptr()),
                         _stream(stream)))
    return out


def cache_clear():
    _check(lib().hank_cache_clear())


def cache_bytes() -> int:
    return int(lib().hank_cache_bytes())


def cache_limit(nbytes: int):
    """Device bytes the plan cache may hold before least recently used plans are freed."""
    _check(lib().hank_cache_limit(int(nbytes)))


def profile(enable: bool = True):
    """Start (and reset) or stop per-kernel event timing."""
    _check(lib().hank_profile(1 if enable else 0))


def profile_report() -> list:
    """[{name, launches, total_ms, bytes, work}] for the kernels timed since profile(True)."""
    arr = (KernelStat * 16)()
    n = ctypes.c_int32(0)
    _check(lib().hank_profile_report(arr, 16, ctypes.byref(n)))
    return [{"name": arr[i].name.decode(), "launches": arr[i].launches, "total_ms": arr[i].total_ms,
             "bytes": arr[i].bytes, "work": arr[i].work} for i in range(min(n.value, 16))]


class ServerSummary(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("mean_batch", ctypes.c_double), ("p50_ms", ctypes.c_double),
                ("p90_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("max_ms", ctypes.c_double),
                ("mean_ms", ctypes.c_double), ("wall_s", ctypes.c_double), ("throughput", ctypes.c_double),
                ("plans_built", ctypes.c_int64)]


def _server_fns():
    L = lib()
    if not getattr(L, "_server_typed", False):
        p, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.hank_server_create.restype = i32
        L.hank_server_create.argtypes = [i64, i32, i64, p, ctypes.POINTER(p)]
        L.hank_server_warm.restype = i32
        L.hank_server_warm.argtypes = [p, ctypes.POINTER(Request)]
        L.hank_server_submit.restype = i32
        L.hank_server_submit.argtypes = [p, ctypes.POINTER(Request), d, ctypes.POINTER(i64)]
        for name in ("hank_server_start", "hank_server_drain", "hank_server_destroy"):
            f = getattr(L, name)
            f.restype = i32
            f.argtypes = [p]
        L.hank_server_status.restype = i32
        L.hank_server_status.argtypes = [p, i64, ctypes.POINTER(i32), ctypes.POINTER(d)]
        L.hank_server_stats.restype = i32
        L.hank_server_stats.argtypes = [p, ctypes.POINTER(ServerSummary)]
        L._server_typed = True
    return L


def _request(r) -> Request:
    c = _dev_f64(r["c"], "c")
    o = _dev_f64(r["out"], "out")
    N = c.shape[-1]
    nrhs = 1 if c.dim() == 1 else c.shape[0]
    return Request(_task(r["task"]), int(r.get("precision", 0)), N, nrhs, N, N, float(r["eps"]),
                   c.data_ptr(), o.data_ptr(), int(r.get("nu", 0)), int(r.get("shift", 0)))


class Server:
    """Continuous-batching server of the C library (hank_server_*).

    Requests are dicts like those of batch(); their tensors are kept alive by
    this object until close()."""

    STATES = {0: "waiting", 1: "admitted", 2: "done", 3: "rejected"}

    def __init__(self, budget_bytes: int, max_batch: int = 64, max_pending: int = 256, stream=None):
        L = _server_fns()
        h = ctypes.c_void_p()
        _check(L.hank_server_create(int(budget_bytes), int(max_batch), int(max_pending), _stream(stream),
                                    ctypes.byref(h)))
        self._h = h
        self._keep = []

    def warm(self, req):
        _check(_server_fns().hank_server_warm(self._h, ctypes.byref(_request(req))))

    def submit(self, req, arrival_s: float = -1.0) -> int:
        t = ctypes.c_int64()
        _check(_server_fns().hank_server_submit(self._h, ctypes.byref(_request(req)), float(arrival_s),
                                                ctypes.byref(t)))
        self._keep.append(req)
        return t.value

    def start(self):
        _check(_server_fns().hank_server_start(self._h))

    def drain(self):
        _check(_server_fns().hank_server_drain(self._h))

    def status(self, ticket: int):
        s, lat = ctypes.c_int32(), ctypes.c_double()
        _check(_server_fns().hank_server_status(self._h, int(ticket), ctypes.byref(s), ctypes.byref(lat)))
        return self.STATES[s.value], lat.value

    def stats(self) -> dict:
        s = ServerSummary()
        _check(_server_fns().hank_server_stats(self._h, ctypes.byref(s)))
        return {name: getattr(s, name) for name, _ in ServerSummary._fields_}

    def close(self):
        if self._h:
            _check(_server_fns().hank_server_destroy(self._h))
            self._h = None
            self._keep = []

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
