"""Python binding of libai.so (the C ABI in include/ai.h): argument
marshalling only.  Every step of the integration runs in the HIP kernels.

The entry points keep the C names.  Buffers are torch CUDA (HIP) float64
tensors laid out as planes: y0 and final_state of shape (12, ld), obs of
shape (13, ld), contiguous, so plane c starts at c * ld.  If the library has
not been built, or does not load, every call raises; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libai.so")

NSTATE = 12
NOBS = 13
KERNELS = {"plain": 0, "persistent": 1}
SCHEDULE_LONGEST_FIRST = 16
SCHEDULES = {None: 0, "index": 0, "longest-first": SCHEDULE_LONGEST_FIRST}
FP32_STAGES = 32                      # AI_FP32_STAGES
PRECISIONS = {"fp64": 0, "fp32-stages": FP32_STAGES}
TIME_KERNEL = 64                      # AI_TIME_KERNEL
OK, WRTOL, EINVAL, EHIP, ENOMEM, EUNSUPPORTED, EAGAIN = 0, 1, -1, -2, -3, -4, -5

# exported symbols of the C ABI, in declaration order
SYMBOLS = ("ai_integrate", "ai_integrate_async", "ai_integrate_static_async", "ai_integrate_batch",
           "ai_integrate_batch_async", "ai_batch_plan_create", "ai_batch_plan_launch",
           "ai_batch_plan_destroy", "ai_tune", "ai_tune_batch", "ai_trace", "ai_server_create",
           "ai_server_submit", "ai_server_wait", "ai_server_destroy", "ai_kernel_time",
           "ai_get_kernel_info", "ai_last_error", "ai_nobs", "ai_version")


class AiParams(C.Structure):
    _fields_ = [
        ("m_ion", C.c_double), ("m_atom", C.c_double),
        ("n", C.c_int32), ("m", C.c_int32),
        ("Cn", C.c_double), ("Cm", C.c_double),
        ("a", C.c_double * 3), ("q", C.c_double * 3),
        ("omega_rf", C.c_double), ("r_exit", C.c_double), ("r_bounce", C.c_double),
        ("max_steps", C.c_int64), ("hmax", C.c_double),
    ]


class AiBatchItem(C.Structure):
    """ai_batch_item: one ensemble of a batched call."""
    _fields_ = [
        ("params", AiParams), ("y0", C.c_void_p), ("n", C.c_int64), ("ld", C.c_int64),
        ("t0", C.c_double), ("tmax", C.c_double), ("rtol", C.c_double), ("atol", C.c_double),
        ("final_state", C.c_void_p), ("obs", C.c_void_p),
    ]


class AiServerConfig(C.Structure):
    _fields_ = [("max_batch", C.c_int64), ("schedule", C.c_int32), ("workers", C.c_int32),
                ("mode", C.c_int32), ("ring", C.c_int32), ("slab_bytes", C.c_int64),
                ("idle_ms", C.c_double), ("refill_min", C.c_int32), ("reserved", C.c_int32)]


SERVE_MODES = {"launches": 0, "resident": 1}   # enum ai_serve_mode


class AiRequestInfo(C.Structure):
    """ai_request_info: completion record of a served request."""
    _fields_ = [
        ("rc", C.c_int32), ("batch_size", C.c_int32), ("batch_id", C.c_int64),
        ("batch_trajectories", C.c_int64),
        ("submit_s", C.c_double), ("start_s", C.c_double), ("end_s", C.c_double),
        ("error", C.c_char * 128),
    ]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["error"] = self.error.decode()
        return d


class AiKernelInfo(C.Structure):
    _fields_ = [
        ("block_threads", C.c_int32), ("vgprs", C.c_int32), ("spill_bytes", C.c_int32),
        ("blocks_per_cu", C.c_int32), ("waves_per_simd", C.c_int32),
        ("compute_units", C.c_int32), ("persistent_blocks", C.c_int64),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class AiError(RuntimeError):
    def __init__(self, rc: int, msg: str):
        super().__init__(f"libai error {rc}: {msg}")
        self.rc = rc


_lock = threading.Lock()
_lib = None


def load(path: str = LIB_PATH):
    """Open libai.so; raises if it is missing (build it with
    ``python -m paper_2509_12381_amd.build``)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise FileNotFoundError(f"{path} is not built; run python -m paper_2509_12381_amd.build")
        lib = C.CDLL(path)
        _P = C.POINTER(AiParams)
        _D = C.c_void_p
        args = [_P, _D, C.c_int64, C.c_int64, C.c_double, C.c_double, C.c_double, C.c_double,
                _D, _D, C.c_int32]
        lib.ai_integrate.argtypes = args
        lib.ai_integrate.restype = C.c_int
        lib.ai_integrate_async.argtypes = args + [C.c_void_p]
        lib.ai_integrate_async.restype = C.c_int
        lib.ai_integrate_static_async.argtypes = args + [C.c_void_p]
        lib.ai_integrate_static_async.restype = C.c_int
        lib.ai_integrate_batch.argtypes = [C.POINTER(AiBatchItem), C.c_int32, C.c_int32]
        lib.ai_integrate_batch.restype = C.c_int
        lib.ai_integrate_batch_async.argtypes = [C.POINTER(AiBatchItem), C.c_int32, C.c_int32,
                                                 C.c_void_p]
        lib.ai_integrate_batch_async.restype = C.c_int
        lib.ai_batch_plan_create.argtypes = [C.POINTER(AiBatchItem), C.c_int32, C.c_int32,
                                             C.POINTER(C.c_void_p)]
        lib.ai_batch_plan_create.restype = C.c_int
        lib.ai_batch_plan_launch.argtypes = [C.c_void_p, C.c_void_p]
        lib.ai_batch_plan_launch.restype = C.c_int
        lib.ai_batch_plan_destroy.argtypes = [C.c_void_p]
        lib.ai_batch_plan_destroy.restype = C.c_int
        lib.ai_tune.argtypes = args[:-1] + [C.POINTER(C.c_int32), C.POINTER(C.c_float)]
        lib.ai_tune.restype = C.c_int
        lib.ai_tune_batch.argtypes = [C.POINTER(AiBatchItem), C.c_int32, C.POINTER(C.c_int32),
                                      C.POINTER(C.c_float)]
        lib.ai_tune_batch.restype = C.c_int
        lib.ai_trace.argtypes = [_P, _D, C.c_double, C.c_double, C.c_double, C.c_double,
                                 C.c_int32, C.c_int64, _D, _D, _D, _D, C.POINTER(C.c_int64)]
        lib.ai_trace.restype = C.c_int
        lib.ai_server_create.argtypes = [C.POINTER(AiServerConfig), C.POINTER(C.c_void_p)]
        lib.ai_server_create.restype = C.c_int
        lib.ai_server_submit.argtypes = [C.c_void_p, C.POINTER(AiBatchItem), C.c_int32,
                                         C.POINTER(C.c_uint64)]
        lib.ai_server_submit.restype = C.c_int
        lib.ai_server_wait.argtypes = [C.c_void_p, C.c_uint64, C.c_double,
                                       C.POINTER(AiRequestInfo)]
        lib.ai_server_wait.restype = C.c_int
        lib.ai_server_destroy.argtypes = [C.c_void_p]
        lib.ai_server_destroy.restype = C.c_int
        lib.ai_kernel_time.argtypes = [C.c_int32, C.POINTER(C.c_float)]
        lib.ai_kernel_time.restype = C.c_int
        lib.ai_get_kernel_info.argtypes = [C.c_int32, C.POINTER(AiKernelInfo)]
        lib.ai_get_kernel_info.restype = C.c_int
        lib.ai_last_error.restype = C.c_char_p
        lib.ai_nobs.restype = C.c_int
        lib.ai_version.restype = C.c_int
        _lib = lib
        return lib


def params(system) -> AiParams:
    """ai_params from any object (or mapping) with the System fields."""
    get = (lambda k: system[k]) if isinstance(system, dict) else (lambda k: getattr(system, k))
    p = AiParams()
    p.m_ion, p.m_atom = float(get("m_ion")), float(get("m_atom"))
    p.n, p.m = int(get("n")), int(get("m"))
    p.Cn, p.Cm = float(get("Cn")), float(get("Cm"))
    for k in range(3):
        p.a[k] = float(get("a")[k])
        p.q[k] = float(get("q")[k])
    p.omega_rf = float(get("omega_rf"))
    p.r_exit, p.r_bounce = float(get("r_exit")), float(get("r_bounce"))
    p.max_steps = int(get("max_steps"))
    p.hmax = float(get("hmax"))
    return p


def _planes(t, rows: int, name: str, host_ok: bool = False):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float64 or t.dim() != 2 or t.shape[0] != rows or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 tensor of shape ({rows}, ld)")
    if t.device.type != "cuda" and not (host_ok and t.device.type == "cpu"):
        raise ValueError(f"{name} must live on the GPU")
    return t.data_ptr(), t.shape[1]


def kernel_code(kernel, schedule=None, refill_min=0, precision="fp64") -> int:
    """ai_integrate's kernel argument: "plain" or "persistent" (or an int),
    with schedule "longest-first" adding AI_SCHEDULE_LONGEST_FIRST,
    refill_min adding AI_REFILL_MIN(refill_min) and precision "fp32-stages"
    adding AI_FP32_STAGES."""
    k = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    return k | SCHEDULES[schedule] | (int(refill_min) << 8) | PRECISIONS[precision]


def _args(system, y0, n, t0, tmax, rtol, atol, final_state, obs, kernel):
    p0, ld = _planes(y0, NSTATE, "y0")
    p1, ld1 = _planes(final_state, NSTATE, "final_state")
    p2, ld2 = _planes(obs, NOBS, "obs")
    if not (ld == ld1 == ld2):
        raise ValueError("y0, final_state and obs must share the leading dimension")
    n = ld if n is None else int(n)
    k = kernel if isinstance(kernel, int) else kernel_code(kernel)
    p = system if isinstance(system, AiParams) else params(system)
    return (C.byref(p), p0, n, ld, float(t0), float(tmax), float(rtol), float(atol), p1, p2, k)


def _check(rc: int) -> int:
    if rc < 0:
        raise AiError(rc, load().ai_last_error().decode())
    return rc


def ai_integrate(system, y0, t0, tmax, rtol, atol, final_state, obs, kernel="plain", n=None,
                 schedule=None, refill_min=0, precision="fp64"):
    """Blocking ai_integrate.  Returns AI_OK or AI_WRTOL; raises on errors."""
    k = kernel_code(kernel, schedule, refill_min, precision)
    return _check(load().ai_integrate(*_args(system, y0, n, t0, tmax, rtol, atol, final_state,
                                             obs, k)))


def ai_integrate_async(system, y0, t0, tmax, rtol, atol, final_state, obs, kernel="plain",
                       n=None, stream=None, schedule=None, refill_min=0, precision="fp64"):
    """ai_integrate_async on `stream` (a torch.cuda.Stream; default: torch's
    current stream)."""
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    k = kernel_code(kernel, schedule, refill_min, precision)
    return _check(load().ai_integrate_async(*_args(system, y0, n, t0, tmax, rtol, atol,
                                                   final_state, obs, k),
                                            C.c_void_p(s.cuda_stream)))


def ai_integrate_static_async(system, y0, t0, tmax, rtol, atol, final_state, obs,
                              kernel="plain", n=None, stream=None, schedule=None, refill_min=0,
                              precision="fp64"):
    """ai_integrate_static_async (no device allocation: the library's static
    scratch) on `stream` (default: torch's current stream)."""
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    k = kernel_code(kernel, schedule, refill_min, precision)
    return _check(load().ai_integrate_static_async(*_args(system, y0, n, t0, tmax, rtol, atol,
                                                          final_state, obs, k),
                                                   C.c_void_p(s.cuda_stream)))


def batch_items(items, host_ok: bool = False) -> "C.Array":
    """ai_batch_item array from (system, y0, final_state, obs, t0, tmax, rtol,
    atol[, n]) tuples; the tensors are (12, ld), (12, ld) and (AI_NOBS, ld),
    on the GPU (or, with host_ok, CPU tensors: host memory)."""
    arr = (AiBatchItem * max(len(items), 1))()
    for b, it in enumerate(items):
        system, y0, final_state, obs, t0, tmax, rtol, atol = it[:8]
        p0, ld = _planes(y0, NSTATE, "y0", host_ok)
        p1, ld1 = _planes(final_state, NSTATE, "final_state", host_ok)
        p2, ld2 = _planes(obs, NOBS, "obs", host_ok)
        if not (ld == ld1 == ld2):
            raise ValueError("y0, final_state and obs must share the leading dimension")
        e = arr[b]
        e.params = system if isinstance(system, AiParams) else params(system)
        e.y0, e.final_state, e.obs = p0, p1, p2
        e.n = ld if len(it) < 9 or it[8] is None else int(it[8])
        e.ld = ld
        e.t0, e.tmax, e.rtol, e.atol = float(t0), float(tmax), float(rtol), float(atol)
    return arr


def ai_integrate_batch(items, schedule=None):
    """Blocking ai_integrate_batch over batch_items(items)."""
    arr = batch_items(items)
    return _check(load().ai_integrate_batch(arr, len(items), SCHEDULES[schedule]))


def ai_integrate_batch_async(items, schedule=None, stream=None, time_kernel=False):
    """ai_integrate_batch_async on `stream` (default: torch's current stream);
    time_kernel adds AI_TIME_KERNEL."""
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    arr = batch_items(items)
    k = SCHEDULES[schedule] | (TIME_KERNEL if time_kernel else 0)
    return _check(load().ai_integrate_batch_async(arr, len(items), k,
                                                  C.c_void_p(s.cuda_stream)))


def ai_kernel_time(back: int = 0):
    """Milliseconds of the integration kernel of this thread's call made with
    AI_TIME_KERNEL `back` calls ago (0: the last; the last 64 are kept), or None
    if its stream has not reached the kernel's end."""
    ms = C.c_float()
    rc = load().ai_kernel_time(int(back), C.byref(ms))
    if rc == EAGAIN:
        return None
    _check(rc)
    return ms.value


def ai_tune(system, y0, t0, tmax, rtol, atol, final_state, obs, n=None):
    """ai_tune: time the kernel configurations on this ensemble (the outputs
    hold its results afterwards); returns (best kernel code, its ms)."""
    best, ms = C.c_int32(), C.c_float()
    a = _args(system, y0, n, t0, tmax, rtol, atol, final_state, obs, 0)[:-1]
    _check(load().ai_tune(*a, C.byref(best), C.byref(ms)))
    return best.value, ms.value


def ai_tune_batch(items):
    """ai_tune_batch over batch_items(items): (best kernel code, best ms)."""
    best = C.c_int32()
    ms = C.c_float()
    _check(load().ai_tune_batch(batch_items(items), len(items), C.byref(best), C.byref(ms)))
    return best.value, ms.value


def ai_trace(system, y0, t0, tmax, rtol, atol, capacity: int, refine: int = 1):
    """Replay one trajectory (y0: 12 device doubles) and record its path at
    `refine` points per accepted step: returns (t (capacity,), y (12, capacity),
    final_state (12,), obs (AI_NOBS,), points) with tensors on y0's device;
    points is the trajectory's number of points (1 + refine * accepted steps),
    of which the first `capacity` are stored."""
    import torch
    y = y0.reshape(-1)
    if y.numel() != NSTATE or y.dtype != torch.float64 or not y.is_cuda or not y.is_contiguous():
        raise ValueError("y0 must be 12 contiguous float64 values on the GPU")
    dev = y.device
    t_out = torch.empty((max(capacity, 1),), dtype=torch.float64, device=dev)
    y_out = torch.empty((NSTATE, max(capacity, 1)), dtype=torch.float64, device=dev)
    fin = torch.empty((NSTATE,), dtype=torch.float64, device=dev)
    obs = torch.empty((NOBS,), dtype=torch.float64, device=dev)
    pts = C.c_int64()
    p = system if isinstance(system, AiParams) else params(system)
    _check(load().ai_trace(C.byref(p), C.c_void_p(y.data_ptr()), float(t0), float(tmax),
                           float(rtol), float(atol), int(refine), int(capacity),
                           C.c_void_p(t_out.data_ptr()),
                           C.c_void_p(y_out.data_ptr()), C.c_void_p(fin.data_ptr()),
                           C.c_void_p(obs.data_ptr()), C.byref(pts)))
    return t_out[:capacity], y_out[:, :capacity], fin, obs, pts.value


def ai_server_create(max_batch: int = 0, schedule="longest-first", workers: int = 0,
                     mode="launches", ring: int = 0, slab_bytes: int = 0, idle_ms: float = 0.0,
                     refill_min: int = 0) -> C.c_void_p:
    cfg = AiServerConfig(int(max_batch), SCHEDULES[schedule], int(workers), SERVE_MODES[mode],
                         int(ring), int(slab_bytes), float(idle_ms), int(refill_min), 0)
    h = C.c_void_p()
    _check(load().ai_server_create(C.byref(cfg), C.byref(h)))
    return h


def ai_server_submit(server, item, precision="fp64") -> int:
    """Queue one request (a batch_items tuple; a resident server also takes
    CPU tensors, i.e. host memory); returns its ticket."""
    arr = batch_items([item], host_ok=True)
    ticket = C.c_uint64()
    _check(load().ai_server_submit(server, arr, PRECISIONS[precision], C.byref(ticket)))
    return ticket.value


def ai_server_wait(server, ticket: int, timeout=None):
    """The request's completion record (a dict), or None if it has not
    completed within `timeout` seconds (None: wait without limit)."""
    info = AiRequestInfo()
    rc = load().ai_server_wait(server, C.c_uint64(ticket),
                               -1.0 if timeout is None else float(timeout), C.byref(info))
    if rc == EAGAIN:
        return None
    _check(rc)
    return info.as_dict()


def ai_server_destroy(server) -> int:
    return _check(load().ai_server_destroy(server))


def ai_batch_plan_create(items, schedule="longest-first"):
    """ai_batch_plan_create over batch_items(items); returns (plan handle, rc)."""
    h = C.c_void_p()
    rc = _check(load().ai_batch_plan_create(batch_items(items), len(items), SCHEDULES[schedule],
                                            C.byref(h)))
    return h, rc


def ai_batch_plan_launch(plan, stream=None):
    """Enqueue a plan's kernels on `stream` (default: torch's current stream)."""
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return _check(load().ai_batch_plan_launch(plan, C.c_void_p(s.cuda_stream)))


def ai_batch_plan_destroy(plan):
    return _check(load().ai_batch_plan_destroy(plan))


class BatchPlan:
    """ai_batch_plan: a batch (batch_items tuples) prepared once; launch()
    enqueues only its one kernel (capturable in a HIP graph).  The tensors of
    the items must stay alive while the plan is used."""

    def __init__(self, items, schedule="longest-first"):
        self._h, self.rc = ai_batch_plan_create(items, schedule)

    def launch(self, stream=None):
        return ai_batch_plan_launch(self._h, stream)

    def close(self):
        if self._h:
            h, self._h = self._h, None
            ai_batch_plan_destroy(h)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Server:
    """ai_server: requests (batch_items tuples) served by a resident kernel
    (mode="resident": continuous batching, admission by footprint into the
    server's device slab) or by batched launches (mode="launches").  The
    buffers of a request must stay alive until wait() has returned its
    completion."""

    def __init__(self, max_batch: int = 0, schedule="longest-first", workers: int = 0,
                 mode="launches", ring: int = 0, slab_bytes: int = 0, idle_ms: float = 0.0,
                 refill_min: int = 0):
        self._h = ai_server_create(max_batch, schedule, workers, mode, ring, slab_bytes, idle_ms,
                                   refill_min)

    def submit(self, item, precision="fp64") -> int:
        return ai_server_submit(self._h, item, precision)

    def wait(self, ticket: int, timeout=None):
        return ai_server_wait(self._h, ticket, timeout)

    def close(self):
        if self._h:
            h, self._h = self._h, None
            ai_server_destroy(h)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def ai_get_kernel_info(kernel="plain", precision="fp64") -> dict:
    info = AiKernelInfo()
    k = (KERNELS[kernel] | PRECISIONS[precision] if isinstance(kernel, str)
         else int(kernel) & (0xf | FP32_STAGES))
    _check(load().ai_get_kernel_info(k, C.byref(info)))
    return info.as_dict()


def ai_last_error() -> str:
    return load().ai_last_error().decode()


def ai_nobs() -> int:
    return load().ai_nobs()


def ai_version() -> int:
    return load().ai_version()


def integrate(system, y0, t0, tmax, rtol, atol, kernel="plain", stream=None, schedule=None):
    """Allocate outputs next to y0 (a (12, n) GPU tensor), enqueue the
    integration on the current stream and return (final_state, obs, rc)."""
    import torch
    final_state = torch.empty_like(y0)
    obs = torch.empty((NOBS, y0.shape[1]), dtype=torch.float64, device=y0.device)
    rc = ai_integrate_async(system, y0, t0, tmax, rtol, atol, final_state, obs, kernel,
                            stream=stream, schedule=schedule)
    return final_state, obs, rc
