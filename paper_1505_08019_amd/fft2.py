"""ctypes binding over the C ABI of ``libfft2.so`` (see ``include/fft2.h``).

Argument marshalling only: every step of the transform runs in the HIP
kernels of the library.  Tensors are ``torch`` complex64 CUDA tensors (torch is
used for device memory and streams); raw device pointers work too.  If the
library has not been built the first call raises ``RuntimeError``: there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfft2.so")

FORWARD = -1
INVERSE = +1
PREC_FP32 = 0
PREC_SPLIT_BF16 = 1
PREC_FP16 = 2

SUCCESS = 0
ERR_INVALID_VALUE = -1
ERR_INVALID_SIZE = -2
ERR_UNSUPPORTED = -3
ERR_ALIGNMENT = -4
ERR_ALIAS = -5
ERR_OUT_OF_MEMORY = -6
ERR_DEVICE = -7
ERR_BUDGET = -8
ERR_SHUTDOWN = -9
ERR_TIMEOUT = -10
ERR_NOT_FOUND = -11
NOALLOC_MAX_POINTS = 1 << 22  # FFT2_NOALLOC_MAX_POINTS

# Every symbol include/fft2.h declares (the CPU tests check the library exports them).
EXPORTS = [
    "fft2_validate", "fft2_plan", "fft2_exec", "fft2_exec_partial", "fft2_exec_filter",
    "fft2_plan_destroy", "fft2_exec_pass", "fft2_plan_info", "fft2_batch_plan", "fft2_exec_batch",
    "fft2_batch_destroy", "fft2_serve_start", "fft2_serve_alloc", "fft2_serve_free",
    "fft2_serve_submit", "fft2_serve_wait", "fft2_serve_stats", "fft2_serve_stop",
    "fft2_last_error", "fft2_last_error_text", "fft2_error_string",
    "fft2_describe_schedule", "fft2_plan_describe", "fft2_schedule_candidates", "fft2_plan_schedule",
    "fft2_autotune", "fft2_plan_tables", "fft2_batch_validate", "fft2_batch_plan_tuned", "fft2_exec_batch_graph",
    "fft2_batch_status", "fft2_batch_info", "fft2_exec_filter_ws", "fft2_serve_validate_config",
    "fft2_serve_stats_reset", "fft2_exec_noalloc", "fft2_plan_real", "fft2_exec_real", "fft2_rplan_destroy",
    "fft2_plan_dct", "fft2_exec_dct", "fft2_dplan_destroy",
]

_lib = None
_lock = threading.Lock()


class FFT2Error(RuntimeError):
    def __init__(self, code: int, text: str):
        super().__init__("fft2 error %d: %s" % (code, text))
        self.code = code


def lib() -> ctypes.CDLL:
    """Load libfft2.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libfft2.so is not built; run `python -m paper_1505_08019_amd.build` "
                               "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64
        sig = {
            "fft2_validate": (i32, [i32, i32, i32, i32]),
            "fft2_plan": (vp, [i32, i32, i32, i32]),
            "fft2_exec": (i32, [vp, vp, vp, vp]),
            "fft2_exec_noalloc": (i32, [vp, vp, vp, vp]),
            "fft2_plan_real": (vp, [i32, i32, i32, i32]),
            "fft2_exec_real": (i32, [vp, vp, vp, vp]),
            "fft2_rplan_destroy": (i32, [vp]),
            "fft2_plan_dct": (vp, [i32, i32, i32, i32]),
            "fft2_exec_dct": (i32, [vp, vp, vp, vp]),
            "fft2_dplan_destroy": (i32, [vp]),
            "fft2_exec_partial": (i32, [vp, vp, vp, i32, i32, vp]),
            "fft2_exec_filter": (i32, [vp, vp, vp, ctypes.c_float, vp]),
            "fft2_exec_filter_ws": (i32, [vp, vp, vp, ctypes.c_float, vp, ctypes.c_size_t, vp]),
            "fft2_serve_validate_config": (i32, [vp]),
            "fft2_serve_stats_reset": (i32, [vp]),
            "fft2_plan_destroy": (i32, [vp]),
            "fft2_exec_pass": (i32, [vp, i32, vp, vp, vp]),
            "fft2_plan_info": (i32, [vp, ctypes.POINTER(i32), ctypes.POINTER(i64)]),
            "fft2_batch_plan": (vp, [i32, ctypes.POINTER(i32), ctypes.POINTER(i32), i32, i32]),
            "fft2_exec_batch": (i32, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]),
            "fft2_batch_destroy": (i32, [vp]),
            "fft2_plan_tables": (i32, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp)]),
            "fft2_batch_validate": (i32, [i32, ctypes.POINTER(i32), ctypes.POINTER(i32), i32, i32]),
            "fft2_batch_plan_tuned": (vp, [i32, ctypes.POINTER(i32), ctypes.POINTER(i32), i32, i32, i32]),
            "fft2_exec_batch_graph": (i32, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]),
            "fft2_batch_status": (i32, [vp, ctypes.POINTER(i32)]),
            "fft2_batch_info": (i32, [vp, ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i64)]),
            "fft2_serve_start": (i32, [vp, ctypes.POINTER(vp)]),
            "fft2_serve_alloc": (i32, [vp, ctypes.c_size_t, ctypes.POINTER(vp)]),
            "fft2_serve_free": (i32, [vp, vp]),
            "fft2_serve_submit": (i32, [vp, vp, ctypes.POINTER(u64)]),
            "fft2_serve_wait": (i32, [vp, u64, i64, ctypes.POINTER(i32)]),
            "fft2_serve_stats": (i32, [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]),
            "fft2_serve_stop": (i32, [vp]),
            "fft2_last_error": (i32, []),
            "fft2_last_error_text": (ctypes.c_char_p, []),
            "fft2_error_string": (ctypes.c_char_p, [i32]),
            "fft2_describe_schedule": (i32, [i32, i32, ctypes.c_char_p, i32]),
            "fft2_plan_describe": (i32, [vp, ctypes.c_char_p, i32]),
            "fft2_schedule_candidates": (i32, [i32, i32, ctypes.c_char_p, i32]),
            "fft2_plan_schedule": (vp, [i32, i32, i32, i32, ctypes.c_char_p]),
            "fft2_autotune": (i32, [i32, i32, i32, i32, i32, ctypes.c_char_p, i32]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
        return _lib


def last_error() -> tuple[int, str]:
    L = lib()
    return L.fft2_last_error(), (L.fft2_last_error_text() or b"").decode()


def check(rc: int) -> None:
    if rc != SUCCESS:
        code, text = last_error()
        raise FFT2Error(rc, text or lib().fft2_error_string(rc).decode())


def describe_schedule(rows: int, cols: int) -> str:
    buf = ctypes.create_string_buffer(1024)
    check(lib().fft2_describe_schedule(rows, cols, buf, len(buf)))
    return buf.value.decode()


def schedule_candidates(rows: int, cols: int) -> list[str]:
    buf = ctypes.create_string_buffer(1 << 17)
    n = lib().fft2_schedule_candidates(rows, cols, buf, len(buf))
    if n < 0:
        check(n)
    return [s for s in buf.value.decode().split("\n") if s]


def autotune(rows: int, cols: int, direction: int = FORWARD, precision: int = PREC_FP32, reps: int = 5) -> str:
    """Time every candidate schedule and remember the fastest (see fft2_autotune)."""
    buf = ctypes.create_string_buffer(256)
    check(lib().fft2_autotune(rows, cols, direction, precision, reps, buf, len(buf)))
    return buf.value.decode()


def validate(rows: int, cols: int, direction: int = FORWARD, precision: int = PREC_FP32) -> int:
    return lib().fft2_validate(rows, cols, direction, precision)


def _ptr(x) -> int:
    if x is None:
        return 0
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _check_tensor(x, rows: int, cols: int, name: str) -> None:
    import torch
    if not isinstance(x, torch.Tensor):
        return
    if x.dtype != torch.complex64:
        raise TypeError("%s must be complex64, got %s" % (name, x.dtype))
    if not x.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if not x.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if x.numel() != rows * cols:
        raise ValueError("%s has %d elements, plan needs %d x %d" % (name, x.numel(), rows, cols))


class Plan:
    """A plan for rows x cols images (fft2_plan / fft2_plan_destroy)."""

    def __init__(self, rows: int, cols: int, direction: int = FORWARD, precision: int = PREC_FP32,
                 schedule: str | None = None):
        self.rows, self.cols, self.direction, self.precision = rows, cols, direction, precision
        if schedule is None:
            self._h = lib().fft2_plan(rows, cols, direction, precision)
        else:
            self._h = lib().fft2_plan_schedule(rows, cols, direction, precision, schedule.encode())
        if not self._h:
            code, text = last_error()
            raise FFT2Error(code, text)

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().fft2_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self) -> int:
        return self._h

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(1024)
        check(lib().fft2_plan_describe(self._h, buf, len(buf)))
        return buf.value.decode()

    def info(self) -> tuple[int, int]:
        p = ctypes.c_int()
        b = ctypes.c_int64()
        check(lib().fft2_plan_info(self._h, ctypes.byref(p), ctypes.byref(b)))
        return p.value, b.value

    def _out(self, x, out):
        if out is None:
            import torch
            out = torch.empty((self.rows, self.cols), dtype=torch.complex64, device=x.device)
        return out

    def exec(self, x, out=None, stream=None):
        out = self._out(x, out)
        _check_tensor(x, self.rows, self.cols, "in")
        _check_tensor(out, self.rows, self.cols, "out")
        check(lib().fft2_exec(self._h, _ptr(x), _ptr(out), _stream(stream)))
        return out

    def exec_noalloc(self, x, out=None, stream=None):
        """fft2_exec_noalloc: the library allocates nothing (in-place calls use
        its static scratch image; images of at most FFT2_NOALLOC_MAX_POINTS)."""
        out = self._out(x, out)
        _check_tensor(x, self.rows, self.cols, "in")
        _check_tensor(out, self.rows, self.cols, "out")
        check(lib().fft2_exec_noalloc(self._h, _ptr(x), _ptr(out), _stream(stream)))
        return out

    def exec_partial(self, x, row_stages: int, col_stages: int, out=None, stream=None):
        out = self._out(x, out)
        _check_tensor(x, self.rows, self.cols, "in")
        _check_tensor(out, self.rows, self.cols, "out")
        check(lib().fft2_exec_partial(self._h, _ptr(x), _ptr(out), row_stages, col_stages, _stream(stream)))
        return out

    def exec_pass(self, i: int, x, out, stream=None):
        """Enqueue only pass i of the schedule (instrumentation)."""
        check(lib().fft2_exec_pass(self._h, i, _ptr(x), _ptr(out), _stream(stream)))
        return out

    def exec_filter(self, x, cutoff: float, out=None, stream=None):
        out = self._out(x, out)
        _check_tensor(x, self.rows, self.cols, "in")
        _check_tensor(out, self.rows, self.cols, "out")
        check(lib().fft2_exec_filter(self._h, _ptr(x), _ptr(out), float(cutoff), _stream(stream)))
        return out


class RealPlan:
    """A real-image plan (fft2_plan_real): forward takes a (rows, cols) float32
    device tensor and returns its (rows, cols/2 + 1) complex64 half spectrum;
    inverse takes the half spectrum and returns the float32 image."""

    def __init__(self, rows: int, cols: int, direction: int = FORWARD, precision: int = PREC_FP32):
        self.rows, self.cols, self.direction, self.precision = rows, cols, direction, precision
        self._h = lib().fft2_plan_real(rows, cols, direction, precision)
        if not self._h:
            code, text = last_error()
            raise FFT2Error(code, text)

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().fft2_rplan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self) -> int:
        return self._h

    def exec(self, x, out=None, stream=None):
        import torch
        half = (self.rows, self.cols // 2 + 1)
        full = (self.rows, self.cols)
        want_in, want_out = (torch.float32, torch.complex64) if self.direction == FORWARD else (torch.complex64,
                                                                                              torch.float32)
        shape_in, shape_out = (full, half) if self.direction == FORWARD else (half, full)
        if isinstance(x, torch.Tensor):
            if x.dtype != want_in or not x.is_cuda or not x.is_contiguous() or tuple(x.shape) != shape_in:
                raise ValueError("input must be a contiguous %s device tensor of shape %r" % (want_in, shape_in))
        if out is None:
            out = torch.empty(shape_out, dtype=want_out, device=x.device)
        elif isinstance(out, torch.Tensor):
            if out.dtype != want_out or not out.is_cuda or not out.is_contiguous() or tuple(out.shape) != shape_out:
                raise ValueError("output must be a contiguous %s device tensor of shape %r" % (want_out, shape_out))
        check(lib().fft2_exec_real(self._h, _ptr(x), _ptr(out), _stream(stream)))
        return out


class DctPlan:
    """A 2D DCT plan (fft2_plan_dct): forward = DCT-II, inverse = the DCT-III
    that undoes it; (rows, cols) float32 device tensors in and out."""

    def __init__(self, rows: int, cols: int, direction: int = FORWARD, precision: int = PREC_FP32):
        self.rows, self.cols, self.direction, self.precision = rows, cols, direction, precision
        self._h = lib().fft2_plan_dct(rows, cols, direction, precision)
        if not self._h:
            code, text = last_error()
            raise FFT2Error(code, text)

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().fft2_dplan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self) -> int:
        return self._h

    def exec(self, x, out=None, stream=None):
        import torch
        shape = (self.rows, self.cols)
        for t, name in ((x, "input"), (out, "output")):
            if isinstance(t, torch.Tensor) and (t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous()
                                                or tuple(t.shape) != shape):
                raise ValueError("%s must be a contiguous float32 device tensor of shape %r" % (name, shape))
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=x.device)
        check(lib().fft2_exec_dct(self._h, _ptr(x), _ptr(out), _stream(stream)))
        return out


_plan_cache: dict = {}


def _cached_plan(rows, cols, direction, precision) -> Plan:
    key = (rows, cols, direction, precision)
    p = _plan_cache.get(key)
    if p is None:
        p = Plan(rows, cols, direction, precision)
        _plan_cache[key] = p
    return p


def fft2(x, precision: int = PREC_FP32, out=None, stream=None):
    """Forward 2D DFT of a (rows, cols) complex64 CUDA tensor."""
    rows, cols = x.shape
    return _cached_plan(rows, cols, FORWARD, precision).exec(x, out, stream)


def ifft2(x, precision: int = PREC_FP32, out=None, stream=None):
    """Inverse 2D DFT (scaled by 1/(rows*cols))."""
    rows, cols = x.shape
    return _cached_plan(rows, cols, INVERSE, precision).exec(x, out, stream)


def filter_gaussian(x, cutoff: float, out=None, stream=None, precision: int = PREC_FP32):
    """Gaussian low-pass filter request: ifft2(fft2(x) * H)."""
    rows, cols = x.shape
    return _cached_plan(rows, cols, FORWARD, precision).exec_filter(x, cutoff, out, stream)


def _int_array(vals):
    arr = (ctypes.c_int * len(vals))(*[int(v) for v in vals])
    return arr


def batch_validate(shapes, direction: int = FORWARD, precision: int = PREC_FP32) -> int:
    rows = _int_array([r for r, c in shapes])
    cols = _int_array([c for r, c in shapes])
    return lib().fft2_batch_validate(len(shapes), rows, cols, direction, precision)


class Batch:
    """A ragged batch of images run by one persistent launch (fft2_batch_*)."""

    def __init__(self, shapes, direction: int = FORWARD, precision: int = PREC_FP32, tuned_reps: int = 0):
        self.shapes = [(int(r), int(c)) for r, c in shapes]
        self.direction, self.precision = direction, precision
        rows = _int_array([r for r, c in self.shapes])
        cols = _int_array([c for r, c in self.shapes])
        n = len(self.shapes)
        if tuned_reps > 0:
            self._h = lib().fft2_batch_plan_tuned(n, rows, cols, direction, precision, tuned_reps)
        else:
            self._h = lib().fft2_batch_plan(n, rows, cols, direction, precision)
        if not self._h:
            code, text = last_error()
            raise FFT2Error(code, text)

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().fft2_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _ptrs(self, xs, outs):
        if xs is None:
            return None, None
        if len(xs) != len(self.shapes) or len(outs) != len(self.shapes):
            raise ValueError("need one input and one output per image")
        for (r, c), x, y in zip(self.shapes, xs, outs):
            _check_tensor(x, r, c, "in")
            _check_tensor(y, r, c, "out")
        pin = (ctypes.c_void_p * len(xs))(*[_ptr(x) for x in xs])
        pout = (ctypes.c_void_p * len(outs))(*[_ptr(y) for y in outs])
        return pin, pout

    def exec(self, xs=None, outs=None, stream=None, graph: bool = False):
        pin, pout = self._ptrs(xs, outs)
        f = lib().fft2_exec_batch_graph if graph else lib().fft2_exec_batch
        check(f(self._h, pin, pout, _stream(stream)))
        return outs

    def status(self) -> int:
        v = ctypes.c_int()
        check(lib().fft2_batch_status(self._h, ctypes.byref(v)))
        return v.value

    def info(self) -> tuple[int, int, int]:
        a, b, c = ctypes.c_int64(), ctypes.c_int(), ctypes.c_int64()
        check(lib().fft2_batch_info(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value


# ---- serving loop -----------------------------------------------------------

KIND_FORWARD, KIND_INVERSE, KIND_FILTER = 0, 1, 2


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_inflight_launches", ctypes.c_int),
                ("max_batch", ctypes.c_int), ("device", ctypes.c_int), ("max_image_points", ctypes.c_int64),
                ("persistent_min", ctypes.c_int)]


class Request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("rows", ctypes.c_int), ("cols", ctypes.c_int), ("precision", ctypes.c_int),
                ("cutoff", ctypes.c_float), ("in_", ctypes.c_void_p), ("out", ctypes.c_void_p),
                ("wait_stream", ctypes.c_int), ("stream", ctypes.c_void_p)]


def serve_validate_config(hbm_budget_bytes: int, inflight: int = 4, max_batch: int = 8, device: int = 0,
                          max_image_points: int = 0, persistent_min: int = 0) -> int:
    cfg = ServerConfig(hbm_budget_bytes, inflight, max_batch, device, max_image_points, persistent_min)
    return lib().fft2_serve_validate_config(ctypes.byref(cfg))


class Server:
    """Serving loop (fft2_serve_*): submit requests, wait for tickets, read stats."""

    def __init__(self, hbm_budget_bytes: int = 64 << 30, inflight: int = 4, max_batch: int = 8, device: int = 0,
                 max_image_points: int = 0, persistent_min: int = 0):
        self.cfg = ServerConfig(hbm_budget_bytes, inflight, max_batch, device, max_image_points, persistent_min)
        h = ctypes.c_void_p()
        check(lib().fft2_serve_start(ctypes.byref(self.cfg), ctypes.byref(h)))
        self._h = h.value
        self._held = {}  # ticket -> the request's tensors, kept alive until wait()

    def alloc(self, nbytes: int) -> int:
        p = ctypes.c_void_p()
        check(lib().fft2_serve_alloc(self._h, nbytes, ctypes.byref(p)))
        return p.value

    def free(self, ptr: int) -> None:
        check(lib().fft2_serve_free(self._h, ptr))

    def submit(self, kind: int, x, out, precision: int = PREC_FP32, cutoff: float = 0.0, stream=None) -> int:
        """Queue a request on tensors.  It runs after the work already enqueued
        on `stream` (default: torch's current stream), and the tensors are kept
        alive until wait() returns for the ticket."""
        rows, cols = x.shape
        _check_tensor(x, rows, cols, "in")
        _check_tensor(out, rows, cols, "out")
        t = self.submit_ptr(kind, rows, cols, _ptr(x), _ptr(out), precision, cutoff, stream=_stream(stream))
        self._held[t] = (x, out)
        return t

    def submit_ptr(self, kind: int, rows: int, cols: int, pin: int, pout: int, precision: int = PREC_FP32,
                   cutoff: float = 0.0, stream: int | None = None) -> int:
        """Queue a request on raw device pointers; with `stream` (a hipStream_t
        handle, 0 = the null stream) it runs after the work enqueued there."""
        r = Request(kind, rows, cols, precision, float(cutoff), pin, pout, 0 if stream is None else 1, stream or 0)
        t = ctypes.c_uint64()
        check(lib().fft2_serve_submit(self._h, ctypes.byref(r), ctypes.byref(t)))
        return t.value

    def wait(self, ticket: int, timeout_s: float | None = None) -> int:
        st = ctypes.c_int()
        ns = -1 if timeout_s is None else int(timeout_s * 1e9)
        check(lib().fft2_serve_wait(self._h, ticket, ns, ctypes.byref(st)))
        self._held.pop(ticket, None)
        return st.value

    def stats(self) -> dict:
        p50, p99, rps = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        counts = (ctypes.c_int64 * 4)()
        check(lib().fft2_serve_stats(self._h, ctypes.byref(p50), ctypes.byref(p99), ctypes.byref(rps), counts))
        return {"p50_ms": p50.value, "p99_ms": p99.value, "req_per_s": rps.value, "submitted": counts[0],
                "completed": counts[1], "rejected": counts[2], "failed": counts[3]}

    def reset_stats(self) -> None:
        check(lib().fft2_serve_stats_reset(self._h))

    def stop(self) -> None:
        if getattr(self, "_h", None):
            h, self._h = self._h, None
            check(lib().fft2_serve_stop(h))

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.stop()

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass
