"""Python binding of libjefi (ctypes; argument marshalling only).

Every computation runs in the HIP library ``libjefi.so`` built from
``csrc/``; this module only converts grids, torch device tensors and streams
to the C ABI declared in ``include/libjefi.h`` and raises ``JefiError`` on a
failed status.  Importing it without a built library raises immediately:
there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libjefi.so")

JEFI_OK, JEFI_PENDING = 0, 1
JEFI_EINVAL, JEFI_ENOMEM, JEFI_EDEVICE, JEFI_EBUSY, JEFI_ENOENT, JEFI_ETOOLARGE = -1, -2, -3, -4, -5, -6
JEFI_F32, JEFI_F64 = 0, 1
JEFI_PREC_F64, JEFI_PREC_F32_COMP = 0, 1
JEFI_FLAG_INDEX_GUARD, JEFI_FLAG_INDEX_TABLE = 1, 2
JEFI_FLAG_DERIV_SLOPE, JEFI_FLAG_PAST_HOLD, JEFI_FLAG_TIME_CUBIC, JEFI_FLAG_PAST_CUT = 4, 8, 16, 32
INT32_MIN = -(2 ** 31)

STATUS_NAMES = {0: "OK", 1: "PENDING", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EBUSY",
                -5: "ENOENT", -6: "ETOOLARGE"}

# Every function the header declares (the CPU tests check the exports).
EXPORTS = [
    "jefi_version", "jefi_last_error", "jefi_options_default", "jefi_history_bytes",
    "jefi_history_init", "jefi_history_push", "jefi_eval_fields", "jefi_eval_fields_noalloc",
    "jefi_slice_index_dump",
    "jefi_slice_fingerprint", "jefi_eval_batch", "jefi_autotune",
    "jefi_server_create", "jefi_server_open_session", "jefi_server_submit", "jefi_server_poll",
    "jefi_server_wait", "jefi_server_close_session", "jefi_server_get_stats", "jefi_server_destroy",
    "jefi_coupler_create", "jefi_coupler_step", "jefi_coupler_collect", "jefi_coupler_destroy",
]


class JefiError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class jefi_grid(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("origin", C.c_double * 3), ("spacing", C.c_double * 3)]


class jefi_history(C.Structure):
    _fields_ = [("data", C.c_void_p), ("dtype", C.c_int32), ("capacity", C.c_int32),
                ("newest", C.c_int64), ("t0", C.c_double)]


class jefi_fields(C.Structure):
    _fields_ = [("E", C.c_void_p), ("B", C.c_void_p), ("dtype", C.c_int32)]


class jefi_options(C.Structure):
    _fields_ = [("c", C.c_double), ("screen", C.c_double * 3), ("screen_set", C.c_int32),
                ("precision", C.c_int32), ("flags", C.c_uint32), ("tile_config", C.c_int32),
                ("reserve_cus", C.c_int32)]


class jefi_problem(C.Structure):
    _fields_ = [("src", jefi_grid), ("hist", jefi_history), ("dt", C.c_double), ("nt", C.c_int32),
                ("obs", jefi_grid), ("t", C.c_double), ("out", jefi_fields)]


class jefi_server_config(C.Structure):
    _fields_ = [("arena", C.c_void_p), ("arena_bytes", C.c_uint64), ("pinned_bytes", C.c_uint64),
                ("precision", C.c_int32), ("max_inflight", C.c_int32), ("max_batch", C.c_int32),
                ("max_queue", C.c_int32), ("flags", C.c_uint32), ("reserve_cus", C.c_int32),
                ("express_cus", C.c_int32), ("express_pairs", C.c_uint64)]


class jefi_request(C.Structure):
    _fields_ = [("session", C.c_uint64), ("new_slice", C.c_void_p), ("obs", jefi_grid), ("t", C.c_double),
                ("E", C.c_void_p), ("B", C.c_void_p), ("out_dtype", C.c_int32), ("out_on_host", C.c_int32)]


class jefi_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("batch_size", C.c_int32), ("t_submit_ns", C.c_uint64),
                ("t_admit_ns", C.c_uint64), ("t_start_ns", C.c_uint64), ("t_done_ns", C.c_uint64),
                ("pairs", C.c_uint64)]


class jefi_server_stats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in ("submitted", "completed", "failed", "batches", "max_batch",
                                         "evictions", "rematerialisations", "arena_bytes", "arena_used",
                                         "arena_high_water", "pairs", "express_batches", "express_cus",
                                         "cu_masked")]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build() or "
                          f"python {os.path.join(_HERE, 'build.py')}")
    lib = C.CDLL(LIB_PATH)
    P = C.POINTER
    vp = C.c_void_p
    sig = {
        "jefi_version": ([], C.c_char_p),
        "jefi_last_error": ([], C.c_char_p),
        "jefi_options_default": ([P(jefi_options)], None),
        "jefi_history_bytes": ([P(jefi_grid), C.c_int32, C.c_int32], C.c_uint64),
        "jefi_history_init": ([P(jefi_history), vp, C.c_uint64, P(jefi_grid), C.c_int32, C.c_int32,
                               C.c_double, vp], C.c_int),
        "jefi_history_push": ([P(jefi_history), P(jefi_grid), vp, vp], C.c_int),
        "jefi_eval_fields": ([P(jefi_grid), P(jefi_history), C.c_double, C.c_int32, P(jefi_grid),
                              C.c_double, P(jefi_fields), P(jefi_options), vp], C.c_int),
        "jefi_eval_fields_noalloc": ([P(jefi_grid), P(jefi_history), C.c_double, C.c_int32, P(jefi_grid),
                                      C.c_double, P(jefi_fields), P(jefi_options), vp], C.c_int),
        "jefi_slice_index_dump": ([P(jefi_grid), C.c_int32, C.c_double, C.c_int64, C.c_double,
                                   P(jefi_grid), C.c_double, P(jefi_options), vp, vp], C.c_int),
        "jefi_slice_fingerprint": ([P(jefi_grid), P(jefi_history), C.c_double, C.c_int32,
                                    P(jefi_grid), C.c_double, P(jefi_options), vp, vp], C.c_int),
        "jefi_eval_batch": ([P(jefi_problem), C.c_int32, P(jefi_options), vp], C.c_int),
        "jefi_autotune": ([P(jefi_problem), C.c_int32, P(jefi_options), C.c_int32, vp,
                           P(C.c_int32), P(C.c_double)], C.c_int),
        "jefi_server_create": ([P(jefi_server_config), P(vp)], C.c_int),
        "jefi_server_open_session": ([vp, C.c_uint64, P(jefi_grid), C.c_int32, C.c_int32, C.c_double,
                                      C.c_double, vp, C.c_int32], C.c_int),
        "jefi_server_submit": ([vp, P(jefi_request), P(C.c_uint64)], C.c_int),
        "jefi_server_poll": ([vp, C.c_uint64, P(jefi_result)], C.c_int),
        "jefi_server_wait": ([vp, C.c_uint64, P(jefi_result)], C.c_int),
        "jefi_server_close_session": ([vp, C.c_uint64], C.c_int),
        "jefi_server_get_stats": ([vp, P(jefi_server_stats)], C.c_int),
        "jefi_server_destroy": ([vp], C.c_int),
        "jefi_coupler_create": ([P(jefi_grid), P(jefi_history), C.c_double, C.c_int32, P(jefi_grid),
                                 P(jefi_options), C.c_int32, P(vp)], C.c_int),
        "jefi_coupler_step": ([vp, vp, C.c_int32, vp, P(C.c_int64)], C.c_int),
        "jefi_coupler_collect": ([vp, C.c_int64, vp, vp], C.c_int),
        "jefi_coupler_destroy": ([vp], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


lib = _load()


def _check(st: int):
    if st != JEFI_OK:
        raise JefiError(st, lib.jefi_last_error().decode())


def make_grid(g) -> jefi_grid:
    """A jefi_grid from anything with ``n``, ``origin`` and ``spacing``."""
    out = jefi_grid()
    for a in range(3):
        out.n[a] = int(g.n[a])
        out.origin[a] = float(g.origin[a])
        out.spacing[a] = float(g.spacing[a])
    return out


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    import torch
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return t.data_ptr()


def jefi_version() -> str:
    return lib.jefi_version().decode()


def jefi_last_error() -> str:
    return lib.jefi_last_error().decode()


def jefi_options_default(precision: Optional[int] = None, c: Optional[float] = None,
                         screen: Optional[Sequence[float]] = None) -> jefi_options:
    opt = jefi_options()
    lib.jefi_options_default(C.byref(opt))
    if precision is not None:
        opt.precision = int(precision)
    if c is not None:
        opt.c = float(c)
    if screen is not None:
        opt.screen_set = 1
        for a in range(3):
            opt.screen[a] = float(screen[a])
    return opt


def jefi_history_bytes(src, capacity: int, dtype: int) -> int:
    return int(lib.jefi_history_bytes(C.byref(make_grid(src)), int(capacity), int(dtype)))


def jefi_history_init(data, src, capacity: int, dtype: int, t0: float = 0.0,
                      stream=None) -> jefi_history:
    """``data``: a contiguous device tensor of at least jefi_history_bytes() bytes
    (the caller keeps it alive as long as the history is used)."""
    h = jefi_history()
    nbytes = data.numel() * data.element_size()
    _check(lib.jefi_history_init(C.byref(h), _ptr(data), nbytes, C.byref(make_grid(src)),
                                 int(capacity), int(dtype), float(t0), _stream_ptr(stream)))
    return h


def jefi_history_push(h: jefi_history, src, slice_, stream=None) -> None:
    """``slice_``: device tensor [4][n_src] of the history dtype."""
    _check(lib.jefi_history_push(C.byref(h), C.byref(make_grid(src)), _ptr(slice_),
                                 _stream_ptr(stream)))


def jefi_eval_fields(src, h: jefi_history, dt: float, nt: int, obs, t: float, E, B,
                     opt: Optional[jefi_options] = None, stream=None) -> None:
    """E, B: device tensors [3][n_obs] (float32 or float64)."""
    import torch
    dt_out = JEFI_F64 if E.dtype == torch.float64 else JEFI_F32
    if B.dtype != E.dtype:
        raise ValueError("E and B must share a dtype")
    f = jefi_fields(_ptr(E), _ptr(B), dt_out)
    _check(lib.jefi_eval_fields(C.byref(make_grid(src)), C.byref(h), float(dt), int(nt),
                                C.byref(make_grid(obs)), float(t), C.byref(f),
                                C.byref(opt) if opt is not None else None, _stream_ptr(stream)))


def jefi_eval_fields_noalloc(src, h: jefi_history, dt: float, nt: int, obs, t: float, E, B,
                             opt: Optional[jefi_options] = None, stream=None) -> None:
    """As jefi_eval_fields, with the library's fixed device scratch: no
    device memory is allocated.  Calls that overlap on one GPU race."""
    import torch
    dt_out = JEFI_F64 if E.dtype == torch.float64 else JEFI_F32
    if B.dtype != E.dtype:
        raise ValueError("E and B must share a dtype")
    f = jefi_fields(_ptr(E), _ptr(B), dt_out)
    _check(lib.jefi_eval_fields_noalloc(C.byref(make_grid(src)), C.byref(h), float(dt), int(nt),
                                        C.byref(make_grid(obs)), float(t), C.byref(f),
                                        C.byref(opt) if opt is not None else None, _stream_ptr(stream)))


def jefi_slice_index_dump(src, nt: int, dt: float, newest: int, t0: float, obs, t: float, out,
                          opt: Optional[jefi_options] = None, stream=None) -> None:
    """out: device int32 tensor [n_obs][n_src]."""
    _check(lib.jefi_slice_index_dump(C.byref(make_grid(src)), int(nt), float(dt), int(newest),
                                     float(t0), C.byref(make_grid(obs)), float(t),
                                     C.byref(opt) if opt is not None else None, _ptr(out),
                                     _stream_ptr(stream)))


def jefi_slice_fingerprint(src, h: jefi_history, dt: float, nt: int, obs, t: float, fp,
                           opt: Optional[jefi_options] = None, stream=None) -> None:
    """fp: device int64 tensor [n_obs][4]."""
    _check(lib.jefi_slice_fingerprint(C.byref(make_grid(src)), C.byref(h), float(dt), int(nt),
                                      C.byref(make_grid(obs)), float(t),
                                      C.byref(opt) if opt is not None else None, _ptr(fp),
                                      _stream_ptr(stream)))


def make_problem(src, h: jefi_history, dt: float, nt: int, obs, t: float, E, B) -> jefi_problem:
    """A jefi_problem for one batch entry (E, B: device tensors [3][n_obs])."""
    import torch
    dt_out = JEFI_F64 if E.dtype == torch.float64 else JEFI_F32
    return jefi_problem(make_grid(src), h, float(dt), int(nt), make_grid(obs), float(t),
                        jefi_fields(_ptr(E), _ptr(B), dt_out))


def jefi_eval_batch(problems, opt: Optional[jefi_options] = None, stream=None) -> None:
    """problems: a sequence of jefi_problem (see make_problem)."""
    arr = (jefi_problem * len(problems))(*problems)
    _check(lib.jefi_eval_batch(arr, len(problems), C.byref(opt) if opt is not None else None,
                               _stream_ptr(stream)))


def jefi_autotune(problems, opt: Optional[jefi_options] = None, reps: int = 3, stream=None):
    """Tune the launch configuration on `problems` (one: a single launch,
    several: a batch); returns (packed configuration, ms per run): tile
    | index mode << 2 | granularity << 4."""
    arr = (jefi_problem * len(problems))(*problems)
    best = C.c_int32(0)
    ms = C.c_double(0.0)
    _check(lib.jefi_autotune(arr, len(problems), C.byref(opt) if opt is not None else None,
                             int(reps), _stream_ptr(stream), C.byref(best), C.byref(ms)))
    return int(best.value), float(ms.value)


def upload_history(src, hist_np, dtype: int, t0: float = 0.0, newest: Optional[int] = None,
                   capacity: Optional[int] = None, device: str = "cuda", stream=None):
    """Push the slices ``hist_np[nt][4][n_src]`` (oldest first) into a fresh
    ring; returns (storage tensor, jefi_history).  When ``newest`` is given
    the first slice becomes step newest - nt + 1."""
    import torch
    nt = int(hist_np.shape[0])
    capacity = int(capacity or nt)
    nbytes = jefi_history_bytes(src, capacity, dtype)
    store = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=device)
    h = jefi_history_init(store, src, capacity, dtype, t0, stream)
    if newest is not None:
        h.newest = int(newest) - nt
    tdt = torch.float64 if dtype == JEFI_F64 else torch.float32
    for j in range(nt):
        sl = torch.as_tensor(hist_np[j], dtype=tdt).to(device).contiguous()
        jefi_history_push(h, src, sl, stream)
    return store, h


class Server:
    """Thin owner of a jefi_server handle (the C calls do all the work).
    ``arena``: a device tensor whose bytes the server may use."""

    def __init__(self, arena, precision=JEFI_PREC_F32_COMP, max_inflight=2, max_batch=256,
                 max_queue=65536, pinned_bytes=0, flags=0, reserve_cus=0, express_pairs=0, express_cus=0):
        self.arena = arena
        cfg = jefi_server_config(_ptr(arena), arena.numel() * arena.element_size(), int(pinned_bytes),
                                 int(precision), int(max_inflight), int(max_batch), int(max_queue),
                                 int(flags), int(reserve_cus), int(express_cus), int(express_pairs))
        h = C.c_void_p()
        _check(lib.jefi_server_create(C.byref(cfg), C.byref(h)))
        self.h = h
        self.precision = precision

    def open_session(self, session, src, capacity, window, t0, dt, init_history=None):
        """init_history: numpy [init_nt][4][n_src] in the server's precision (or None)."""
        import numpy as np
        ptr, nt = None, 0
        if init_history is not None:
            arr = np.ascontiguousarray(init_history,
                                       dtype=np.float64 if self.precision == JEFI_PREC_F64 else np.float32)
            ptr, nt = arr.ctypes.data, int(arr.shape[0])
        _check(lib.jefi_server_open_session(self.h, int(session), C.byref(make_grid(src)), int(capacity),
                                            int(window), float(t0), float(dt), ptr, nt))

    def submit(self, session, obs, E, B, new_slice=None, t=float("nan"), out_on_host=True):
        """E, B: numpy arrays [3][n_obs] (out_on_host) or device tensors;
        new_slice: numpy [4][n_src] in the server's precision or None.
        Returns (status, ticket); the caller keeps E/B alive until done."""
        import numpy as np
        if out_on_host:
            eptr, bptr = E.ctypes.data, B.ctypes.data
            odt = JEFI_F64 if E.dtype == np.float64 else JEFI_F32
        else:
            import torch
            eptr, bptr = _ptr(E), _ptr(B)
            odt = JEFI_F64 if E.dtype == torch.float64 else JEFI_F32
        sl = None
        if new_slice is not None:
            sl = np.ascontiguousarray(new_slice,
                                      dtype=np.float64 if self.precision == JEFI_PREC_F64 else np.float32)
        rq = jefi_request(int(session), sl.ctypes.data if sl is not None else None, make_grid(obs), float(t),
                          eptr, bptr, odt, 1 if out_on_host else 0)
        tk = C.c_uint64(0)
        st = lib.jefi_server_submit(self.h, C.byref(rq), C.byref(tk))
        return st, int(tk.value)

    def poll(self, ticket):
        res = jefi_result()
        st = lib.jefi_server_poll(self.h, int(ticket), C.byref(res))
        return st, res

    def wait(self, ticket):
        res = jefi_result()
        st = lib.jefi_server_wait(self.h, int(ticket), C.byref(res))
        return st, res

    def close_session(self, session):
        return lib.jefi_server_close_session(self.h, int(session))

    def stats(self):
        out = jefi_server_stats()
        _check(lib.jefi_server_get_stats(self.h, C.byref(out)))
        return {n: int(getattr(out, n)) for n, _ in jefi_server_stats._fields_}

    def destroy(self):
        if self.h is not None:
            st = lib.jefi_server_destroy(self.h)
            self.h = None
            return st
        return JEFI_OK


class Coupler:
    """Thin owner of a jefi_coupler handle (the C calls do all the work):
    per-step push + evaluation with the slice and field copies overlapped."""

    def __init__(self, src, h: jefi_history, dt: float, nt: int, obs, opt: Optional[jefi_options] = None,
                 out_dtype: int = JEFI_F32):
        self.hist = h  # the coupler pushes into this structure
        self.src = make_grid(src)
        self.obs = make_grid(obs)
        hnd = C.c_void_p()
        _check(lib.jefi_coupler_create(C.byref(self.src), C.byref(h), float(dt), int(nt), C.byref(self.obs),
                                       C.byref(opt) if opt is not None else None, int(out_dtype),
                                       C.byref(hnd)))
        self.h = hnd

    def step(self, slice_, stream=None):
        """slice_: numpy [4][n_src] (host) or a device tensor made on `stream`
        (default: torch's current stream); returns the step."""
        import numpy as np
        st = C.c_int64(0)
        if isinstance(slice_, np.ndarray):
            arr = np.ascontiguousarray(slice_)
            _check(lib.jefi_coupler_step(self.h, arr.ctypes.data, 1, None, C.byref(st)))
        else:
            _check(lib.jefi_coupler_step(self.h, _ptr(slice_), 0, _stream_ptr(stream), C.byref(st)))
        return int(st.value)

    def collect(self, step, E, B):
        """E, B: numpy arrays [3][n_obs] of the coupler's output dtype."""
        _check(lib.jefi_coupler_collect(self.h, int(step), E.ctypes.data, B.ctypes.data))

    def destroy(self):
        if self.h is not None:
            st = lib.jefi_coupler_destroy(self.h)
            self.h = None
            return st
        return JEFI_OK
