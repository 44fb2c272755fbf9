"""FP64 CPU oracle of the discretised Jefimenko sums -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the bench's CPU-baseline leg use this
package.  It wraps ``jefi_oracle.c`` (plain C, OpenMP over observation
points) through ctypes and shares nothing with the HIP library.  The
pure-Python second implementation lives in ``oracle.tiny``.

The arithmetic follows the paper's discretised equations for E, B and the
retarded time (section "GPU implementation of Jefimenko's equations"); the
readings of what the paper leaves open are listed in ``jefi_oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "jefi_oracle.c")
_DEFAULT_LIB = os.path.join(_HERE, "libjefi_oracle.so")
_LIB = _DEFAULT_LIB

SCREENED = -(2 ** 31)
STENCIL_SLOPE = 1  # time derivative = slope of the linear interpolant
STENCIL_HOLD = 2   # history before the oldest slice = the oldest slice
STENCIL_CUBIC = 4  # cubic through slices k-2 .. k+1 (not with STENCIL_SLOPE)
STENCIL_CUT = 8    # history starts at the oldest slice (not with STENCIL_HOLD)


class _Grid(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("origin", C.c_double * 3), ("spacing", C.c_double * 3)]


def build(force: bool = True, source: Optional[str] = None, target: Optional[str] = None) -> str:
    """Compile the oracle with contraction and fast-math off (``source`` and
    ``target`` default to the oracle's own files)."""
    if source is not None:
        tmp = target + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off",
                        "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-o", tmp, source, "-lm"],
                       check=True)
        os.replace(tmp, target)
        return target
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _use_library(path: Optional[str]):
    """Point the wrapper at another build of the oracle (None = the default
    one).  Used by the tests that plant mistakes in a copy of the oracle to
    show that the pins catch them."""
    global _lib, _LIB
    _lib = None
    _LIB = path or _DEFAULT_LIB


def _load():
    global _lib
    if _lib is None:
        stale = not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)
        if _LIB == _DEFAULT_LIB and stale:
            build(force=True)
        lib = C.CDLL(_LIB)
        P = C.POINTER
        lib.orc_eval.argtypes = [P(_Grid), P(_Grid), P(C.c_double), C.c_int32, C.c_double, C.c_double,
                                 C.c_double, C.c_double, C.c_int64, P(C.c_double), P(C.c_int64),
                                 C.c_int64, P(C.c_double), P(C.c_double), C.c_int32, C.c_int32]
        lib.orc_eval.restype = C.c_int
        lib.orc_slice_index_dump.argtypes = [P(_Grid), P(_Grid), C.c_int32, C.c_double, C.c_double,
                                             C.c_double, C.c_double, C.c_int64, P(C.c_double),
                                             P(C.c_int32)]
        lib.orc_slice_index_dump.restype = C.c_int
        lib.orc_slice_fingerprint.argtypes = [P(_Grid), P(_Grid), C.c_int32, C.c_double, C.c_double,
                                              C.c_double, C.c_double, C.c_int64, P(C.c_double),
                                              P(C.c_int64), C.c_int64, P(C.c_int64)]
        lib.orc_slice_fingerprint.restype = C.c_int
        lib.orc_max_threads.restype = C.c_int
        _lib = lib
    return _lib


def _grid(g) -> _Grid:
    out = _Grid()
    for a in range(3):
        out.n[a] = int(g.n[a])
        out.origin[a] = float(g.origin[a])
        out.spacing[a] = float(g.spacing[a])
    return out


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def max_threads() -> int:
    return int(_load().orc_max_threads())


def _delta(src, screen):
    if screen is None:
        return tuple(0.5 * s for s in src.spacing)
    return tuple(float(v) for v in screen)


def eval_fields(src, obs, hist: np.ndarray, dt: float, t: float, t0: float = 0.0,
                newest: Optional[int] = None, c: float = 1.0,
                screen: Optional[Sequence[float]] = None, sel: Optional[Sequence[int]] = None,
                threads: int = 0, stencil: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """E, B (FP64 [3][n_out]) at time t from ``hist[nt][4][n_src]``
    (oldest slice first; ``newest`` = absolute step of the last slice,
    default nt-1).  ``screen`` = half-widths (default half the source
    spacing); ``sel`` = observation linear indices (default all).
    ``stencil``: reading of the time stencil, bit 0 = derivative as the
    slope of the interpolant (``STENCIL_SLOPE``), bit 1 = history before
    the oldest slice held at its values (``STENCIL_HOLD``), bit 2 = cubic
    time interpolation through slices k-2 .. k+1 (``STENCIL_CUBIC``, not
    with bit 0), bit 3 = the history starts at the oldest slice: earlier
    retarded times contribute nothing and no derivative is taken across the
    start (``STENCIL_CUT``, not with bit 1); 0 = the interpolated backward
    difference and a zero past."""
    lib = _load()
    h = np.ascontiguousarray(hist, dtype=np.float64)
    nt = int(h.shape[0])
    if h.ndim != 3 or h.shape[1] != 4 or h.shape[2] != src.size:
        raise ValueError("history must be [nt][4][n_src]")
    if newest is None:
        newest = nt - 1
    delta = (C.c_double * 3)(*_delta(src, screen))
    if sel is not None:
        sel_a = np.ascontiguousarray(np.asarray(sel, dtype=np.int64))
        nout = int(sel_a.shape[0])
        sel_p = sel_a.ctypes.data_as(C.POINTER(C.c_int64))
    else:
        sel_a = None
        nout = obs.size
        sel_p = None
    E = np.zeros((3, nout), dtype=np.float64)
    B = np.zeros((3, nout), dtype=np.float64)
    gs, go = _grid(src), _grid(obs)
    rc = lib.orc_eval(C.byref(gs), C.byref(go), _dptr(h), nt, float(dt), float(c), float(t),
                      float(t0), int(newest), delta, sel_p, nout, _dptr(E), _dptr(B), int(threads),
                      int(stencil))
    if rc != 0:
        raise ValueError(f"oracle rejected the problem (code {rc})")
    return E, B


def eval_problem(p, sel=None, threads: int = 0, stencil: int = 0):
    """``eval_fields`` for a ``workloads.Problem``."""
    return eval_fields(p.src, p.obs, p.hist, p.dt, p.t, p.t0, p.newest, p.c, p.screen, sel, threads,
                       stencil)


def slice_index_dump(src, obs, nt: int, dt: float, t: float, t0: float = 0.0,
                     newest: Optional[int] = None, c: float = 1.0,
                     screen: Optional[Sequence[float]] = None) -> np.ndarray:
    """int32 [n_obs][n_src]: SCREENED, -2 (stencil before the oldest slice) or k."""
    lib = _load()
    if newest is None:
        newest = nt - 1
    out = np.zeros((obs.size, src.size), dtype=np.int32)
    delta = (C.c_double * 3)(*_delta(src, screen))
    gs, go = _grid(src), _grid(obs)
    rc = lib.orc_slice_index_dump(C.byref(gs), C.byref(go), int(nt), float(dt), float(c), float(t),
                                  float(t0), int(newest), delta,
                                  out.ctypes.data_as(C.POINTER(C.c_int32)))
    if rc != 0:
        raise ValueError(f"oracle rejected the problem (code {rc})")
    return out


def slice_fingerprint(src, obs, nt: int, dt: float, t: float, t0: float = 0.0,
                      newest: Optional[int] = None, c: float = 1.0,
                      screen: Optional[Sequence[float]] = None,
                      sel: Optional[Sequence[int]] = None) -> np.ndarray:
    """int64 [n_out][4]: (live pairs, sum k, sum k*(s+1) mod 2^64, screened)."""
    lib = _load()
    if newest is None:
        newest = nt - 1
    delta = (C.c_double * 3)(*_delta(src, screen))
    if sel is not None:
        sel_a = np.ascontiguousarray(np.asarray(sel, dtype=np.int64))
        nout = int(sel_a.shape[0])
        sel_p = sel_a.ctypes.data_as(C.POINTER(C.c_int64))
    else:
        nout = obs.size
        sel_p = None
    fp = np.zeros((nout, 4), dtype=np.int64)
    gs, go = _grid(src), _grid(obs)
    rc = lib.orc_slice_fingerprint(C.byref(gs), C.byref(go), int(nt), float(dt), float(c), float(t),
                                   float(t0), int(newest), delta, sel_p, nout,
                                   fp.ctypes.data_as(C.POINTER(C.c_int64)))
    if rc != 0:
        raise ValueError(f"oracle rejected the problem (code {rc})")
    return fp
