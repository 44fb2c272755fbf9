"""A second, independent pure-Python oracle for tiny problems.

TEST INFRASTRUCTURE ONLY (used by tests to check the C oracle).  It follows
the paper's discretised sums (section "GPU implementation of Jefimenko's
equations": the discrete E, B and retarded-time equations) literally, with
Python floats (IEEE FP64, no contraction) and ``math.fsum`` for every sum, so
it shares neither code nor summation scheme with the C oracle.  The same
readings apply: linear interpolation in time between slices, backward
differences interpolated the same way, zero history before the oldest slice,
the slice index from the FP64 split a = a_i + a_f, and the cube screening.
The alternative time-stencil readings (derivative as the slope of the
interpolant; history before the oldest slice held at its values; cubic time
interpolation through slices k-2 .. k+1; a history that starts at the oldest
slice, so that earlier retarded times contribute nothing and no derivative is
taken across the start) are selected by the same ``stencil`` bits as the C
oracle.  The cubic is written here in Newton's
forward-difference form, the C oracle uses Lagrange weights.

Cost is O(n_obs * n_src * 4) Python operations: keep n_obs * n_src <= ~3e5.
"""
from __future__ import annotations

import math
from typing import Sequence, Tuple

SCREENED = -(2 ** 31)


def _centre(g, lin):
    nx, ny, _ = g.n
    i = lin % nx
    j = (lin // nx) % ny
    k = lin // (nx * ny)
    return (g.origin[0] + float(i) * g.spacing[0],
            g.origin[1] + float(j) * g.spacing[1],
            g.origin[2] + float(k) * g.spacing[2])


def time_split(t, t0, dt, newest, nt, c):
    """(a_i, a_f, inv_cdt) for evaluation time t; raises when t is after
    the newest slice by more than rounding."""
    s_old = newest - nt + 1
    a = (t - t0) / dt - float(s_old)
    top = float(nt - 1)
    if not a <= top:
        if a - top <= 1e-9 * (1.0 + abs(a) + abs(float(s_old))):
            a = top
        else:
            raise ValueError("evaluation time after the newest slice")
    ai = math.floor(a)
    return int(ai), a - float(ai), 1.0 / (c * dt)


def slice_decision(ro, rs, delta, ai, af, inv_cdt):
    """None for a screened pair, else (d, R, k, f)."""
    d = (ro[0] - rs[0], ro[1] - rs[1], ro[2] - rs[2])
    if abs(d[0]) <= delta[0] and abs(d[1]) <= delta[1] and abs(d[2]) <= delta[2]:
        return None
    R = math.sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2])
    if R == 0.0:
        return None
    u = af - R * inv_cdt
    m = math.floor(u)
    return d, R, ai + int(m), u - float(m)


def eval_fields(src, obs, hist, dt, t, t0, newest, c=1.0, delta=(0.0, 0.0, 0.0),
                sel: Sequence[int] | None = None, stencil: int = 0):
    """E, B as lists [3][n_out] of floats.  ``hist[j][ch][s]`` with j = 0
    the oldest of nt slices.  ``stencil`` bit 0: slope derivative; bit 1:
    held past; bit 2: cubic; bit 3: history starting at the oldest slice."""
    slope = bool(stencil & 1)
    cubic = bool(stencil & 4)
    cut = bool(stencil & 8)
    if slope and cubic:
        raise ValueError("the slope and cubic readings exclude each other")
    if cut and stencil & 2:
        raise ValueError("a held past and a history starting at the oldest slice exclude each other")
    hold = bool(stencil & 2) or cut  # stencils reaching before the start read the oldest slice
    nt = len(hist)
    ai, af, inv_cdt = time_split(t, t0, dt, newest, nt, c)
    ns = src.n[0] * src.n[1] * src.n[2]
    no = obs.n[0] * obs.n[1] * obs.n[2]
    idx = list(range(no)) if sel is None else list(sel)
    vol = src.spacing[0] * src.spacing[1] * src.spacing[2]
    scale = vol / (4.0 * math.pi)
    E = [[0.0] * len(idx) for _ in range(3)]
    B = [[0.0] * len(idx) for _ in range(3)]

    def H(j, ch, s):
        if j < 0:
            return float(hist[0][ch][s]) if hold else 0.0
        return float(hist[j][ch][s])

    for q, o in enumerate(idx):
        ro = _centre(obs, o)
        terms = [[] for _ in range(6)]
        for s in range(ns):
            rs = _centre(src, s)
            dec = slice_decision(ro, rs, delta, ai, af, inv_cdt)
            if dec is None:
                continue
            d, R, k, f = dec
            if cut and k < 0:
                continue  # retarded time before the start of the history
            if k < -1 and not hold:
                continue
            # value and backward difference at the retarded time, both as
            # linear interpolations between slices k and k+1
            val = []
            der = []
            if cubic:
                if k + 1 > nt - 1:
                    raise ValueError("stencil reaches past the newest slice")
                for ch in range(4):
                    # Newton form on nodes -2, -1, 0, 1 with x = f + 2 steps from
                    # the first node: p = y0 + x D1 + x(x-1) D2/2 + x(x-1)(x-2) D3/6
                    y = [H(k - 2 + i, ch, s) for i in range(4)]
                    d1 = y[1] - y[0]
                    d2 = y[2] - 2.0 * y[1] + y[0]
                    d3 = y[3] - 3.0 * y[2] + 3.0 * y[1] - y[0]
                    x = f + 2.0
                    val.append(math.fsum([y[0], x * d1, x * (x - 1.0) * d2 / 2.0,
                                          x * (x - 1.0) * (x - 2.0) * d3 / 6.0]))
                    dp = math.fsum([d1, (2.0 * x - 1.0) * d2 / 2.0,
                                    (3.0 * x * x - 6.0 * x + 2.0) * d3 / 6.0])
                    der.append(dp / dt)
            for ch in range(4 if not cubic else 0):
                lo = H(k, ch, s)
                dlo = (lo - H(k - 1, ch, s)) / dt
                if f != 0.0:
                    if k + 1 > nt - 1:
                        raise ValueError("stencil reaches past the newest slice")
                    hi = H(k + 1, ch, s)
                    dhi = (hi - lo) / dt
                    val.append(math.fsum([(1.0 - f) * lo, f * hi]))
                    der.append(math.fsum([(1.0 - f) * dlo, f * dhi]))
                else:
                    val.append(lo)
                    der.append(dlo)
                if slope:
                    # derivative of the piecewise-linear interpolant on [k, k+1]
                    if k + 1 > nt - 1:
                        raise ValueError("stencil reaches past the newest slice")
                    der[-1] = (H(k + 1, ch, s) - lo) / dt
            rho, rhod = val[0], der[0]
            J, Jd = val[1:], der[1:]
            for a in range(3):
                terms[a].append(d[a] * rho / R ** 3)
                terms[a].append(d[a] * rhod / R ** 2)
                terms[a].append(-Jd[a] / R)
            crossJ = (d[1] * J[2] - d[2] * J[1], d[2] * J[0] - d[0] * J[2], d[0] * J[1] - d[1] * J[0])
            crossD = (d[1] * Jd[2] - d[2] * Jd[1], d[2] * Jd[0] - d[0] * Jd[2], d[0] * Jd[1] - d[1] * Jd[0])
            for a in range(3):
                terms[3 + a].append(-crossJ[a] / R ** 3)
                terms[3 + a].append(-crossD[a] / R ** 2)
        for a in range(3):
            E[a][q] = math.fsum(terms[a]) * scale
            B[a][q] = math.fsum(terms[3 + a]) * scale
    return E, B


def slice_index_dump(src, obs, nt, dt, t, t0, newest, c=1.0, delta=(0.0, 0.0, 0.0)):
    """Per-pair codes [n_obs][n_src]: SCREENED, -2 (stencil wholly before
    the oldest slice) or the slice index k."""
    ai, af, inv_cdt = time_split(t, t0, dt, newest, nt, c)
    ns = src.n[0] * src.n[1] * src.n[2]
    no = obs.n[0] * obs.n[1] * obs.n[2]
    out = []
    for o in range(no):
        ro = _centre(obs, o)
        row = []
        for s in range(ns):
            dec = slice_decision(ro, _centre(src, s), delta, ai, af, inv_cdt)
            if dec is None:
                row.append(SCREENED)
            else:
                k = dec[2]
                row.append(-2 if k < -1 else k)
        out.append(row)
    return out
