"""Pins of the oracle's per-point slice fingerprint (``orc_slice_fingerprint``).

The fingerprint summarises the slice decisions of the discrete retarded-time
equation (section "GPU implementation of Jefimenko's equations", the
discretised t_r) per observation point: the number of pairs that are neither
screened nor wholly before the oldest slice, the sum of their slice index k,
the sum of k*(s+1) modulo 2^64 (s = linear source index) and the number of
screened pairs.  It is the reference for every bit-exact slice-index claim
on problems too large for per-pair dumps, so it is pinned here against
things other than itself:

  * hand-computed fingerprints of configurations whose separations and times
    are exact binary fractions (every k follows from integer arithmetic);
  * the same four numbers rebuilt in plain Python from the per-pair decisions
    of the independent pure-Python oracle (``oracle.tiny``), on random small
    problems that hold screened pairs, pairs at k = -1, pairs wholly before
    the oldest slice (k < -1), negative k whose weighted sums wrap modulo
    2^64, and subsets of observation points.
"""
import numpy as np
import pytest

import oracle
from oracle import tiny
from workloads import Grid

MASK64 = (1 << 64) - 1


def _signed64(v):
    v &= MASK64
    return v - (1 << 64) if v >= (1 << 63) else v


def _fingerprint_from_codes(codes):
    """(live, sum k, sum k*(s+1) mod 2^64, screened) per row of per-pair
    codes: SCREENED, -2 (wholly before the oldest slice) or k >= -1."""
    rows = []
    for row in codes:
        live = sk = skw = scr = 0
        for s, code in enumerate(row):
            code = int(code)
            if code == tiny.SCREENED:
                scr += 1
            elif code >= -1:
                live += 1
                sk += code
                skw += code * (s + 1)
        rows.append([live, sk, _signed64(skw), scr])
    return np.array(rows, dtype=np.int64)


def test_hand_computed_fingerprints():
    """Two source cells on the x axis (x = -0.5, 0), points at x = 0 .. 2 in
    steps of 0.5, dt = 0.25, c = 1: R/(c dt) is an even integer, so with t on
    a slice every k is a_i minus that integer."""
    src = Grid((2, 1, 1), (-0.5, 0.0, 0.0), (0.5, 0.5, 0.5))
    obs = Grid((5, 1, 1), (0.0, 0.0, 0.0), (0.5, 0.5, 0.5))
    nt, dt = 9, 0.25
    # t = 2.0: a = 8.  Point x = 0 sits on cell s = 1 (R = 0: screened even
    # with zero screening width) and is 2 slices from s = 0.
    fp = oracle.slice_fingerprint(src, obs, nt, dt, t=2.0, screen=(0, 0, 0))
    expect = [
        [1, 6, 6 * 1, 1],                # s=0: R 0.5 -> k 6; s=1 screened
        [2, 4 + 6, 4 * 1 + 6 * 2, 0],    # R 1.0, 0.5 -> k 4, 6
        [2, 2 + 4, 2 * 1 + 4 * 2, 0],    # R 1.5, 1.0 -> k 2, 4
        [2, 0 + 2, 0 * 1 + 2 * 2, 0],    # R 2.0, 1.5 -> k 0, 2
        [1, 0, 0 * 2, 0],                # R 2.5 -> k -2 (wholly before the oldest slice), R 2.0 -> k 0
    ]
    assert fp.tolist() == expect
    # t = 1.25: a = 5.  k = 5 - 2R/0.5: R 1.5 gives k = -1 (live, f = 0),
    # R 2.0 and beyond give k <= -3 (dead).
    fp = oracle.slice_fingerprint(src, obs, nt, dt, t=1.25, screen=(0, 0, 0))
    expect = [
        [1, 3, 3 * 1, 1],
        [2, 1 + 3, 1 * 1 + 3 * 2, 0],
        [2, -1 + 1, -1 * 1 + 1 * 2, 0],
        [1, -1, _signed64(-1 * 2), 0],   # s=0 at R 2.0: k = -3, dead
        [0, 0, 0, 0],
    ]
    assert fp.tolist() == expect
    # a selection of points, in any order, gives the same rows
    fp_sel = oracle.slice_fingerprint(src, obs, nt, dt, t=1.25, screen=(0, 0, 0), sel=[3, 0, 3])
    assert fp_sel.tolist() == [expect[3], expect[0], expect[3]]


def test_hand_computed_fingerprint_off_slice_and_screening_cube():
    """t between slices (a = 5.2), and a screening cube whose half-width is
    one spacing: it screens the 3x3x3 block of cells around a point."""
    src = Grid((3, 1, 1), (-0.5, 0.0, 0.0), (0.5, 0.5, 0.5))
    obs = Grid((1, 1, 1), (0.0, 0.0, 0.0), (0.5, 0.5, 0.5))
    nt, dt = 9, 0.25
    # a = 5.2: u = 0.2 - 2R/0.5 ... floor gives k = 5 + floor(0.2 - 4R)
    fp = oracle.slice_fingerprint(src, obs, nt, dt, t=1.3, screen=(0, 0, 0))
    # s = 0 at R 0.5 -> floor(-1.8) = -2 -> k 3; s = 1 at R 0 -> screened;
    # s = 2 at R 0.5 -> k 3
    assert fp.tolist() == [[2, 6, 3 * 1 + 3 * 3, 1]]
    fp = oracle.slice_fingerprint(src, obs, nt, dt, t=1.3, screen=(0.5, 0.5, 0.5))
    assert fp.tolist() == [[0, 0, 0, 3]]
    # 5x5x5 cells of spacing 0.5 around the point, cube half-width 0.5:
    # 27 screened, the other 98 all live (the history is long enough)
    src = Grid((5, 5, 5), (-1.0, -1.0, -1.0), (0.5, 0.5, 0.5))
    fp = oracle.slice_fingerprint(src, obs, 40, dt, t=39 * dt, screen=(0.5, 0.5, 0.5))
    assert fp[0, 0] == 125 - 27 and fp[0, 3] == 27


def _random_problem(rng):
    sp = tuple(rng.uniform(0.07, 0.13, 3))
    n_src = tuple(int(v) for v in rng.integers(2, 5, 3))
    n_obs = tuple(int(v) for v in rng.integers(2, 4, 3))
    so = tuple(rng.uniform(-0.2, 0.0, 3))
    src = Grid(n_src, so, sp)
    # observation points among the source cells (screened pairs)
    obs = Grid(n_obs, tuple(o + rng.uniform(-0.5, 1.0) * h for o, h in zip(so, sp)),
               tuple(rng.uniform(0.05, 0.12, 3)))
    nt = int(rng.integers(5, 9))
    dt = float(rng.uniform(0.05, 0.09))
    c = float(rng.uniform(0.8, 1.25))
    s_old = int(rng.integers(-3, 20))
    newest = s_old + nt - 1
    t0 = float(rng.uniform(-0.3, 0.3))
    # evaluation time near the start of the window: far pairs lie wholly
    # before the oldest slice, near ones at k = -1 and above
    a = float(rng.uniform(1.5, 3.5))
    t = t0 + (s_old + a) * dt
    screen = tuple(rng.uniform(0.5, 1.2) * h for h in sp)
    return src, obs, nt, dt, t, t0, newest, c, screen


def _problem_with_every_category(rng):
    """Draws until the problem holds screened pairs, pairs wholly before the
    oldest slice, pairs at k = -1 and pairs at k >= 0."""
    while True:
        prob = _random_problem(rng)
        src, obs, nt, dt, t, t0, newest, c, screen = prob
        codes = tiny.slice_index_dump(src, obs, nt, dt, t, t0, newest, c, screen)
        flat = np.array(codes).ravel()
        if (flat == tiny.SCREENED).any() and (flat == -2).any() and (flat == -1).any() and (flat >= 0).any():
            return prob, codes


@pytest.mark.parametrize("seed", range(10))
def test_fingerprint_equals_the_pure_python_pair_decisions(seed):
    rng = np.random.default_rng(900 + seed)
    (src, obs, nt, dt, t, t0, newest, c, screen), codes = _problem_with_every_category(rng)
    expect = _fingerprint_from_codes(codes)
    fp = oracle.slice_fingerprint(src, obs, nt, dt, t, t0, newest, c, screen)
    assert np.array_equal(fp, expect)
    # the C oracle's own per-pair dump reduces to the same rows
    assert np.array_equal(_fingerprint_from_codes(oracle.slice_index_dump(src, obs, nt, dt, t, t0, newest, c, screen)),
                          expect)
    # a subset of points, repeated and out of order
    sel = list(rng.integers(0, obs.size, 5))
    fp_sel = oracle.slice_fingerprint(src, obs, nt, dt, t, t0, newest, c, screen, sel=sel)
    assert np.array_equal(fp_sel, expect[sel])


def test_negative_indices_wrap_the_weighted_sum():
    """k = -1 pairs contribute -(s+1) modulo 2^64 to the weighted sum."""
    src = Grid((4, 1, 1), (0.0, 0.0, 0.0), (0.5, 0.5, 0.5))
    obs = Grid((1, 1, 1), (-0.5, 0.0, 0.0), (0.5, 0.5, 0.5))
    nt, dt = 3, 0.25
    # a = 2 (t = newest): R = 0.5, 1.0, 1.5, 2.0 -> k = 0, -2, -4, -6
    fp = oracle.slice_fingerprint(src, obs, nt, dt, t=(nt - 1) * dt, screen=(0, 0, 0))
    assert fp.tolist() == [[1, 0, 0, 0]]
    src = Grid((4, 1, 1), (0.0, 0.0, 0.0), (0.125, 0.5, 0.5))
    obs = Grid((1, 1, 1), (-0.125, 0.0, 0.0), (0.5, 0.5, 0.5))
    # R = 0.125 .. 0.5 -> R/(c dt) = 0.5 .. 2; a = 2: u = -0.5, -1, -1.5, -2
    # -> k = 1, 1, 0, 0: all live.  At a = 1 (t one slice earlier): k = 0,
    # 0, -1, -1, so the weighted sum is 0 + 0 - 3 - 4 (mod 2^64).
    fp = oracle.slice_fingerprint(src, obs, nt, dt, t=(nt - 2) * dt, screen=(0, 0, 0))
    assert fp.tolist() == [[4, -2, _signed64(-3 - 4), 0]]
