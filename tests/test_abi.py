"""The C-ABI library loads without a GPU, exports every function the header
declares, and its host-side validation rejects bad arguments before any
device work (these paths make no HIP call)."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "libjefi.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(jefi_[a-z0-9_]+)\s*\(", text)))


def test_header_and_exports_agree():
    import paper_2104_05426_amd as J
    out = subprocess.run(["nm", "-D", "--defined-only", J.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = sorted(set(re.findall(r"\bT (jefi_[a-z0-9_]+)", out)))
    declared = _declared()
    assert declared == exported
    assert sorted(J.EXPORTS) == declared
    for name in declared:
        assert hasattr(J.lib, name)


def test_version_and_defaults():
    import paper_2104_05426_amd as J
    assert "gfx950" in J.jefi_version()
    opt = J.jefi_options_default()
    assert opt.c == 1.0 and opt.screen_set == 0 and opt.precision == J.JEFI_PREC_F32_COMP


def test_history_bytes():
    import paper_2104_05426_amd as J
    from workloads import centred_grid
    g = centred_grid((5, 4, 3), 0.1)
    # bricks of 2x2x2: 3*2*2 = 12 bricks of 8 cells, 4 channels
    assert J.jefi_history_bytes(g, 7, J.JEFI_F32) == 7 * 12 * 8 * 4 * 4
    assert J.jefi_history_bytes(g, 7, J.JEFI_F64) == 7 * 12 * 8 * 4 * 8
    assert J.jefi_history_bytes(g, 0, J.JEFI_F32) == 0
    assert J.jefi_history_bytes(g, 3, 7) == 0


def _grid(n=(4, 4, 4), h=0.1):
    from workloads import centred_grid
    return centred_grid(n, h)


@pytest.mark.parametrize("case", [
    "null-src", "bad-spacing", "nt-zero", "nt-over-capacity", "nt-over-pushed", "t-after-newest",
    "dtype-mismatch", "bad-c", "negative-screen", "null-out", "bad-dt", "bad-flags", "both-flags",
    "slope-and-cubic", "hold-and-cut", "bad-tile", "bad-reserve",
])
def test_eval_validation(case):
    """Each bad input returns EINVAL with a message, before any device call."""
    import paper_2104_05426_amd as J
    src, obs = J.make_grid(_grid()), J.make_grid(_grid((3, 3, 3)))
    h = J.jefi_history(C.c_void_p(0x1000), J.JEFI_F32, 8, 7, 0.0)
    nt, dt, t = 8, 0.05, 7 * 0.05
    opt = J.jefi_options_default()
    fields = J.jefi_fields(C.c_void_p(0x2000), C.c_void_p(0x3000), J.JEFI_F32)
    src_p = C.byref(src)
    if case == "null-src":
        src_p = None
    elif case == "bad-spacing":
        src.spacing[1] = 0.0
    elif case == "nt-zero":
        nt = 0
    elif case == "nt-over-capacity":
        nt = 9
    elif case == "nt-over-pushed":
        h.newest = 3
    elif case == "t-after-newest":
        t = 7 * 0.05 + 0.01
    elif case == "dtype-mismatch":
        opt.precision = J.JEFI_PREC_F64
    elif case == "bad-c":
        opt.c = -1.0
    elif case == "negative-screen":
        opt.screen_set = 1
        opt.screen[2] = -0.1
    elif case == "null-out":
        fields.E = None
    elif case == "bad-dt":
        dt = 0.0
    elif case == "bad-flags":
        opt.flags = 64
    elif case == "hold-and-cut":
        opt.flags = J.JEFI_FLAG_PAST_HOLD | J.JEFI_FLAG_PAST_CUT
    elif case == "slope-and-cubic":
        opt.flags = J.JEFI_FLAG_DERIV_SLOPE | J.JEFI_FLAG_TIME_CUBIC
    elif case == "both-flags":
        opt.flags = J.JEFI_FLAG_INDEX_GUARD | J.JEFI_FLAG_INDEX_TABLE | J.JEFI_FLAG_PAST_HOLD
    elif case == "bad-tile":
        opt.tile_config = 4
    elif case == "bad-reserve":
        opt.reserve_cus = -1
    st = J.lib.jefi_eval_fields(src_p, C.byref(h), dt, nt, C.byref(obs), t, C.byref(fields),
                                C.byref(opt), None)
    assert st == J.JEFI_EINVAL
    assert len(J.jefi_last_error()) > 0


def test_time_exactly_at_newest_is_accepted_by_validation():
    """t = t0 + newest*dt passes the time check (rounding slack); with an
    empty observation grid the call then returns without device work."""
    import paper_2104_05426_amd as J
    from workloads import Grid
    src = J.make_grid(_grid())
    obs = J.make_grid(Grid((0, 0, 0), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0)))
    h = J.jefi_history(C.c_void_p(0x1000), J.JEFI_F32, 64, 63, 0.0)
    fields = J.jefi_fields(C.c_void_p(0x2000), C.c_void_p(0x3000), J.JEFI_F32)
    st = J.lib.jefi_eval_fields(C.byref(src), C.byref(h), 0.025, 64, C.byref(obs), 63 * 0.025,
                                C.byref(fields), None, None)
    assert st == J.JEFI_OK, J.jefi_last_error()


def test_push_validation():
    import paper_2104_05426_amd as J
    src = J.make_grid(_grid())
    h = J.jefi_history(None, J.JEFI_F32, 8, -1, 0.0)
    assert J.lib.jefi_history_push(C.byref(h), C.byref(src), C.c_void_p(0x10), None) == J.JEFI_EINVAL
    h.data = 0x1000
    assert J.lib.jefi_history_push(C.byref(h), C.byref(src), None, None) == J.JEFI_EINVAL
    assert h.newest == -1


def test_dump_validation():
    import paper_2104_05426_amd as J
    src, obs = J.make_grid(_grid()), J.make_grid(_grid())
    st = J.lib.jefi_slice_index_dump(C.byref(src), 0, 0.05, 7, 0.0, C.byref(obs), 0.3, None,
                                     C.c_void_p(0x10), None)
    assert st == J.JEFI_EINVAL


def test_coupler_validation():
    """Bad coupler arguments are rejected before any stream, event or
    allocation is made."""
    import paper_2104_05426_amd as J
    src, obs = J.make_grid(_grid()), J.make_grid(_grid())
    h = J.jefi_history(C.c_void_p(0x1000), J.JEFI_F32, 8, -1, 0.0)
    out = C.c_void_p()

    def create(**kw):
        a = dict(src=C.byref(src), hist=C.byref(h), dt=0.05, nt=4, obs=C.byref(obs), out_dtype=J.JEFI_F32,
                 out=C.byref(out))
        a.update(kw)
        return J.lib.jefi_coupler_create(a["src"], a["hist"], a["dt"], a["nt"], a["obs"], None, a["out_dtype"],
                                         a["out"])
    assert create(src=None) == J.JEFI_EINVAL
    assert create(out=None) == J.JEFI_EINVAL
    assert create(nt=0) == J.JEFI_EINVAL
    assert create(nt=9) == J.JEFI_EINVAL
    assert create(dt=0.0) == J.JEFI_EINVAL
    assert create(out_dtype=5) == J.JEFI_EINVAL
    bad = J.make_grid(_grid((0, 4, 4)))
    assert create(obs=C.byref(bad)) == J.JEFI_EINVAL
    h.dtype = 3
    assert create() == J.JEFI_EINVAL
    assert out.value is None
    st = C.c_int64(0)
    assert J.lib.jefi_coupler_step(None, C.c_void_p(0x10), 1, None, C.byref(st)) == J.JEFI_EINVAL
    assert J.lib.jefi_coupler_collect(None, 0, C.c_void_p(0x10), C.c_void_p(0x10)) == J.JEFI_EINVAL
    assert J.lib.jefi_coupler_destroy(None) == J.JEFI_EINVAL
