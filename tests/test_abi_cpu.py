"""The C ABI on the CPU: the library loads, exports every declared symbol,
and rejects bad arguments before touching the device (so these checks need
no GPU; the pointers below are never dereferenced)."""
import ctypes
import os
import re

import pytest

import paper_2608_11882_amd as hc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "heatcg.h")

HC_OK, HC_EINVAL, HC_EUNSTABLE, HC_EALIAS = 0, -1, -2, -3


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "sizeof")))


@pytest.fixture(scope="module")
def lib():
    return hc.load()


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ("heat_step", "heat_step_ex", "cg_solve", "cg_solve_ex", "hc_lap7_apply",
                     "hc_copy_probe", "hc_strerror", "hc_last_error_message"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), "libheatcg.so does not export " + name


def test_status_names(lib):
    assert hc.strerror(0) == "HC_OK"
    assert hc.strerror(-2) == "HC_EUNSTABLE"
    assert hc.strerror(12345) == "HC_UNKNOWN"


FAKE_U = ctypes.c_void_p(0x10000)
FAKE_V = ctypes.c_void_p(0x10000 + 8 * 10 ** 6)


@pytest.mark.parametrize("args,code", [
    ((None, FAKE_V, 10, 10, 10, 0.1, 1), HC_EINVAL),          # null pointer
    ((FAKE_U, FAKE_V, 2, 10, 10, 0.1, 1), HC_EINVAL),         # edge < 3
    ((FAKE_U, FAKE_V, 10, 10, 10, 0.2, 1), HC_EUNSTABLE),     # r > 1/6
    ((FAKE_U, FAKE_V, 10, 10, 10, -0.01, 1), HC_EUNSTABLE),   # r < 0
    ((FAKE_U, FAKE_V, 10, 10, 10, float("nan"), 1), HC_EUNSTABLE),
    ((FAKE_U, FAKE_V, 10, 10, 10, float("inf"), 1), HC_EUNSTABLE),
    ((FAKE_U, FAKE_V, 10, 10, 10, 0.1, -1), HC_EINVAL),       # negative steps
    ((FAKE_U, FAKE_U, 10, 10, 10, 0.1, 1), HC_EALIAS),        # same buffer
    ((FAKE_U, ctypes.c_void_p(0x10000 + 8 * 999), 10, 10, 10, 0.1, 1), HC_EALIAS),  # overlap
    ((FAKE_U, FAKE_V, 10, 10, 10, 0.1, 0), HC_OK),            # steps = 0: no-op
])
def test_heat_step_validation_happens_before_device_work(lib, args, code):
    assert lib.heat_step(*args) == code
    if code != HC_OK:
        assert lib.hc_last_error_message().decode() != ""


def test_heat_step_streams_validates_before_any_device_work(lib):
    """Arguments are checked before the library touches a device or a
    stream (these calls run without a GPU)."""
    f = lib.heat_step_streams
    s = ctypes.c_void_p(0)
    assert f(FAKE_U, FAKE_V, 10, 10, 10, 0.2, 4, 0, 1, s, s) == HC_EUNSTABLE
    assert f(FAKE_U, FAKE_V, 10, 10, 10, 0.1, 4, 0, 0, s, s) == HC_EINVAL    # parts < 1
    assert f(FAKE_U, FAKE_V, 10, 10, 10, 0.1, 4, 9, 1, s, s) == HC_EINVAL    # dtype
    assert f(FAKE_U, FAKE_U, 10, 10, 10, 0.1, 4, 0, 1, s, s) == HC_EALIAS
    assert f(FAKE_U, FAKE_V, 10, 10, 10, 0.1, 0, 0, 1, s, s) == 0            # nothing to do


def test_heat_step_ex_rejects_bad_mode_dtype_and_parts(lib):
    f = lib.heat_step_ex
    assert f(FAKE_U, FAKE_V, 10, 10, 10, 0.1, 1, 7, 0, 1, None) == HC_EINVAL      # dtype
    assert f(FAKE_U, FAKE_V, 10, 10, 10, 0.1, 1, 0, 9, 1, None) == HC_EINVAL      # mode
    assert f(FAKE_U, FAKE_V, 10, 10, 10, 0.1, 1, 0, 0, 0, None) == HC_EINVAL      # parts 0
    assert f(FAKE_U, FAKE_V, 10, 10, 10, 0.1, 1, 0, 0, 9, None) == HC_EINVAL      # > nz-2
    assert f(FAKE_U, FAKE_V, 10, 10, 10, 0.1, 1, 0, 1, 2, None) == HC_EINVAL      # parts w/o split
    assert f(FAKE_U, FAKE_V, 10, 10, 10, 1.0 / 6.0, 0, 0, 0, 8, None) == HC_OK    # r = 1/6 allowed


def test_cg_validation(lib):
    b, x = FAKE_U, FAKE_V
    assert lib.cg_solve(None, x, 8, 1e-10, 10) == HC_EINVAL
    assert lib.cg_solve(b, x, 0, 1e-10, 10) == HC_EINVAL
    assert lib.cg_solve(b, x, 8, 0.0, 10) == HC_EINVAL
    assert lib.cg_solve(b, x, 8, float("nan"), 10) == HC_EINVAL
    assert lib.cg_solve(b, x, 8, 1e-10, -1) == HC_EINVAL
    assert lib.cg_solve(b, b, 8, 1e-10, 10) == HC_EALIAS
    small = ctypes.c_size_t(16)
    assert lib.cg_solve_ex(b, x, 8, 8, 8, 1e-10, 10, FAKE_U, small, None, None, None) == HC_EINVAL


def test_cg_ir_validation(lib):
    b, x = FAKE_U, FAKE_V
    f = lib.cg_solve_ir
    out = (None, None, None)
    assert f(None, x, 8, 8, 8, 1e-10, 10, 0.0, None, 0, None, *out) == HC_EINVAL
    assert f(b, x, 0, 8, 8, 1e-10, 10, 0.0, None, 0, None, *out) == HC_EINVAL
    assert f(b, x, 8, 8, 8, 0.0, 10, 0.0, None, 0, None, *out) == HC_EINVAL
    assert f(b, x, 8, 8, 8, 1e-10, -1, 0.0, None, 0, None, *out) == HC_EINVAL
    assert f(b, x, 8, 8, 8, 1e-10, 10, 1.0, None, 0, None, *out) == HC_EINVAL     # inner_tol
    assert f(b, x, 8, 8, 8, 1e-10, 10, float("nan"), None, 0, None, *out) == HC_EINVAL
    assert f(b, b, 8, 8, 8, 1e-10, 10, 0.0, None, 0, None, *out) == HC_EALIAS
    assert f(b, x, 8, 8, 8, 1e-10, 10, 0.0, FAKE_U, 16, None, *out) == HC_EINVAL  # small work
    n = 64
    need = lib.cg_ir_workspace_bytes(n, n, n)
    assert 4 * 4 * n ** 3 <= need < lib.cg_workspace_bytes(n, n, n)
    assert lib.cg_ir_workspace_bytes(0, 4, 4) == 0
    assert lib.hc_lap7_apply_f32(FAKE_U, FAKE_U, 4, 4, 4, None) == HC_EALIAS
    assert lib.hc_lap7_apply_f32(None, FAKE_V, 4, 4, 4, None) == HC_EINVAL
    assert lib.hc_cg_ir_set_tiling(8, 1, 8, 16, 0) == HC_EINVAL     # 8-node float lanes
    assert lib.hc_cg_ir_set_tiling(4, 1, 8, 12, 0) == HC_EINVAL
    assert lib.hc_cg_ir_set_tiling(4, 1, 8, 16, 65) == HC_EINVAL
    assert lib.hc_cg_ir_set_tiling(2, 2, 8, 32, 3) == HC_OK
    assert hc.get_cg_ir_tiling() == dict(vec=2, wx=2, by=8, zdepth=32, xcd=3)
    hc.set_cg_ir_tiling()
    assert hc.get_cg_ir_tiling() == hc.DEFAULT_CG_IR_TILING


def test_workspace_size_formula(lib):
    n = 64
    need = lib.cg_workspace_bytes(n, n, n)
    assert need >= 3 * 8 * n ** 3
    assert lib.cg_workspace_bytes(0, 4, 4) == 0


def test_copy_probe_and_lap7_validation(lib):
    assert lib.hc_copy_probe(FAKE_U, FAKE_V, 17, None) == HC_EINVAL
    assert lib.hc_copy_probe(FAKE_U, FAKE_U, 16, None) == HC_EALIAS
    assert lib.hc_copy_probe(FAKE_U, FAKE_V, 0, None) == HC_OK
    assert lib.hc_lap7_apply(FAKE_U, FAKE_U, 4, 4, 4, None) == HC_EALIAS
    assert lib.hc_lap7_apply(FAKE_U, FAKE_V, 0, 4, 4, None) == HC_EINVAL


def test_tiling_knob(lib):
    assert lib.hc_heat_set_tiling(0, 2, 4, 2, 16, 2, 0) == HC_EINVAL   # ring needs more threads
    assert lib.hc_heat_set_tiling(0, 1, 1, 4, 48, 2, 0) == HC_EINVAL   # depth not built
    assert lib.hc_heat_set_tiling(0, 3, 1, 4, 16, 2, 0) == HC_EINVAL
    assert lib.hc_heat_set_tiling(0, 1, 1, 8, 16, 2, 65) == HC_EINVAL  # xcd run length
    assert lib.hc_heat_set_tiling(0, 4, 4, 4, 32, 2, 0) == HC_EINVAL   # 4-node lanes: FP32 only
    assert lib.hc_heat_set_tiling(1, 2, 4, 4, 16, 2, 0) == HC_EINVAL   # shape not built for FP32
    assert lib.hc_heat_set_tiling(3, 1, 4, 4, 16, 2, 0) == HC_EINVAL   # unknown dtype
    assert lib.hc_heat_get_tiling(3, None, None, None, None, None, None) == HC_EINVAL
    assert lib.hc_heat_set_tiling(0, 1, 4, 4, 32, 2, 1) == HC_OK
    assert hc.get_tiling() == dict(vec=1, wx=4, by=4, zdepth=32, pf=2, xcd=1)
    # the precisions keep separate shapes
    assert lib.hc_heat_set_tiling(1, 4, 2, 8, 16, 2, 3) == HC_OK
    assert hc.get_tiling("f32") == dict(vec=4, wx=2, by=8, zdepth=16, pf=2, xcd=3)
    assert hc.get_tiling("f64") == dict(vec=1, wx=4, by=4, zdepth=32, pf=2, xcd=1)
    assert lib.hc_heat_set_tiling(2, 8, 2, 4, 32, 2, 0) == HC_OK
    assert hc.get_tiling("bf16")["vec"] == 8
    for dt in ("f64", "f32", "bf16"):
        hc.set_tiling(dtype=dt)
        assert hc.get_tiling(dt) == hc.DEFAULT_TILING[dt] == hc.AUTO_TILING
        # the one-node fallback shape is built for every precision
        hc.set_tiling(1, 4, 4, 16, 2, 0, dtype=dt)
        hc.set_tiling(dtype=dt)


def tiling_for(lib, dtype, nx, u=None, un=None):
    v = [ctypes.c_int(0) for _ in range(6)]
    rc = lib.hc_heat_tiling_for(dtype, nx, u, un, *[ctypes.byref(x) for x in v])
    assert rc == HC_OK
    return tuple(x.value for x in v)


def test_automatic_tiling_choice(lib):
    """Every shape the automatic choice can return is built, tiles are never
    more than 1/8 wider than the narrowest candidate's, the widest fitting
    tile wins, and lanes of vec nodes need whole, aligned lanes."""
    for dt in (0, 1, 2, 3):
        for nx in list(range(3, 300)) + [510, 511, 512, 513, 600, 1000, 1023, 1024, 1030, 4096]:
            vec, wx, by, zd, pf, xcd = tiling_for(lib, dt, nx)
            sdt = min(dt, 2)   # the stochastic form takes bfloat16's shapes
            assert lib.hc_heat_set_tiling(sdt, vec, wx, by, zd, pf, xcd) == HC_OK, (dt, nx)
            assert nx % vec == 0 or vec == 1
        assert lib.hc_heat_set_tiling(min(dt, 2), 0, 0, 0, 0, 0, 0) == HC_OK
    assert tiling_for(lib, 0, 512) == (2, 4, 4, 32, 2, 8)
    assert tiling_for(lib, 1, 512) == (2, 4, 4, 32, 2, 8)
    assert tiling_for(lib, 1, 1024) == (4, 4, 4, 16, 2, 8)
    assert tiling_for(lib, 2, 1024) == (8, 1, 8, 16, 2, 8)
    assert tiling_for(lib, 2, 512) == (8, 1, 8, 16, 2, 8)
    assert tiling_for(lib, 3, 1024) == (8, 1, 4, 32, 2, 8)      # stochastic rounding
    # 1030 needs narrow tiles, which have two-node lanes; 1027 is odd
    assert tiling_for(lib, 1, 1030) == (2, 1, 8, 32, 2, 8)
    assert tiling_for(lib, 1, 1027)[0] == 1
    # misaligned arrays: one-node lanes
    off = lambda p, b: ctypes.c_void_p(p.value + b)  # noqa: E731
    assert tiling_for(lib, 0, 512, off(FAKE_U, 8), FAKE_V)[0] == 1
    assert tiling_for(lib, 2, 1024, FAKE_U, off(FAKE_V, 2))[0] == 1
    assert tiling_for(lib, 2, 1024, FAKE_U, FAKE_V)[0] == 8
    # an explicit setting wins over the automatic one
    assert lib.hc_heat_set_tiling(1, 4, 2, 8, 16, 2, 3) == HC_OK
    assert tiling_for(lib, 1, 1024) == (4, 2, 8, 16, 2, 3)
    hc.set_tiling(dtype="f32")
    v = [ctypes.c_int(0) for _ in range(6)]
    assert lib.hc_heat_tiling_for(5, 64, None, None, *[ctypes.byref(x) for x in v]) == HC_EINVAL
    assert lib.hc_heat_tiling_for(0, 2, None, None, *[ctypes.byref(x) for x in v]) == HC_EINVAL


def test_cg_tiling_knob(lib):
    assert lib.hc_cg_set_tiling(2, 4, 2, 16, 0) == HC_EINVAL
    assert lib.hc_cg_set_tiling(2, 2, 8, 12, 0) == HC_EINVAL
    assert lib.hc_cg_set_tiling(2, 2, 8, 16, 65) == HC_EINVAL
    assert lib.hc_cg_set_tiling(1, 1, 4, 32, 3) == HC_OK
    assert hc.get_cg_tiling() == dict(vec=1, wx=1, by=4, zdepth=32, xcd=3)
    hc.set_cg_tiling()
    assert hc.get_cg_tiling() == hc.DEFAULT_CG_TILING


def test_binding_raises_without_tensors():
    import torch
    with pytest.raises(ValueError):
        hc.heat_step(torch.zeros(4, 4, 4, dtype=torch.float64),
                     torch.zeros(4, 4, 4, dtype=torch.float64), 0.1, 1)


def test_batch_validation_happens_before_device_work(lib):
    import numpy as np
    h = ctypes.c_void_p(None)

    def create(dims, r, dtype=1, count=None):
        d = np.ascontiguousarray(np.asarray(dims, dtype=np.int32).reshape(-1, 3))
        rr = np.ascontiguousarray(np.asarray(r, dtype=np.float64))
        n = len(d) if count is None else count
        return lib.hc_batch_create(n, d.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                   rr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), dtype,
                                   ctypes.byref(h))
    assert create([[10, 10, 10], [2, 5, 5]], [0.1, 0.1]) == HC_EINVAL          # edge < 3
    assert create([[10, 10, 10]], [0.2]) == HC_EUNSTABLE
    assert create([[10, 10, 10]], [float("nan")]) == HC_EUNSTABLE
    assert create([[10, 10, 10]], [0.1], dtype=3) == HC_EINVAL                  # no SR batch
    assert create([[10, 10, 10]], [0.1], count=0) == HC_EINVAL
    assert lib.hc_batch_create(1, None, None, 1, ctypes.byref(h)) == HC_EINVAL
    assert lib.hc_batch_step(None, FAKE_U, FAKE_V, 1, 0, None) == HC_EINVAL
    assert lib.hc_batch_layout(None, None, None, None, None) == HC_EINVAL
    lib.hc_batch_destroy(None)                                                   # no-op


FAKE_K = ctypes.c_void_p(0x10000 + 16 * 10 ** 6)
FAKE_R = ctypes.c_void_p(0x10000 + 24 * 10 ** 6)


def test_heat_vk_step_validation_happens_before_device_work(lib):
    f = lib.heat_vk_step
    u, v, k, r = FAKE_U, FAKE_V, FAKE_K, FAKE_R
    ok = (10, 10, 10, 0.04, 1, 0, 0, 1, None)
    assert f(u, v, None, r, *ok) == HC_EINVAL
    assert f(u, v, k, None, *ok) == HC_EINVAL
    assert f(None, v, k, r, *ok) == HC_EINVAL
    assert f(u, v, k, r, 10, 10, 10, 0.04, 1, 2, 0, 1, None) == HC_EINVAL       # bfloat16
    assert f(u, v, k, r, 10, 10, 10, 0.04, 1, 3, 0, 1, None) == HC_EINVAL       # bfloat16 SR
    assert f(u, v, k, r, 10, 10, 10, -0.01, 1, 0, 0, 1, None) == HC_EUNSTABLE
    assert f(u, v, k, r, 10, 10, 10, float("nan"), 1, 0, 0, 1, None) == HC_EUNSTABLE
    assert f(u, v, k, r, 10, 10, 10, float("inf"), 1, 0, 0, 1, None) == HC_EUNSTABLE
    assert f(u, v, k, r, 2, 10, 10, 0.04, 1, 0, 0, 1, None) == HC_EINVAL        # edge < 3
    assert f(u, v, k, r, 10, 10, 10, 0.04, -1, 0, 0, 1, None) == HC_EINVAL      # steps
    assert f(u, v, k, r, 10, 10, 10, 0.04, 1, 0, 9, 1, None) == HC_EINVAL       # mode
    assert f(u, v, k, r, 10, 10, 10, 0.04, 1, 0, 1, 2, None) == HC_EINVAL       # parts w/o split
    assert f(u, u, k, r, *ok) == HC_EALIAS
    assert f(u, v, u, r, *ok) == HC_EALIAS                                       # kappa = u
    assert f(u, v, k, v, *ok) == HC_EALIAS                                       # rhs = u_new
    assert f(u, v, ctypes.c_void_p(0x10000 + 8 * 999), r, *ok) == HC_EALIAS      # kappa overlaps u
    assert f(u, v, k, k, 10, 10, 10, 0.04, 0, 0, 0, 1, None) == HC_OK            # steps 0; kappa = rhs
    assert f(u, v, k, r, 10, 10, 10, 0.04, 0, 1, 2, 1, None) == HC_OK            # f32, plain
    assert lib.hc_last_error_message().decode() == ""


def test_vk_tiling_settings_and_automatic_choice(lib):
    assert lib.hc_heat_vk_set_tiling(2, 1, 4, 4, 16, 2, 8) == HC_EINVAL     # bfloat16
    assert lib.hc_heat_vk_set_tiling(0, 8, 1, 8, 16, 2, 8) == HC_EINVAL     # not built
    assert lib.hc_heat_vk_set_tiling(0, 2, 2, 8, 16, 2, 65) == HC_EINVAL    # xcd
    assert lib.hc_heat_vk_set_tiling(0, 2, 1, 8, 16, 2, 3) == HC_OK
    assert hc.get_vk_tiling("f64") == dict(vec=2, wx=1, by=8, zdepth=16, pf=2, xcd=3)
    assert hc.get_vk_tiling("f32") == hc.AUTO_TILING
    hc.set_vk_tiling(dtype="f64")
    assert hc.get_vk_tiling("f64") == hc.AUTO_TILING

    def tiling_for(dtype, nx, ptrs):
        v = [ctypes.c_int(0) for _ in range(6)]
        assert lib.hc_heat_vk_tiling_for(dtype, nx, *ptrs, *[ctypes.byref(x) for x in v]) == HC_OK
        return tuple(x.value for x in v)

    aligned = [ctypes.c_void_p(0x100000 * (q + 1)) for q in range(4)]
    t = tiling_for(0, 512, aligned)
    assert t[0] == 2 and lib.hc_heat_vk_set_tiling(0, *t) == HC_OK      # a built shape
    hc.set_vk_tiling(dtype="f64")
    t = tiling_for(1, 512, aligned)
    assert t[0] == 1 and lib.hc_heat_vk_set_tiling(1, *t) == HC_OK      # one-node lanes
    hc.set_vk_tiling(dtype="f32")
    assert tiling_for(0, 513, aligned)[0] == 1                 # odd rows: one-node lanes
    odd = list(aligned)
    odd[3] = ctypes.c_void_p(0x100000 * 4 + 8)                 # rhs not 16-byte aligned
    assert tiling_for(0, 512, odd)[0] == 1
    assert lib.hc_heat_vk_tiling_for(2, 512, *aligned, *([None] * 6)) == HC_EINVAL


def test_time_block_and_two_step_tiling_settings(lib):
    assert lib.hc_heat_get_time_block() in (1, 2)
    saved = lib.hc_heat_get_time_block()
    assert lib.hc_heat_set_time_block(0) == HC_EINVAL
    assert lib.hc_heat_set_time_block(3) == HC_EINVAL
    assert lib.hc_heat_get_time_block() == saved
    assert lib.hc_heat_set_time_block(2) == HC_OK and hc.get_time_block() == 2
    assert lib.hc_heat_set_time_block(saved) == HC_OK
    assert lib.hc_heat2_set_tiling(3, 8, 1, 8, 16, 2, 8) == HC_EINVAL     # SR: single steps
    assert lib.hc_heat2_set_tiling(0, 8, 1, 8, 16, 2, 8) == HC_EINVAL     # not built
    assert lib.hc_heat2_set_tiling(0, 2, 2, 8, 16, 2, 65) == HC_EINVAL    # xcd
    assert lib.hc_heat2_set_tiling(0, 2, 1, 16, 16, 2, 4) == HC_OK
    assert hc.get_tiling2("f64") == dict(vec=2, wx=1, by=16, zdepth=16, pf=2, xcd=4)
    hc.set_tiling2(dtype="f64")
    assert hc.get_tiling2("f64") == hc.AUTO_TILING

    def tiling_for(dtype, nx, a, b):
        v = [ctypes.c_int(0) for _ in range(6)]
        assert lib.hc_heat2_tiling_for(dtype, nx, a, b, *[ctypes.byref(x) for x in v]) == HC_OK
        return tuple(x.value for x in v)

    a, b = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x200000)
    for dtype, vec in ((0, 2), (1, 4), (2, 4)):
        t = tiling_for(dtype, 512, a, b)
        assert t[0] == vec and lib.hc_heat2_set_tiling(dtype, *t) == HC_OK   # a built shape
        lib.hc_heat2_set_tiling(dtype, 0, 0, 0, 0, 0, 0)
    assert tiling_for(0, 511, a, b)[0] == 1
    assert tiling_for(0, 512, ctypes.c_void_p(0x100008), b)[0] == 1


def test_run_length_settings(lib):
    for setter, getter, dtypes in ((lib.hc_heat2_set_zrun, lib.hc_heat2_get_zrun, (0, 1, 2)),
                                   (lib.hc_heat_vk2_set_zrun, lib.hc_heat_vk2_get_zrun, (0, 1))):
        for dt in dtypes:
            assert getter(dt) == 0
            assert setter(dt, -1) == HC_EINVAL and setter(dt, (1 << 20) + 1) == HC_EINVAL
            assert setter(dt, 96) == HC_OK and getter(dt) == 96
            assert setter(dt, 0) == HC_OK and getter(dt) == 0
        assert setter(3, 64) == HC_EINVAL and getter(3) == HC_EINVAL
    assert lib.hc_heat_vk2_set_zrun(2, 64) == HC_EINVAL     # bfloat16: no variable kappa


def test_every_automatic_shape_is_a_built_shape(lib):
    """The automatic tile shape of every sweep, for widths that allow each
    lane width, is one the library is built with (a launch would refuse any
    other)."""
    a, b, c, d = (ctypes.c_void_p(0x100000 * (q + 1)) for q in range(4))
    v = [ctypes.c_int(0) for _ in range(6)]
    refs = [ctypes.byref(x) for x in v]
    for nx in (3, 7, 64, 130, 512, 1000, 1024):
        for dtype in (0, 1, 2):
            assert lib.hc_heat_tiling_for(dtype, nx, a, b, *refs) == HC_OK
            assert lib.hc_heat_set_tiling(dtype, *(x.value for x in v)) == HC_OK
            assert lib.hc_heat2_tiling_for(dtype, nx, a, b, *refs) == HC_OK
            assert lib.hc_heat2_set_tiling(dtype, *(x.value for x in v)) == HC_OK
        for dtype in (0, 1):
            assert lib.hc_heat_vk_tiling_for(dtype, nx, a, b, c, d, *refs) == HC_OK
            assert lib.hc_heat_vk_set_tiling(dtype, *(x.value for x in v)) == HC_OK
            assert lib.hc_heat_vk2_tiling_for(dtype, nx, a, b, c, d, *refs) == HC_OK
            assert lib.hc_heat_vk2_set_tiling(dtype, *(x.value for x in v)) == HC_OK
    for dtype in (0, 1, 2):
        for f in (lib.hc_heat_set_tiling, lib.hc_heat2_set_tiling):
            assert f(dtype, 0, 0, 0, 0, 0, 0) == HC_OK
    for dtype in (0, 1):
        for f in (lib.hc_heat_vk_set_tiling, lib.hc_heat_vk2_set_tiling):
            assert f(dtype, 0, 0, 0, 0, 0, 0) == HC_OK
