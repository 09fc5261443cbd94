"""GPU parity of the two-steps-per-pass sweep (temporal blocking) against
the CPU oracle, bit for bit: every value of the intermediate state is
evaluated with the single step's expression and rounding, so the result
must not depend on the number of steps per pass.  Covers the split form
(one and several slabs, slabs too thin for an Interior part), the fused
form, odd step counts (a last single pass), FP64, FP32 and bfloat16
storage, every built two-step tile shape, and the 512^3 FP64 headline
configuration in full.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2608_11882_amd import inputs

pytestmark = pytest.mark.gpu

TORCH = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}


def note(msg):
    print("[case] " + msg, flush=True)


@pytest.fixture
def two_steps(gpu):
    saved = gpu.get_time_block()
    gpu.set_time_block(2)
    yield gpu
    gpu.set_time_block(saved)


def start(dims, seed, dtype):
    nx, ny, nz = dims
    if dtype == "f64":
        return inputs.sine_field(nx, ny, nz, noise=0.05, seed=seed)
    return inputs.sine_field_lowp(nx, ny, nz, noise=0.05, seed=seed, dtype=dtype)


def reference(u0, r, steps, dtype):
    if dtype == "f64":
        return oracle.heat(u0, r, steps)
    if dtype == "f32":
        return oracle.heat_f32(u0, r, steps)
    return oracle.heat_bf16(u0, r, steps)


def run(hc, u0, r, steps, dtype, mode="split", parts=1):
    if dtype == "bf16":
        u = torch.from_numpy(u0.view(np.int16)).cuda().view(torch.bfloat16)
    else:
        u = torch.from_numpy(np.ascontiguousarray(u0)).cuda()
    un = torch.empty_like(u)
    hc.heat_step(u, un, r, steps, mode=mode, parts=parts)
    torch.cuda.synchronize()
    if dtype == "bf16":
        return u.view(torch.int16).cpu().numpy().view(np.uint16)
    return u.cpu().numpy()


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("dims", [(3, 3, 3), (6, 5, 4), (130, 9, 7), (67, 33, 41),
                                  (264, 19, 75), (1029, 6, 9), (64, 131, 36)])
@pytest.mark.parametrize("mode", ["split", "fused"])
def test_two_steps_per_pass_bitwise(two_steps, dtype, dims, mode):
    r = 0.15
    u0 = start(dims, sum(dims), dtype)
    for steps in (2, 3, 6):
        note("heat2 %s %s %s steps=%d" % (dtype, dims, mode, steps))
        want = reference(u0, r, steps, dtype)
        got = run(two_steps, u0, r, steps, dtype, mode=mode)
        assert np.array_equal(got, want), (dtype, dims, mode, steps)


@pytest.mark.parametrize("parts", [2, 3, 7, 16])
def test_split_into_slabs_bitwise(two_steps, parts):
    dims = (70, 20, 40)       # 16 slabs of 2-3 planes: Boundary kernel only
    note("heat2 split parts=%d %s" % (parts, dims))
    u0 = start(dims, 3, "f64")
    want = oracle.heat(u0, 0.12, 7)
    assert np.array_equal(run(two_steps, u0, 0.12, 7, "f64", parts=parts), want)


@pytest.mark.parametrize("dtype,parts,steps", [("f64", 1, 7), ("f64", 3, 6), ("f32", 2, 5),
                                               ("bf16", 1, 4)])
def test_caller_boundary_stream_bitwise(two_steps, dtype, parts, steps):
    """heat_step_streams: the Boundary kernels on a stream of the caller's
    (a second torch stream, or the Interior stream itself) give the oracle's
    bits, and the result is complete once the Interior stream's work is
    done (the run joins the two streams at every step, the last included)."""
    dims = (67, 33, 41)
    r = 0.14
    u0 = start(dims, 11 + parts, dtype)
    want = reference(u0, r, steps, dtype)
    side = torch.cuda.Stream()
    for which in ("second stream", "same stream"):
        note("heat_step_streams %s parts=%d steps=%d, %s" % (dtype, parts, steps, which))
        if dtype == "bf16":
            u = torch.from_numpy(u0.view(np.int16)).cuda().view(torch.bfloat16)
        else:
            u = torch.from_numpy(np.ascontiguousarray(u0)).cuda()
        un = torch.empty_like(u)
        main = torch.cuda.current_stream()
        bnd = side if which == "second stream" else main
        torch.cuda.synchronize()
        two_steps.heat_step(u, un, r, steps, parts=parts, stream=main, bnd_stream=bnd)
        main.synchronize()                 # only the Interior stream
        got = u.view(torch.int16).cpu().numpy().view(np.uint16) if dtype == "bf16" \
            else u.cpu().numpy()
        torch.cuda.synchronize()
        assert np.array_equal(got, want), (dtype, parts, steps, which)


def test_caller_boundary_stream_rejects_fused_mode(gpu):
    u = torch.zeros((8, 8, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        gpu.heat_step(u, torch.empty_like(u), 0.1, 2, mode="fused",
                      bnd_stream=torch.cuda.Stream())


def built_shapes(hc, dtype):
    lib = hc.load()
    code = hc.DTYPES[dtype]
    out = []
    for vec in (1, 2, 4, 8):
        for wx in (1, 2, 4):
            for by in (4, 8, 16):
                for zd in (16, 32, 64):
                    for pf in (1, 2, 3):
                        if lib.hc_heat2_set_tiling(code, vec, wx, by, zd, pf, 0) == 0:
                            out.append((vec, wx, by, zd, pf))
    hc.set_tiling2(dtype=dtype)
    return out


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_every_built_two_step_shape_bitwise(two_steps, dtype):
    hc = two_steps
    shapes = built_shapes(hc, dtype)
    assert len(shapes) >= 5
    dims = (264, 19, 75)      # ragged in x, y and z for every shape
    u0 = start(dims, 21, dtype)
    want = reference(u0, 0.14, 5, dtype)
    try:
        for shape in shapes:
            for xcd in (0, 8):
                for mode in ("split", "fused"):
                    note("heat2 %s shape %s xcd=%d %s" % (dtype, shape, xcd, mode))
                    hc.set_tiling2(*shape, xcd=xcd, dtype=dtype)
                    got = run(hc, u0, 0.14, 5, dtype, mode=mode)
                    assert np.array_equal(got, want), (shape, xcd, mode)
    finally:
        hc.set_tiling2(dtype=dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_run_lengths_bitwise(two_steps, dtype):
    """Blocks that march runs of several z-blocks (queues carried across,
    the first sub-block started early to end on the run's last plane), and
    whole columns, give the single steps' bits."""
    hc = two_steps
    dims = (130, 21, 150)     # 146 Interior planes: runs of every length end ragged
    u0 = start(dims, 31, dtype)
    want = reference(u0, 0.13, 6, dtype)
    try:
        for zrun in (1, 40, 64, 96, 1 << 20):
            for mode in ("split", "fused"):
                note("heat2 %s run of %d planes %s" % (dtype, zrun, mode))
                hc.set_zrun2(zrun, dtype=dtype)
                got = run(hc, u0, 0.13, 6, dtype, mode=mode)
                assert np.array_equal(got, want), (zrun, mode)
    finally:
        hc.set_zrun2(0, dtype=dtype)


def test_settings_and_fallback(two_steps):
    hc = two_steps
    assert hc.get_time_block() == 2
    with pytest.raises(hc.HeatCGError):
        hc.set_time_block(3)
    assert hc.get_time_block() == 2
    t = lambda *s: torch.zeros(*s, dtype=torch.float64, device="cuda")  # noqa: E731
    assert hc.tiling2_for(t(8, 8, 512))["vec"] == 2
    assert hc.tiling2_for(t(8, 8, 511))["vec"] == 1
    # stochastic rounding still takes single steps, with the same bits
    u0 = start((40, 12, 10), 4, "bf16")
    u = torch.from_numpy(u0.view(np.int16)).cuda().view(torch.bfloat16)
    hc.heat_step_sr(u, torch.empty_like(u), 0.1, 4, seed=7)
    torch.cuda.synchronize()
    want = oracle.heat_bf16_sr(u0, 0.1, 4, 7)
    assert np.array_equal(u.view(torch.int16).cpu().numpy().view(np.uint16), want)


@pytest.mark.parametrize("mode", ["split", "fused"])
def test_headline_configuration_full_size(two_steps, mode):
    cfg = inputs.HEAT_LARGE
    n, steps = cfg["n"], 5
    note("heat2 %d^3 FP64 %d steps %s (full size)" % (n, steps, mode))
    u0 = inputs.heat_large_f64(seed=cfg["seed"], n=n)
    want = oracle.heat(u0, cfg["r"], steps)
    assert np.array_equal(run(two_steps, u0, cfg["r"], steps, "f64", mode=mode), want)
